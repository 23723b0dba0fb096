// Last layer of the FP32 form, sender side (paths (l, l, 0), 64 or 128
// channels): the same formulation as the BF16 form's kernels in k_fast.hip,
// with every contraction on the FP32 MFMA (16x16x4, one k-slot per lane
// group) and every operand and stored value in FP32.
//
// Rows j are walked and every edge e' = (j <- i) of row j stands for its
// reverse e = (i <- j), whose sender is the row's own atom (same length,
// unit vector -u, Y_l(-u) = (-1)^l Y_l(u)), so the sender features h~_j are
// staged once per row in a wave-private LDS slice instead of gathered per
// edge.
//   messages: m_e[c] = sum_l R_e[l, c] X_e[l, c],  X_e[l, c] = sum_m YC_e[lm] h~_j[lm, c]
//             written to the receiver-side slot rev(e') of the message array;
//   sum:      A_i = sum over row i's slots / n_avg;
//   adjoint:  dR = dA_i X / n_avg (MLP adjoint), dE/dYC = h~_j (R dA_i) / n_avg
//             and the pull h~bar_j = sum_e YC_e (R dA_i) / n_avg, with the
//             radial MLP evaluated once per edge for all of them.
//
// Weights sit in LDS once per workgroup, row-major with an odd row stride so
// that both the forward (W^T as the A operand) and the adjoint (W as the A
// operand) read them without bank conflicts from one copy:
//   W1 [8][65], W2 [64][65] (rows the input feature), W3 [64][P C + 1]
//   (rows hidden, columns path-major channels of the live paths).
// D tiles of a 16x16x4 product: row 4 g + r, column lane % 16; the A operand
// of lane (g, l16) is A[l16][g], the B operand B[g][l16].
#include "edge_common.h"

namespace mpip {

namespace {

__device__ __forceinline__ bool guard32(const FastArgs& a) {
  return (int64_t)a.row_ptr[a.n] > a.capacity || a.status[ST_FLAGS] != 0;
}

template <int L>
struct CgD {
  float c[(L + 1) * (L + 1)];
};
template <int L>
__device__ __forceinline__ CgD<L> cg_diag32(const float* cg) {
  CgD<L> d;
  int off = 0;
#pragma unroll
  for (int l = 0; l <= L; ++l) {
    const int n = 2 * l + 1;
#pragma unroll
    for (int m = 0; m < n; ++m)
      d.c[l * l + m] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(cg[off + m * n + m])));
    off += n * n;
  }
  return d;
}

template <int NF>
__device__ __forceinline__ void stage32(float* dst, const float* src) {
  for (int t = threadIdx.x; t < NF; t += blockDim.x) dst[t] = src[t];
}

// the X operands of this lane's edge: YC[4 q + g] masked to degree l
template <int L>
struct YOps {
  float y[L + 1][3];
};
template <int L>
__device__ __forceinline__ YOps<L> x_ops(const float* yc, int g) {
  YOps<L> o;
  o.y[0][0] = g == 0 ? yc[0] : 0.f;
  float y1 = 0.f;   // selects rather than an indexed read, so yc stays in registers
  y1 = g == 1 ? yc[1] : y1;
  y1 = g == 2 ? yc[2] : y1;
  y1 = g == 3 ? yc[3] : y1;
  o.y[1][0] = y1;
  if constexpr (L == 2) {
    float y4 = yc[4];
    y4 = g == 1 ? yc[5] : y4;
    y4 = g == 2 ? yc[6] : y4;
    y4 = g == 3 ? yc[7] : y4;
    o.y[2][1] = y4;
    o.y[2][2] = g == 0 ? yc[8] : 0.f;
  }
  return o;
}

// X_l tile (channels 16 t + 4 g + r) x (edge lane % 16) from the staged row
// features sh [NLMP][C] (rows past NLM zero)
template <int C, int L, int l>
__device__ __forceinline__ f32x4 x_tile(const float* sh, int t, int g, int el, const YOps<L>& yo) {
  f32x4 x = {0.f, 0.f, 0.f, 0.f};
  if constexpr (l < 2) {
    x = mfma_f32(sh[g * C + 16 * t + el], yo.y[l][0], x);
  } else {
    x = mfma_f32(sh[(4 + g) * C + 16 * t + el], yo.y[2][1], x);
    x = mfma_f32(sh[(8 + g) * C + 16 * t + el], yo.y[2][2], x);
  }
  return x;
}

}  // namespace

template <int C, int L>
struct L2F32 {
  static constexpr int NLM = (L + 1) * (L + 1), P = L + 1, NLMP = (NLM + 3) / 4 * 4, NT = C / 16;
  static constexpr int WS = P * C + 1;                      // W3 row stride (odd)
  static constexpr int NW3 = 64 * WS, NW2 = 64 * 65, NW1 = 8 * 65;
};

// staged row features: rows 0..NLM-1 of h~_j, rows NLM..NLMP-1 zero
template <int C, int L>
__device__ __forceinline__ void stage_row32(float* sh, const float* hj, int lane) {
  typedef L2F32<C, L> D;
  constexpr int N4 = D::NLMP * C / 4;
#pragma unroll
  for (int p0 = 0; p0 < N4; p0 += 64) {
    const int p = p0 + lane;
    if (p < N4) {
      const int row = (4 * p) / C;
      ((float4*)sh)[p] = row < D::NLM ? *(const float4*)(hj + 4 * p) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

// Messages (FP32): m_e written to the receiver-side slot rev(e').
template <int C, int L, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(1))) void k_l2_msg32(FastArgs a) {
  typedef L2F32<C, L> D;
  constexpr int NLM = D::NLM, NT = D::NT, WS = D::WS;
  __shared__ float sW3[D::NW3], sW2[D::NW2], sW1[D::NW1];
  __shared__ __align__(16) float sH[NW][D::NLMP * C];
  if (guard32(a)) return;
  const GeoK gk = geo_consts(a.rc, a.envelope_p);
  const CgD<L> cgd = cg_diag32<L>(a.cg);
  stage32<D::NW3>(sW3, a.w3r);
  stage32<D::NW2>(sW2, a.w2r);
  stage32<D::NW1>(sW1, a.w1r);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, el = lane & 15, wv = threadIdx.x >> 6;
  float* sh = sH[wv];
  const float* ht = (const float*)a.ht;
  float* M = (float*)a.msg;
  const RowWalk rw = row_walk<NW>(a.n);
  for (int64_t j = rw.i; j < rw.end; j += rw.step) {
    const int e0 = a.row_ptr[j], e1 = a.row_end ? a.row_end[j] : a.row_ptr[j + 1];
    stage_row32<C, L>(sh, ht + j * NLM * C, lane);
    wave_lds_sync();
    for (int t0 = e0; t0 < e1; t0 += kTileE) {
      const int e = t0 + el;
      const bool valid = e < e1;
      const int rv = valid ? a.e_rev[e] : -1;
      Geo geo;
      const float4 v = valid ? a.e_vec[e] : make_float4(-1.f, 0.f, 0.f, 0.f);
      edge_geometry(make_float4(-v.x, -v.y, -v.z, 0.f), valid, gk, geo);
      float yc[NLM];
#pragma unroll
      for (int k = 0; k < NLM; ++k) yc[k] = cgd.c[k] * geo.Y[k];
      const YOps<L> yo = x_ops<L>(yc, g);
      f32x4 p1[4], a1[4], p2[4], a2[4];
      mlp_fwd_rows(geo, lane, sW1, sW2, p1, a1, p2);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) a2[mt][r] = silu(p2[mt][r]);
      float* dst = M + (int64_t)(rv < 0 ? 0 : rv) * C + 4 * g;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        f32x4 m = {0.f, 0.f, 0.f, 0.f};
        static_for<L + 1>([&](auto lc) {
          constexpr int l = decltype(lc)::value;
          f32x4 R = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kc = 0; kc < 16; ++kc) R = mfma_f32(sW3[phi_f(kc, g) * WS + l * C + 16 * t + el], a2[kc / 4][kc % 4], R);
          const f32x4 X = x_tile<C, L, l>(sh, t, g, el, yo);
#pragma unroll
          for (int r = 0; r < 4; ++r) m[r] += R[r] * X[r];
        });
        if (rv >= 0) *(float4*)(dst + 16 * t) = make_float4(m[0], m[1], m[2], m[3]);
      }
    }
    wave_lds_sync();
  }
}

// A_i[c] = sum_{e in row i} M[e][c] / n_avg: one wave per row, C/4 lanes per
// edge (4 channels each)
template <int C>
__global__ __launch_bounds__(256) void k_l2_msum32(FastArgs a) {
  constexpr int LPE = C / 4, EPI = 64 / LPE;
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (guard32(a) || i >= a.n) return;
  const int lane = threadIdx.x & 63, s = lane / LPE, c4 = lane % LPE;
  const int e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
  const float* M = (const float*)a.msg + 4 * c4;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  int e = e0 + s;
  for (; e + 3 * EPI < e1; e += 4 * EPI) {
    float4 u[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) u[b] = *(const float4*)(M + (int64_t)(e + b * EPI) * C);
#pragma unroll
    for (int b = 0; b < 4; ++b) { acc.x += u[b].x; acc.y += u[b].y; acc.z += u[b].z; acc.w += u[b].w; }
  }
  for (; e < e1; e += EPI) {
    const float4 u = *(const float4*)(M + (int64_t)e * C);
    acc.x += u.x; acc.y += u.y; acc.z += u.z; acc.w += u.w;
  }
#pragma unroll
  for (int o = LPE; o < 64; o <<= 1) {
    acc.x += __shfl_xor(acc.x, o);
    acc.y += __shfl_xor(acc.y, o);
    acc.z += __shfl_xor(acc.z, o);
    acc.w += __shfl_xor(acc.w, o);
  }
  if (s == 0)
    *(float4*)(a.A + i * C + 4 * c4) = make_float4(a.inv_n * acc.x, a.inv_n * acc.y, a.inv_n * acc.z, a.inv_n * acc.w);
}

// Fused adjoint (FP32).  Per tile: the radial MLP forward; per channel tile t
// and path l: R and X (channels x edges), dR = dA X and RA = dA R; the MLP
// adjoint's input ab2 += W3 dR (A = W3 rows hidden); dE/dYC_l += h~ RA
// (A = the row's features, rows lm); the pull h~bar += YC RA^T, with RA
// moved to edges x channels through a wave-private LDS tile.  Then the MLP
// backward, and dE/dr of the reverse edge to g2p[e'] (or added to g[rev]).
template <int C, int L, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(1))) void k_l2_adj32(FastArgs a) {
  typedef L2F32<C, L> D;
  constexpr int NLM = D::NLM, NT = D::NT, WS = D::WS;
  constexpr int TS = 20;   // row stride of the transposition tile (16-byte rows)
  constexpr int SY = 17;   // row stride of the per-edge YC table
  __shared__ float sW3[D::NW3], sW2[D::NW2], sW1[D::NW1];
  __shared__ __align__(16) float sH[NW][D::NLMP * C];
  __shared__ __align__(16) float sT[NW][2][16 * TS];
  __shared__ float sY[NW][16 * SY];
  if (guard32(a)) return;
  const GeoK gk = geo_consts(a.rc, a.envelope_p);
  const CgD<L> cgd = cg_diag32<L>(a.cg);
  stage32<D::NW3>(sW3, a.w3r);
  stage32<D::NW2>(sW2, a.w2r);
  stage32<D::NW1>(sW1, a.w1r);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, el = lane & 15, wv = threadIdx.x >> 6;
  float* sh = sH[wv];
  float* syc = sY[wv];
  for (int k = lane; k < 16 * SY; k += 64) syc[k] = 0.f;   // columns NLM .. SY-1 stay zero
  const float* ht = (const float*)a.ht;
  const float inv_n = a.inv_n;
  // degree of the pull's A-operand row lm = lane % 16
  const int lml = el < 1 ? 0 : (el < 4 ? 1 : (el < 9 ? 2 : 3));
  const RowWalk rw = row_walk<NW>(a.n);
  for (int64_t j = rw.i; j < rw.end; j += rw.step) {
    const int e0 = a.row_ptr[j], e1 = a.row_end ? a.row_end[j] : a.row_ptr[j + 1];
    stage_row32<C, L>(sh, ht + j * NLM * C, lane);
    wave_lds_sync();
    f32x4 hb[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) hb[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
    int par = 0;
    for (int t0 = e0; t0 < e1; t0 += kTileE) {
      const int e = t0 + el;
      const bool valid = e < e1;
      const int i = valid ? a.e_src[e] : 0;
      const float* Ai = a.Abar + (int64_t)i * C + 4 * g;
      Geo geo;
      const float4 v = valid ? a.e_vec[e] : make_float4(-1.f, 0.f, 0.f, 0.f);
      edge_geometry(make_float4(-v.x, -v.y, -v.z, 0.f), valid, gk, geo);
      float yc[NLM];
#pragma unroll
      for (int k = 0; k < NLM; ++k) yc[k] = cgd.c[k] * geo.Y[k];
      if (g == 0) {
#pragma unroll
        for (int k = 0; k < NLM; ++k) syc[el * SY + k] = yc[k];
      }
      const YOps<L> yo = x_ops<L>(yc, g);
      f32x4 p1[4], a1[4], p2[4], a2[4];
      mlp_fwd_rows(geo, lane, sW1, sW2, p1, a1, p2);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) a2[mt][r] = silu(p2[mt][r]);
      wave_lds_sync();
      // pull A operands: row lm = lane % 16, k-slot g of chunk q = edge 4 q + g,
      // masked to the rows of degree l (and lm < NLM)
      float ya[L + 1][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float y = syc[(4 * q + g) * SY + el];   // columns NLM .. 15 are zero
#pragma unroll
        for (int l = 0; l <= L; ++l) ya[l][q] = lml == l ? y : 0.f;
      }
      f32x4 ab2[4], dy[L + 1];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) ab2[mt] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int l = 0; l <= L; ++l) dy[l] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const float4 ad = *(const float4*)(Ai + 16 * t);
        const float ai[4] = {inv_n * ad.x, inv_n * ad.y, inv_n * ad.z, inv_n * ad.w};
        static_for<L + 1>([&](auto lc) {
          constexpr int l = decltype(lc)::value;
          f32x4 R = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kc = 0; kc < 16; ++kc) R = mfma_f32(sW3[phi_f(kc, g) * WS + l * C + 16 * t + el], a2[kc / 4][kc % 4], R);
          const f32x4 X = x_tile<C, L, l>(sh, t, g, el, yo);
          float dR[4], RA[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) { dR[r] = ai[r] * X[r]; RA[r] = ai[r] * R[r]; }
          // MLP adjoint input: ab2[h][e] += sum_c W3[h][(l, c)] dR[c][e]
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
              ab2[mt] = mfma_f32(sW3[(16 * mt + el) * WS + l * C + 16 * t + 4 * g + r], dR[r], ab2[mt]);
          // dE/dYC_l[lm][e] += sum_c h~[lm][c] RA[c][e]; rows lm >= NLM of the
          // staged features are zero, so lanes el >= NLM read row NLMP - 1
          const float4 hv4 = *(const float4*)(sh + (el < D::NLMP ? el : D::NLMP - 1) * C + 16 * t + 4 * g);
          const float hv[4] = {hv4.x, hv4.y, hv4.z, hv4.w};
#pragma unroll
          for (int r = 0; r < 4; ++r) dy[l] = mfma_f32(hv[r], RA[r], dy[l]);
          // pull: RA (channels x edges) to edges x channels through LDS, then
          // h~bar[lm][c] += sum_e YC[lm][e] RA[c][e]
          float* tt = sT[wv][par];
          *(float4*)(tt + el * TS + 4 * g) = make_float4(RA[0], RA[1], RA[2], RA[3]);
          wave_lds_sync();
#pragma unroll
          for (int q = 0; q < 4; ++q) hb[t] = mfma_f32(ya[l][q], tt[(4 * q + g) * TS + el], hb[t]);
          par ^= 1;
        });
      }
      // dE/dYC of edge el: rows lm = 4 g' + r of dy[l(lm)] live in lane el + 16 g'
      float ycb[NLM];
#pragma unroll
      for (int lm = 0; lm < NLM; ++lm) {
        const int l = lm < 1 ? 0 : (lm < 4 ? 1 : 2);
        ycb[lm] = __shfl(dy[l][lm % 4], el + 16 * (lm / 4));
      }
      float eb[kNB];
      mlp_bwd_rows(ab2, p1, p2, lane, sW1, sW2, eb);
      if (lane < kTileE && valid) {
        float Yb[kMaxNlm];
#pragma unroll
        for (int k = 0; k < kMaxNlm; ++k) Yb[k] = k < NLM ? cgd.c[k < NLM ? k : 0] * ycb[k < NLM ? k : 0] : 0.f;
        // geometry backward: dE/dr = dbar u + (I - u u^T)/d (dP/du)^T Ybar
        float dbar = 0.f;
#pragma unroll
        for (int n = 0; n < kNB; ++n) dbar += eb[n] * geo.dbasis[n];
        float gu[3];
        sh_grad_contract(Yb, geo.u, gu);
        const float ud = gu[0] * geo.u[0] + gu[1] * geo.u[1] + gu[2] * geo.u[2];
        const float invd = __builtin_amdgcn_rcpf(geo.d);
        const float4 gr = make_float4(dbar * geo.u[0] + (gu[0] - ud * geo.u[0]) * invd,
                                      dbar * geo.u[1] + (gu[1] - ud * geo.u[1]) * invd,
                                      dbar * geo.u[2] + (gu[2] - ud * geo.u[2]) * invd, 0.f);
        if (a.g2p) {
          a.g2p[e] = gr;   // dE/dr of the reverse edge, kept in this edge's slot
        } else {
          const int rv = a.e_rev[e];
          if (rv >= 0) {
            float4 acc = a.g[rv];
            acc.x += gr.x; acc.y += gr.y; acc.z += gr.z;
            a.g[rv] = acc;
          }
        }
      }
      wave_lds_sync();
    }
    // h~bar_j[lm][c]: D rows lm = 4 g + r, column c = 16 t + el
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lm = 4 * g + r;
      if (lm < NLM) {
        float* dst = a.htbar + ((int64_t)j * NLM + lm) * C + el;
#pragma unroll
        for (int t = 0; t < NT; ++t) dst[16 * t] = hb[t][r];
      }
    }
    wave_lds_sync();
  }
}

// persistent grid: a multiple of 8 workgroups of NW waves (one row range per
// XCD), one workgroup per CU (the weights fill most of the LDS)
static int grid32(int64_t n, int nw) {
  const int64_t need = (n / 8 + nw - 1) / nw;
  const int64_t per = need < 1 ? 1 : (need < 32 ? need : 32);
  return (int)(8 * per);
}

template <int C, int L>
static void l2_32(int which, const FastArgs& a, hipStream_t s) {
  constexpr int NW = 4;
  if (which == 0) k_l2_msg32<C, L, NW><<<grid32(a.n, NW), 64 * NW, 0, s>>>(a);
  else if (which == 1) k_l2_msum32<C><<<(unsigned)((a.n + 3) / 4), 256, 0, s>>>(a);
  else k_l2_adj32<C, L, NW><<<grid32(a.n, NW), 64 * NW, 0, s>>>(a);
}

void launch_l2_32(int C, int L, int which, const FastArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  if (C == 64 && L == 1) l2_32<64, 1>(which, a, s);
  else if (C == 64) l2_32<64, 2>(which, a, s);
  else if (L == 1) l2_32<128, 1>(which, a, s);
  else l2_32<128, 2>(which, a, s);
}

}  // namespace mpip
