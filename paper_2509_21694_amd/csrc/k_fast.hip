// Specialised edge kernels for the first and the last message-passing layer
// (l_max <= 2, 64 or 128 channels) -- the layers of a depth-pruned model.
//
// First layer (input features depend on the sender's species only).
//   A_i[lm, c] = sum_e R_e[l, c] ht1[s_e, c] YC_e[lm] / n_avg with
//   R_e[l, c] = sum_k a2_e[k] W3[k, (l, c)], so
//   A_i[lm, c] = sum_{s,k} Q_i[lm, (s, k)] V_l[(s, k), c],
//   Q_i[lm, (s, k)] = sum_{e: s_e = s} a2_e[k] YC_e[lm],
//   V_l[(s, k), c]  = ht1[s, c] W3[k, (l, c)] / n_avg.
// The per-edge work drops to the two hidden MLP layers plus a 16-edge MFMA
// contraction into Q; the channel dimension moves to one node GEMM per l.
// Its adjoint uses P_i = dA_i V^T: dE/da2_e[k] = sum_lm YC_e[lm] P_i[lm, (s_e, k)]
// and dE/dYC_e[lm] = sum_k a2_e[k] P_i[lm, (s_e, k)], both small MFMAs.
//
// Last layer (only scalars out, paths (l, l, 0)).
//   forward:  A_i[c] = sum_e sum_l R_e[l, c] <ht_j[l, :, c], YC_e[l, :]> / n_avg
//             with R in edges x channels MFMA layout (each lane: 4 edges x
//             C/16 contiguous channels), messages summed in registers.
//   adjoint a: channels x edges layout (each lane: one edge x C/4 channels):
//             dR, dE/dY, and the MLP adjoint fed straight from registers.
//   adjoint b: edges x channels layout: the sender-side feature adjoint
//             pulled through the reverse edge (same length, Y_l(-u) =
//             (-1)^l Y_l(u)), summed in registers.
#include "edge_common.h"

namespace mpip {

typedef __attribute__((ext_vector_type(4))) short s16x4;

__device__ __forceinline__ short bfbits(float x) {
  __bf16 b = (__bf16)x;
  return __builtin_bit_cast(short, b);
}
__device__ __forceinline__ float bf2f(unsigned short u) { return __uint_as_float(((unsigned)u) << 16); }

__device__ __forceinline__ f32x4 mfma_bf16_k16(s16x4 a, s16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bool fast_guard(const FastArgs& a) {
  return (int64_t)a.row_ptr[a.n] > a.capacity || a.status[ST_FLAGS] != 0;
}

// YC of the first-layer paths (0, l, l): YC[l^2 + m] = sum_m2 C[0][m2][m] Y[l^2 + m2]
template <int L>
__device__ __forceinline__ void yc_first(const float* cg, const float* Y, float* yc) {
  int off = 0;
#pragma unroll
  for (int l = 0; l <= L; ++l) {
    const int n = 2 * l + 1;
#pragma unroll
    for (int m = 0; m < n; ++m) {
      float s = 0.f;
#pragma unroll
      for (int m2 = 0; m2 < n; ++m2) s += cg[off + m2 * n + m] * Y[l * l + m2];
      yc[l * l + m] = s;
    }
    off += n * n;
  }
}

// YC of the last-layer paths (l, l, 0): YC[l^2 + m] = sum_m2 C[m][m2][0] Y[l^2 + m2]
template <int L>
__device__ __forceinline__ void yc_last(const float* cg, const float* Y, float* yc) {
  int off = 0;
#pragma unroll
  for (int l = 0; l <= L; ++l) {
    const int n = 2 * l + 1;
#pragma unroll
    for (int m = 0; m < n; ++m) {
      float s = 0.f;
#pragma unroll
      for (int m2 = 0; m2 < n; ++m2) s += cg[off + m * n + m2] * Y[l * l + m2];
      yc[l * l + m] = s;
    }
    off += n * n;
  }
}

// adjoint of yc_last: Ybar[l^2 + m2] = sum_m C[m][m2][0] ycbar[l^2 + m]
template <int L>
__device__ __forceinline__ void yc_last_adj(const float* cg, const float* ycb, float* Yb) {
  int off = 0;
#pragma unroll
  for (int l = 0; l <= L; ++l) {
    const int n = 2 * l + 1;
#pragma unroll
    for (int m2 = 0; m2 < n; ++m2) {
      float s = 0.f;
#pragma unroll
      for (int m = 0; m < n; ++m) s += cg[off + m * n + m2] * ycb[l * l + m];
      Yb[l * l + m2] = s;
    }
    off += n * n;
  }
}

template <int L>
__device__ __forceinline__ void yc_first_adj(const float* cg, const float* ycb, float* Yb) {
  int off = 0;
#pragma unroll
  for (int l = 0; l <= L; ++l) {
    const int n = 2 * l + 1;
#pragma unroll
    for (int m2 = 0; m2 < n; ++m2) {
      float s = 0.f;
#pragma unroll
      for (int m = 0; m < n; ++m) s += cg[off + m2 * n + m] * ycb[l * l + m];
      Yb[l * l + m2] = s;
    }
    off += n * n;
  }
}

// geometry backward: g_e += dbar u + (I - u u^T)/d (dP/du)^T Ybar
__device__ __forceinline__ void add_edge_grad(float4* g, int e, const Geo& geo, const float* ebar, const float* Yb) {
  float dbar = 0.f;
#pragma unroll
  for (int n = 0; n < kNB; ++n) dbar += ebar[n] * geo.dbasis[n];
  float gu[3];
  sh_grad_contract(Yb, geo.u, gu);
  const float ud = gu[0] * geo.u[0] + gu[1] * geo.u[1] + gu[2] * geo.u[2];
  const float invd = 1.0f / geo.d;
  float4 acc = g[e];
  acc.x += dbar * geo.u[0] + (gu[0] - ud * geo.u[0]) * invd;
  acc.y += dbar * geo.u[1] + (gu[1] - ud * geo.u[1]) * invd;
  acc.z += dbar * geo.u[2] + (gu[2] - ud * geo.u[2]) * invd;
  g[e] = acc;
}

// remaining MLP adjoint: pb2 = ab2 * silu'(p2) -> W2 -> silu'(p1) -> W1 -> ebar (LDS [16][8])
template <int PREC>
__device__ __forceinline__ void mlp_backward(const f32x4* ab2, const f32x4* p1, const f32x4* p2, int lane,
                                             const void* w2b, const void* w1b, float* seb) {
  typedef Op<PREC> O;
  const int g = lane >> 4, el = lane & 15;
  f32x4 pb2[4], pb1[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) pb2[mt][r] = ab2[mt][r] * dsilu(p2[mt][r]);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < O::KC64; ++kc)
      acc = O::mma(O::load(w2b, (mt * O::KC64 + kc) * 64 + lane), O::from_tiles(pb2, kc), acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) pb1[mt][r] = acc[r] * dsilu(p1[mt][r]);
  }
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kc = 0; kc < O::KC64; ++kc) acc = O::mma(O::load(w1b, kc * 64 + lane), O::from_tiles(pb1, kc), acc);
  if (g < 2) {
#pragma unroll
    for (int r = 0; r < 4; ++r) seb[el * kNB + 4 * g + r] = acc[r];
  }
}

// ============================================================ first layer

template <int PREC, int L, int MQ>
__global__ __launch_bounds__(64) void k_l1_fwd(FastArgs a) {
  typedef Op<PREC> O;
  constexpr int NLM = (L + 1) * (L + 1);
  __shared__ float syc[kTileE * NLM];
  __shared__ int ssp[kTileE];
  if (fast_guard(a)) return;
  const int lane = threadIdx.x, g = lane >> 4, el = lane & 15;
  const int S = a.n_species, KQ = 64 * S, MROWS = S * NLM;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    const int e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
    f32x4 q[MQ][4];
#pragma unroll
    for (int mt = 0; mt < MQ; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) q[mt][nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int t0 = e0; t0 < e1; t0 += kTileE) {
      const int e = t0 + el;
      const bool valid = e < e1;
      Geo geo;
      const float4 v = valid ? a.e_vec[e] : make_float4(1.f, 0.f, 0.f, 0.f);
      edge_geometry(v, valid, a.rc, a.envelope_p, geo);
      __syncthreads();
      if (lane < kTileE) {
        float yc[NLM];
        yc_first<L>(a.cg, geo.Y, yc);
#pragma unroll
        for (int k = 0; k < NLM; ++k) syc[el * NLM + k] = yc[k];
        ssp[el] = valid ? __float_as_int(v.w) : -1;
      }
      // radial MLP layer 1 (features x edges), layer 2 (edges x features)
      f32x4 p1[4], a1[4], a2[4];
      {
        const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          f32x4 acc = z;
          if constexpr (PREC == 1) {
            acc = O::mma(O::load(a.w1a, mt * 64 + lane), basis_op_bf16(geo.basis, g), acc);
          } else {
#pragma unroll
            for (int qq = 0; qq < 2; ++qq)
              acc = O::mma(O::load(a.w1a, (mt * 2 + qq) * 64 + lane), geo.basis[4 * qq + g], acc);
          }
          p1[mt] = acc;
#pragma unroll
          for (int r = 0; r < 4; ++r) a1[mt][r] = silu(acc[r]);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          f32x4 acc = z;
#pragma unroll
          for (int kc = 0; kc < O::KC64; ++kc)
            acc = O::mma(O::from_tiles(a1, kc), O::load(a.w2f, (nt * O::KC64 + kc) * 64 + lane), acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) a2[nt][r] = silu(acc[r]);
        }
      }
      __syncthreads();
      // Q^T[(s,lm), k] += sum_e Ysel[e, (s,lm)] a2[e, k]; a2 tile nt: edges 4g + r, hidden 16 nt + el
#pragma unroll
      for (int mt = 0; mt < MQ; ++mt) {
        const int m = 16 * mt + el;
        const int s = m / NLM, lm = m - s * NLM;
        float ys[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ee = 4 * g + r;
          ys[r] = (m < MROWS && ssp[ee] == s) ? syc[ee * NLM + lm] : 0.f;
        }
        if constexpr (PREC == 1) {
          s16x4 av = {bfbits(ys[0]), bfbits(ys[1]), bfbits(ys[2]), bfbits(ys[3])};
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) {
            s16x4 bv = {bfbits(a2[nt][0]), bfbits(a2[nt][1]), bfbits(a2[nt][2]), bfbits(a2[nt][3])};
            q[mt][nt] = mfma_bf16_k16(av, bv, q[mt][nt]);
          }
        } else {
#pragma unroll
          for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) q[mt][nt] = mfma_f32(ys[r], a2[nt][r], q[mt][nt]);
        }
      }
      (void)p1;
    }
    // Q_i[lm][s*64 + k]: D rows (s,lm) = 16 mt + 4 g + r, hidden k = 16 nt + el
#pragma unroll
    for (int mt = 0; mt < MQ; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = 16 * mt + 4 * g + r;
        if (m < MROWS) {
          const int s = m / NLM, lm = m - s * NLM;
          const int64_t o = ((int64_t)i * NLM + lm) * KQ + s * 64 + el;
          if constexpr (PREC == 1) {
            __bf16* dst = (__bf16*)a.Q + o;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) dst[16 * nt] = (__bf16)q[mt][nt][r];
          } else {
            float* dst = a.Q + o;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) dst[16 * nt] = q[mt][nt][r];
          }
        }
      }
  }
}

template <int PREC, int L, int MQ>
__global__ __launch_bounds__(64) void k_l1_bwd(FastArgs a) {
  typedef Op<PREC> O;
  constexpr int NLM = (L + 1) * (L + 1);
  constexpr int KCQ = (PREC == 1) ? (MQ + 1) / 2 : 4 * MQ;   // k-chunks over the (s,lm) rows
  __shared__ float syb[kTileE * 16 * MQ];
  __shared__ float seb[kTileE * kNB];
  if (fast_guard(a)) return;
  const int lane = threadIdx.x, g = lane >> 4, el = lane & 15;
  const int S = a.n_species, KQ = 64 * S, MROWS = S * NLM;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    const int e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
    const float* Pi = a.P + (int64_t)i * NLM * KQ;
    const __bf16* Pbi = (const __bf16*)a.P + (int64_t)i * NLM * KQ;
    auto Pval = [&](int m, int k) -> float {
      if (m >= MROWS) return 0.f;
      const int s = m / NLM, lm = m - s * NLM;
      if constexpr (PREC == 1) return (float)Pbi[lm * KQ + s * 64 + k];
      else return Pi[lm * KQ + s * 64 + k];
    };
    // A operand of dE/da2^T = P^T Ysel^T: rows hidden 16 mt + el, k over (s,lm)
    typename O::T pa[4][KCQ];
    // A operand of dE/dYC^T = P a2^T: rows (s,lm) 16 mq + el, k over hidden (permuted)
    typename O::T pb[MQ][O::KC64];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int kc = 0; kc < KCQ; ++kc) {
        if constexpr (PREC == 1) {
#pragma unroll
          for (int j = 0; j < 8; ++j) pa[mt][kc][j] = (__bf16)Pval(32 * kc + 8 * g + j, 16 * mt + el);
        } else {
          pa[mt][kc] = Pval(4 * kc + g, 16 * mt + el);
        }
      }
#pragma unroll
    for (int mq = 0; mq < MQ; ++mq)
#pragma unroll
      for (int kc = 0; kc < O::KC64; ++kc) {
        if constexpr (PREC == 1) {
#pragma unroll
          for (int j = 0; j < 8; ++j)
            pb[mq][kc][j] = (__bf16)Pval(16 * mq + el, 16 * (2 * kc + j / 4) + 4 * g + (j % 4));
        } else {
          pb[mq][kc] = Pval(16 * mq + el, 16 * (kc / 4) + 4 * g + (kc % 4));
        }
      }
    for (int t0 = e0; t0 < e1; t0 += kTileE) {
      const int e = t0 + el;
      const bool valid = e < e1;
      Geo geo;
      const float4 v = valid ? a.e_vec[e] : make_float4(1.f, 0.f, 0.f, 0.f);
      edge_geometry(v, valid, a.rc, a.envelope_p, geo);
      const int sp = valid ? __float_as_int(v.w) : -1;
      float yc[NLM];
      yc_first<L>(a.cg, geo.Y, yc);
      f32x4 p1[4], p2[4], a2[4], ab2[4];
      mlp_forward<PREC>(geo, lane, a.w1a, a.w2a, p1, p2);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) a2[mt][r] = silu(p2[mt][r]);
      // Ysel^T operand for this lane's edge (column el): slot -> row m of (s, lm)
      auto ysel = [&](int m) -> float {
        if (m >= MROWS) return 0.f;
        const int s = m / NLM, lm = m - s * NLM;
        float val = 0.f;
#pragma unroll
        for (int k = 0; k < NLM; ++k) val = (k == lm) ? yc[k] : val;
        return (s == sp) ? val : 0.f;
      };
      typename O::T yb[KCQ];
#pragma unroll
      for (int kc = 0; kc < KCQ; ++kc) {
        if constexpr (PREC == 1) {
#pragma unroll
          for (int j = 0; j < 8; ++j) yb[kc][j] = (__bf16)ysel(32 * kc + 8 * g + j);
        } else {
          yb[kc] = ysel(4 * kc + g);
        }
      }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < KCQ; ++kc) acc = O::mma(pa[mt][kc], yb[kc], acc);
        ab2[mt] = acc;
      }
      __syncthreads();
#pragma unroll
      for (int mq = 0; mq < MQ; ++mq) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < O::KC64; ++kc) acc = O::mma(pb[mq][kc], O::from_tiles(a2, kc), acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) syb[el * (16 * MQ) + 16 * mq + 4 * g + r] = acc[r];
      }
      mlp_backward<PREC>(ab2, p1, p2, lane, a.w2b, a.w1b, seb);
      __syncthreads();
      if (lane < kTileE && valid) {
        float ycb[NLM], Yb[kMaxNlm];
#pragma unroll
        for (int k = 0; k < kMaxNlm; ++k) Yb[k] = 0.f;
#pragma unroll
        for (int k = 0; k < NLM; ++k) ycb[k] = syb[el * (16 * MQ) + sp * NLM + k];
        yc_first_adj<L>(a.cg, ycb, Yb);
        add_edge_grad(a.g, e, geo, seb + el * kNB, Yb);
      }
    }
  }
}

// ============================================================ last layer

template <int PREC> struct HT;
template <> struct HT<1> {  // bf16 features
  typedef unsigned short T;
  // N consecutive values starting at an address aligned to 2*N bytes (N = 4 or 8)
  template <int N>
  __device__ static void loadN(const T* p, float* out) {
    if constexpr (N == 8) {
      const uint4 w = *(const uint4*)p;
      const unsigned u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        out[2 * k] = __uint_as_float(u[k] << 16);
        out[2 * k + 1] = __uint_as_float(u[k] & 0xffff0000u);
      }
    } else {
      const uint2 w = *(const uint2*)p;
      out[0] = __uint_as_float(w.x << 16);
      out[1] = __uint_as_float(w.x & 0xffff0000u);
      out[2] = __uint_as_float(w.y << 16);
      out[3] = __uint_as_float(w.y & 0xffff0000u);
    }
  }
};
template <> struct HT<0> {
  typedef float T;
  template <int N>
  __device__ static void loadN(const T* p, float* out) {
#pragma unroll
    for (int k = 0; k < N; k += 4) {
      const float4 w = *(const float4*)(p + k);
      out[k] = w.x; out[k + 1] = w.y; out[k + 2] = w.z; out[k + 3] = w.w;
    }
  }
};

template <int PREC, int C, int L>
__global__ __launch_bounds__(64) void k_l2_fwd(FastArgs a) {
  typedef Op<PREC> O;
  typedef typename HT<PREC>::T HTy;
  constexpr int NLM = (L + 1) * (L + 1);
  constexpr int CN = C / 16;                 // channels per lane: CN * (lane % 16) .. + CN
  __shared__ float syc[kTileE * NLM];
  __shared__ int sj[kTileE];
  if (fast_guard(a)) return;
  const int lane = threadIdx.x, g = lane >> 4, el = lane & 15;
  const HTy* ht = (const HTy*)a.ht;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    const int e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
    float acc[CN];
#pragma unroll
    for (int t = 0; t < CN; ++t) acc[t] = 0.f;
    for (int t0 = e0; t0 < e1; t0 += kTileE) {
      const int e = t0 + el;
      const bool valid = e < e1;
      Geo geo;
      const float4 v = valid ? a.e_vec[e] : make_float4(1.f, 0.f, 0.f, 0.f);
      edge_geometry(v, valid, a.rc, a.envelope_p, geo);
      __syncthreads();
      if (lane < kTileE) {
        float yc[NLM];
        yc_last<L>(a.cg, geo.Y, yc);
#pragma unroll
        for (int k = 0; k < NLM; ++k) syc[el * NLM + k] = yc[k];
        sj[el] = valid ? a.e_src[e] : -1;
      }
      f32x4 p1[4], p2[4], a2[4];
      mlp_forward<PREC>(geo, lane, a.w1a, a.w2a, p1, p2);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) a2[mt][r] = silu(p2[mt][r]);
      typename O::T aop[O::KC64];
#pragma unroll
      for (int kc = 0; kc < O::KC64; ++kc) aop[kc] = O::from_tiles(a2, kc);
      __syncthreads();
#pragma unroll
      for (int l = 0; l <= L; ++l) {
        f32x4 R[CN];
#pragma unroll
        for (int nt = 0; nt < CN; ++nt) {
          f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kc = 0; kc < O::KC64; ++kc)
            d = O::mma(aop[kc], O::load(a.w3f, ((l * CN + nt) * O::KC64 + kc) * 64 + lane), d);
          R[nt] = d;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ee = 4 * g + r;
          if (t0 + ee < e1) {
            const int j = sj[ee];
            const HTy* hrow = ht + ((int64_t)j * NLM + l * l) * C + CN * el;
            float s[CN];
#pragma unroll
            for (int t = 0; t < CN; ++t) s[t] = 0.f;
#pragma unroll
            for (int m = 0; m < 2 * l + 1; ++m) {
              const float y = syc[ee * NLM + l * l + m];
              float hv[CN];
              HT<PREC>::template loadN<CN>(hrow + m * C, hv);
#pragma unroll
              for (int t = 0; t < CN; ++t) s[t] += hv[t] * y;
            }
#pragma unroll
            for (int t = 0; t < CN; ++t) acc[t] += R[t][r] * s[t];
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < CN; ++t) {
      float vv = acc[t];
      vv += __shfl_xor(vv, 16);
      vv += __shfl_xor(vv, 32);
      acc[t] = vv;
    }
    if (g == 0) {
#pragma unroll
      for (int t = 0; t < CN; ++t) a.A[(int64_t)i * C + CN * el + t] = a.inv_n * acc[t];
    }
  }
}

// adjoint a: lanes own (channel block g of C/4 channels, edge el)
template <int PREC, int C, int L>
__global__ __launch_bounds__(64) void k_l2_bwd_a(FastArgs a) {
  typedef Op<PREC> O;
  typedef typename HT<PREC>::T HTy;
  constexpr int NLM = (L + 1) * (L + 1);
  constexpr int CB = C / 4;                  // channels per lane: CB * g .. + CB
  constexpr int CN = C / 16;                 // M-tiles of the transposed layer-3 product
  constexpr int KCC = O::kch(C);             // k-chunks over channels (MLP adjoint)
  __shared__ float seb[kTileE * kNB];
  if (fast_guard(a)) return;
  const int lane = threadIdx.x, g = lane >> 4, el = lane & 15;
  const HTy* ht = (const HTy*)a.ht;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    const int e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
    float Ai[CB];
#pragma unroll
    for (int q = 0; q < CB; ++q) Ai[q] = a.inv_n * a.Abar[(int64_t)i * C + CB * g + q];
    for (int t0 = e0; t0 < e1; t0 += kTileE) {
      const int e = t0 + el;
      const bool valid = e < e1;
      Geo geo;
      const float4 v = valid ? a.e_vec[e] : make_float4(1.f, 0.f, 0.f, 0.f);
      edge_geometry(v, valid, a.rc, a.envelope_p, geo);
      const int j = valid ? a.e_src[e] : 0;
      float yc[NLM];
      yc_last<L>(a.cg, geo.Y, yc);
      f32x4 p1[4], p2[4], a2[4], ab2[4];
      mlp_forward<PREC>(geo, lane, a.w1a, a.w2a, p1, p2);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) { a2[mt][r] = silu(p2[mt][r]); ab2[mt][r] = 0.f; }
      typename O::T bop[O::KC64];
#pragma unroll
      for (int kc = 0; kc < O::KC64; ++kc) bop[kc] = O::from_tiles(a2, kc);
      float ycb[NLM];
#pragma unroll
      for (int k = 0; k < NLM; ++k) ycb[k] = 0.f;
#pragma unroll
      for (int l = 0; l <= L; ++l) {
        // R^T: rows = channels CB*g + 4 mt + r of this lane's edge
        float R[CB];
#pragma unroll
        for (int mt = 0; mt < CN; ++mt) {
          f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kc = 0; kc < O::KC64; ++kc)
            d = O::mma(O::load(a.w3t, ((l * CN + mt) * O::KC64 + kc) * 64 + lane), bop[kc], d);
#pragma unroll
          for (int r = 0; r < 4; ++r) R[4 * mt + r] = d[r];
        }
        float rb[CB];
        const HTy* hrow = ht + ((int64_t)j * NLM + l * l) * C + CB * g;
#pragma unroll
        for (int q = 0; q < CB; ++q) rb[q] = 0.f;
        if (valid) {
#pragma unroll
          for (int q0 = 0; q0 < CB; q0 += 8) {
            float h[2 * L + 1][8];
#pragma unroll
            for (int m = 0; m < 2 * l + 1; ++m) HT<PREC>::template loadN<8>(hrow + m * C + q0, h[m]);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              float s = 0.f;
#pragma unroll
              for (int m = 0; m < 2 * l + 1; ++m) s += h[m][q] * yc[l * l + m];
              rb[q0 + q] = Ai[q0 + q] * s;
              const float w = R[q0 + q] * Ai[q0 + q];
#pragma unroll
              for (int m = 0; m < 2 * l + 1; ++m) ycb[l * l + m] += w * h[m][q];
            }
          }
        }
        // MLP adjoint through layer 3: ab2^T += W3_l (hidden x C) x rbar^T
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
          for (int kc = 0; kc < KCC; ++kc) {
            typename O::T bv;
            if constexpr (PREC == 1) {
#pragma unroll
              for (int jj = 0; jj < 8; ++jj) bv[jj] = (__bf16)rb[8 * kc + jj];
            } else {
              bv = rb[kc];
            }
            ab2[mt] = O::mma(O::load(a.w3b, ((l * 4 + mt) * KCC + kc) * 64 + lane), bv, ab2[mt]);
          }
      }
#pragma unroll
      for (int k = 0; k < NLM; ++k) {
        float w = ycb[k];
        w += __shfl_xor(w, 16);
        w += __shfl_xor(w, 32);
        ycb[k] = w;
      }
      __syncthreads();
      mlp_backward<PREC>(ab2, p1, p2, lane, a.w2b, a.w1b, seb);
      __syncthreads();
      if (lane < kTileE && valid) {
        float Yb[kMaxNlm];
#pragma unroll
        for (int k = 0; k < kMaxNlm; ++k) Yb[k] = 0.f;
        yc_last_adj<L>(a.cg, ycb, Yb);
        add_edge_grad(a.g, e, geo, seb + el * kNB, Yb);
      }
    }
  }
}

// adjoint b: the sender-side feature adjoint, pulled through the reverse edge
template <int PREC, int C, int L>
__global__ __launch_bounds__(64) void k_l2_bwd_b(FastArgs a) {
  typedef Op<PREC> O;
  constexpr int NLM = (L + 1) * (L + 1);
  constexpr int CN = C / 16;
  __shared__ float syc[kTileE * NLM];
  __shared__ int sj[kTileE];
  if (fast_guard(a)) return;
  const int lane = threadIdx.x, g = lane >> 4, el = lane & 15;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    const int e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
    float hb[NLM][CN];
#pragma unroll
    for (int k = 0; k < NLM; ++k)
#pragma unroll
      for (int t = 0; t < CN; ++t) hb[k][t] = 0.f;
    for (int t0 = e0; t0 < e1; t0 += kTileE) {
      const int e = t0 + el;
      const bool valid = e < e1;
      Geo geo;
      const float4 v = valid ? a.e_vec[e] : make_float4(1.f, 0.f, 0.f, 0.f);
      edge_geometry(v, valid, a.rc, a.envelope_p, geo);
      __syncthreads();
      if (lane < kTileE) {
        float yc[NLM];
        yc_last<L>(a.cg, geo.Y, yc);
#pragma unroll
        for (int l = 0; l <= L; ++l)
#pragma unroll
          for (int m = 0; m < 2 * l + 1; ++m)
            syc[el * NLM + l * l + m] = (l & 1) ? -yc[l * l + m] : yc[l * l + m];
        sj[el] = valid ? a.e_src[e] : -1;
      }
      f32x4 p1[4], p2[4], a2[4];
      mlp_forward<PREC>(geo, lane, a.w1a, a.w2a, p1, p2);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) a2[mt][r] = silu(p2[mt][r]);
      typename O::T aop[O::KC64];
#pragma unroll
      for (int kc = 0; kc < O::KC64; ++kc) aop[kc] = O::from_tiles(a2, kc);
      __syncthreads();
      // gather dA of the 4 senders of this lane's edges (channels CN*el .. + CN)
      float Aj[4][CN];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ee = 4 * g + r;
        const bool ok = (t0 + ee) < e1;
        const int jj = ok ? sj[ee] : 0;
#pragma unroll
        for (int t = 0; t < CN; ++t) Aj[r][t] = ok ? a.inv_n * a.Abar[(int64_t)jj * C + CN * el + t] : 0.f;
      }
#pragma unroll
      for (int l = 0; l <= L; ++l) {
#pragma unroll
        for (int nt = 0; nt < CN; ++nt) {
          f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kc = 0; kc < O::KC64; ++kc)
            d = O::mma(aop[kc], O::load(a.w3f, ((l * CN + nt) * O::KC64 + kc) * 64 + lane), d);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ee = 4 * g + r;
            const float u = d[r] * Aj[r][nt];
#pragma unroll
            for (int m = 0; m < 2 * l + 1; ++m) hb[l * l + m][nt] += u * syc[ee * NLM + l * l + m];
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NLM; ++k)
#pragma unroll
      for (int t = 0; t < CN; ++t) {
        float vv = hb[k][t];
        vv += __shfl_xor(vv, 16);
        vv += __shfl_xor(vv, 32);
        hb[k][t] = vv;
      }
    if (g == 0) {
#pragma unroll
      for (int k = 0; k < NLM; ++k)
#pragma unroll
        for (int t = 0; t < CN; ++t) a.htbar[((int64_t)i * NLM + k) * C + CN * el + t] = hb[k][t];
    }
  }
}

// ============================================================ dispatch

static int fast_grid(int64_t n) {
  int64_t g = n < 262144 ? n : 262144;
  return (int)(g < 1 ? 1 : g);
}

template <int PREC, int L>
static void l1_launch(bool fwd, int mq, const FastArgs& a, hipStream_t s) {
  const int gr = fast_grid(a.n);
#define MPIP_L1(MQ)                                                       \
  if (fwd) k_l1_fwd<PREC, L, MQ><<<gr, 64, 0, s>>>(a);                      \
  else k_l1_bwd<PREC, L, MQ><<<gr, 64, 0, s>>>(a);
  switch (mq) {
    case 1: MPIP_L1(1) break;
    case 2: MPIP_L1(2) break;
    case 3: MPIP_L1(3) break;
    default: MPIP_L1(4) break;
  }
#undef MPIP_L1
}

void launch_l1(int prec, int L, bool fwd, const FastArgs& a, hipStream_t s) {
  const int nlm = (L + 1) * (L + 1);
  const int mq = (a.n_species * nlm + 15) / 16;
  if (prec == MPIP_BF16_MIXED) {
    if (L == 1) l1_launch<1, 1>(fwd, mq, a, s); else l1_launch<1, 2>(fwd, mq, a, s);
  } else {
    if (L == 1) l1_launch<0, 1>(fwd, mq, a, s); else l1_launch<0, 2>(fwd, mq, a, s);
  }
}

template <int PREC, int C, int L>
static void l2_launch(int which, const FastArgs& a, hipStream_t s) {
  const int gr = fast_grid(a.n);
  if (which == 0) k_l2_fwd<PREC, C, L><<<gr, 64, 0, s>>>(a);
  else if (which == 1) k_l2_bwd_a<PREC, C, L><<<gr, 64, 0, s>>>(a);
  else k_l2_bwd_b<PREC, C, L><<<gr, 64, 0, s>>>(a);
}

template <int PREC>
static void l2_prec(int C, int L, int which, const FastArgs& a, hipStream_t s) {
  if (C == 64 && L == 1) l2_launch<PREC, 64, 1>(which, a, s);
  else if (C == 64 && L == 2) l2_launch<PREC, 64, 2>(which, a, s);
  else if (C == 128 && L == 1) l2_launch<PREC, 128, 1>(which, a, s);
  else l2_launch<PREC, 128, 2>(which, a, s);
}

void launch_l2(int prec, int C, int L, int which, const FastArgs& a, hipStream_t s) {
  if (prec == MPIP_BF16_MIXED) l2_prec<1>(C, L, which, a, s);
  else l2_prec<0>(C, L, which, a, s);
}

}  // namespace mpip
