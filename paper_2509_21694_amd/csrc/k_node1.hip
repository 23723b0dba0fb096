// Fused node-side kernels between a species-factorised first layer and the
// last layer of a two-layer evaluation (BF16 form).
//
// Forward: z_l = Q_l (V_l W_down_l) (the first layer's down projection
// folded into the factorised messages), the gates, and the last layer's
// up projection h~ = h W_up, per tile of 16 atoms with every intermediate
// in registers; only h_0 (FP32, the residual and readout input) and h~
// (BF16, the last layer's gathered features) are written.
// Adjoint: hbar_l = h~bar_l W_up_l^T (+ w_read on root scalars), the gate
// adjoint with z recomputed from Q, and P_l = zbar_l (V_l W_down_l)^T, in
// the same tiles; only P (BF16) is written, over Q's rows of the same atoms.
//
// Orientation: every product is computed transposed (features x atoms), so a
// D tile's rows are features and one lane column is one atom; the rows of a
// D tile become the k operand of the next product through the same
// permutation as the radial MLP (k-slot (g, j) of chunk kc = row
// 16 (2 kc + j/4) + 4 g + j%4), so no data leaves the registers between the
// stages.
#include <utility>

#include "kernels.h"

namespace mpip {

namespace {

__device__ __forceinline__ bf16x8 tiles_to_op(const f32x4* t, int kc) {
  bf16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = (__bf16)t[2 * kc + j / 4][j % 4];
  return v;
}

// 8 values of a lane's contiguous output run as one 16-byte BF16 store
__device__ __forceinline__ void store8_bf16(__bf16* dst, const float* v) {
  bf16x8 o;
#pragma unroll
  for (int j = 0; j < 8; ++j) o[j] = (__bf16)v[j];
  *(bf16x8*)dst = o;
}

// operand tile `tile` of a packed weight array: a uniform base plus a 32-bit
// lane offset, so the address needs no per-lane 64-bit register
__device__ __forceinline__ bf16x8 wtile(const bf16x8* W, int tile, int lane) {
  const bf16x8* b = W + (size_t)tile * 64;
  asm volatile("" : "+s"(b));   // keep the tile base scalar and computed at its use
  return *(const bf16x8*)((const char*)b + (unsigned)lane * 16u);
}

template <typename F, int... Is>
__device__ __forceinline__ void unroll_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}

// D tiles mt = 0..MT-1 of W x B with W given as A-operand tiles
// W[(mt0 + mt) * KS + k0 + kc] (kc < KC) and B as KC operands; the weights
// are streamed from memory one M-tile ahead of their use and each finished
// tile is handed to consume(mt, d), so only two tiles of weights are live.
template <int MT, int KC, typename F>
__device__ __forceinline__ void stream_rows(const bf16x8* W, int mt0, int KS, int k0, const bf16x8* B, int lane,
                                           F&& consume) {
  bf16x8 wb[2][KC];
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) wb[0][kc] = wtile(W, mt0 * KS + k0 + kc, lane);
  unroll_impl([&](auto mc) {
    constexpr int mt = decltype(mc)::value;
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (mt + 1 < MT) {
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) wb[(mt + 1) & 1][kc] = wtile(W, (mt0 + mt + 1) * KS + k0 + kc, lane);
    }
    f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) d = mfma_bf16(wb[mt & 1][kc], B[kc], d);
    consume(mt, d);
  }, std::make_integer_sequence<int, MT>{});
  __builtin_amdgcn_sched_barrier(0);
}

}  // namespace

// a lane's output run, written two D tiles (8 values) at a time as one 16-byte BF16 store
struct PairStore {
  float v[4];
  __device__ __forceinline__ void put(int mt, const f32x4& d, __bf16* base) {
    if (mt & 1) {
      const float o[8] = {v[0], v[1], v[2], v[3], d[0], d[1], d[2], d[3]};
      store8_bf16(base + 4 * (mt - 1), o);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = d[r];
    }
  }
};

// whole-block copy of NT operand tiles (64 lanes x 16 B each) into LDS,
// complete after lds_dma_sync()
template <int NT>
__device__ __forceinline__ void stage_tiles(bf16x8* dst, const bf16x8* src) {
  lds_dma_tiles<NT>(dst, src);
}

// D tiles mt = 0..MT-1 of W x B with W's A-operand tiles in LDS at
// W[(mt * KS + k0 + kc) * 64 + lane] (kc < KC) and B as KC operands; the
// operand reads run PF tiles ahead of the MFMAs, and each finished tile is
// handed to consume(mt, d)
template <int MT, int KC, typename F>
__device__ __forceinline__ void lds_rows(const bf16x8* W, int KS, int k0, const bf16x8* B, int lane, F&& consume) {
  constexpr int T = MT * KC, PF = 4;
  auto ld = [&](int i) { return W[((i / KC) * KS + k0 + i % KC) * 64 + lane]; };
  bf16x8 buf[PF];
#pragma unroll
  for (int i = 0; i < PF && i < T; ++i) buf[i] = ld(i);
  f32x4 d = {0.f, 0.f, 0.f, 0.f};
  unroll_impl([&](auto ic) {
    constexpr int i = decltype(ic)::value, kc = i % KC;
    if constexpr (kc == 0) __builtin_amdgcn_sched_barrier(0);
    const bf16x8 w = buf[i % PF];
    if constexpr (i + PF < T) buf[i % PF] = ld(i + PF);
    d = mfma_bf16(w, B[kc], d);
    if constexpr (kc == KC - 1) {
      consume(i / KC, d);
      d = (f32x4){0.f, 0.f, 0.f, 0.f};
    }
  }, std::make_integer_sequence<int, T>{});
  __builtin_amdgcn_sched_barrier(0);
}

// Workgroups of 8 waves (128 atoms, 16 per wave).  Each stage's weights are
// staged in LDS once per workgroup and read by all its waves, so a weight
// tile crosses L2 once per 128 atoms; waves past the last atom still take
// part in the staging and the barriers.
constexpr int kN1Waves = 8;

template <int C, int L, int S>
__global__ __launch_bounds__(64 * kN1Waves) __attribute__((amdgpu_waves_per_eu(4))) void k_node1_fwd(Node1Args a) {
  constexpr int NLM = (L + 1) * (L + 1), KQ = 64 * S, KCQ = KQ / 32, MTC = C / 16, KCC = C / 32;
  constexpr int NVT = MTC * KCQ, NU = MTC * KCC;   // tiles of one z block of VW^T and of W_up^T
  __shared__ bf16x8 sV[NVT * 64], sU[NU * 64];
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
  const int64_t a0 = ((int64_t)blockIdx.x * kN1Waves + (threadIdx.x >> 6)) * 16;
  const bool act = a0 < a.n;
  const bool av = act && a0 + n < a.n;
  const int64_t at = av ? a0 + n : (act ? a.n - 1 : 0);
  const bf16x8* Q = (const bf16x8*)a.Q;   // [N][NLM][KQ / 8]
  const bf16x8* VT0 = (const bf16x8*)a.vwt[0];
  const int sp = a.spec_s[at];
  auto qload = [&](int lm, bf16x8* qv) {
#pragma unroll
    for (int kc = 0; kc < KCQ; ++kc) qv[kc] = Q[((int64_t)at * NLM + lm) * (KQ / 8) + 4 * kc + g];
  };
  // h~ rows of one (l, m) from the W_up^T tiles in sU: D tile mt, lane (g, n)
  // holds output channel (C/4) g + 4 mt + r
  auto up_store = [&](int lm, const f32x4* h) {
    bf16x8 hb[KCC];
#pragma unroll
    for (int kc = 0; kc < KCC; ++kc) hb[kc] = tiles_to_op(h, kc);
    __bf16* dst = (__bf16*)a.ht + ((int64_t)at * NLM + lm) * C + (C / 4) * g;
    PairStore ps;
    lds_rows<MTC, KCC>(sU, KCC, 0, hb, lane, [&](int mt, f32x4 d) {
      if (av) ps.put(mt, d, dst);
    });
  };
  // scalars: h_0 = emb + SiLU(z_0[0:C])
  stage_tiles<NVT>(sV, VT0);
  stage_tiles<NU>(sU, (const bf16x8*)a.upt[0]);
  lds_dma_sync();
  if (act) {
    bf16x8 q0[KCQ];
    qload(0, q0);
    f32x4 z[MTC];
    lds_rows<MTC, KCQ>(sV, KCQ, 0, q0, lane, [&](int mt, f32x4 d) {
      const float4 e = *(const float4*)(a.emb + (int64_t)sp * C + 16 * mt + 4 * g);
      const float ev[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
      for (int r = 0; r < 4; ++r) z[mt][r] = ev[r] + silu(d[r]);
      if (av) *(float4*)(a.h + (int64_t)at * NLM * C + 16 * mt + 4 * g) = make_float4(z[mt][0], z[mt][1], z[mt][2], z[mt][3]);
    });
    up_store(0, z);
  }
  // degrees l >= 1: h_lm = sigmoid(z_0[gate block l]) * z_lm
#pragma unroll
  for (int l = 1; l <= L; ++l) {
    __syncthreads();
    stage_tiles<NVT>(sV, VT0 + (size_t)l * NVT * 64);
    lds_dma_sync();
    f32x4 gt[MTC];
    if (act) {
      bf16x8 q0[KCQ];
      qload(0, q0);
      lds_rows<MTC, KCQ>(sV, KCQ, 0, q0, lane, [&](int mt, f32x4 d) {
#pragma unroll
        for (int r = 0; r < 4; ++r) gt[mt][r] = sigm(d[r]);
      });
    }
    __syncthreads();
    stage_tiles<NVT>(sV, (const bf16x8*)a.vwt[l]);
    stage_tiles<NU>(sU, (const bf16x8*)a.upt[l]);
    lds_dma_sync();
    if (act) {
      for (int m = 0; m < 2 * l + 1; ++m) {
        const int lm = l * l + m;
        bf16x8 ql[KCQ];
        qload(lm, ql);
        f32x4 z[MTC];
        lds_rows<MTC, KCQ>(sV, KCQ, 0, ql, lane, [&](int mt, f32x4 d) {
#pragma unroll
          for (int r = 0; r < 4; ++r) z[mt][r] = gt[mt][r] * d[r];
        });
        up_store(lm, z);
      }
    }
  }
}

template <int C, int L, int S>
struct N1Bwd {
  static constexpr int NLM = (L + 1) * (L + 1), KQ = 64 * S, KCQ = KQ / 32, MTC = C / 16, KCC = C / 32;
  static constexpr int MTP = KQ / 16, NZC = (1 + L) * KCC;   // P row tiles; k-chunks of z_0
  static constexpr int NVT = MTC * KCQ, NU = MTC * KCC, NVW = MTP * KCC, NP0 = (MTP / 2) * NZC;
  static constexpr int NT = (NVT + NU + NVW) > NP0 ? (NVT + NU + NVW) : NP0;   // LDS tiles
};

template <int C, int L, int S>
__global__ __launch_bounds__(64 * kN1Waves) __attribute__((amdgpu_waves_per_eu(2))) void k_node1_bwd(Node1Args a) {
  typedef N1Bwd<C, L, S> D;
  constexpr int NLM = D::NLM, KQ = D::KQ, KCQ = D::KCQ, MTC = D::MTC, KCC = D::KCC, MTP = D::MTP, NZC = D::NZC;
  constexpr int NVT = D::NVT, NU = D::NU;
  __shared__ bf16x8 sW[D::NT * 64];
  bf16x8* sU = sW;                  // W_up_l (hbar rows)
  bf16x8* sV = sW + NU * 64;        // a z block of VW^T
  bf16x8* sP = sV + NVT * 64;       // VW_l (P rows)
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
  const int64_t a0 = ((int64_t)blockIdx.x * kN1Waves + (threadIdx.x >> 6)) * 16;
  const bool act = a0 < a.n;
  const bool av = act && a0 + n < a.n;
  const int64_t at = av ? a0 + n : (act ? a.n - 1 : 0);
  const bf16x8* Q = (const bf16x8*)a.Q;
  const bf16x8* HB = (const bf16x8*)a.htbar;   // [N][NLM][C / 8]
  const bf16x8* VT0 = (const bf16x8*)a.vwt[0];
  const bool own = a.owned_s[at] != 0;
  auto qload = [&](int lm, bf16x8* qv) {
#pragma unroll
    for (int kc = 0; kc < KCQ; ++kc) qv[kc] = Q[((int64_t)at * NLM + lm) * (KQ / 8) + 4 * kc + g];
  };
  // hbar rows of one (l, m): W_up_l h~bar_lm^T, channel 16 mt + 4 g + r (the positions of z)
  auto hbar_row = [&](int lm, f32x4* hb) {
    bf16x8 hv[KCC];
#pragma unroll
    for (int kc = 0; kc < KCC; ++kc) hv[kc] = HB[((int64_t)at * NLM + lm) * (C / 8) + 4 * kc + g];
    lds_rows<MTC, KCC>(sU, KCC, 0, hv, lane, [&](int mt, f32x4 d) { hb[mt] = d; });
  };
  // P rows: D tile mt, lane (g, n) holds P index (KQ/4) g + 4 mt + r
  auto pdst = [&](int lm) { return (__bf16*)a.P + ((int64_t)at * NLM + lm) * KQ + (KQ / 4) * g; };
  // zbar_0 blocks as B operands (scalars, then one gate block per l); P_0 is
  // formed from them at the end, after the last read of Q_0 (P overwrites Q)
  bf16x8 z0b[(1 + L) * KCC];
  // scalars: zbar_0[0:C] = hbar_0 * SiLU'(z_0[0:C]), hbar_0 = w_read (root atoms) + W_up_0 h~bar_0
  stage_tiles<NU>(sU, (const bf16x8*)a.up[0]);
  stage_tiles<NVT>(sV, VT0);
  lds_dma_sync();
  if (act) {
    f32x4 hb[MTC];
    hbar_row(0, hb);
    bf16x8 q0[KCQ];
    qload(0, q0);
    lds_rows<MTC, KCQ>(sV, KCQ, 0, q0, lane, [&](int mt, f32x4 d) {
      const float4 w = *(const float4*)(a.w_read + 16 * mt + 4 * g);
      const float wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int r = 0; r < 4; ++r) hb[mt][r] = (hb[mt][r] + (own ? wv[r] : 0.f)) * dsilu(d[r]);
    });
#pragma unroll
    for (int kc = 0; kc < KCC; ++kc) z0b[kc] = tiles_to_op(hb, kc);
  }
#pragma unroll
  for (int l = 1; l <= L; ++l) {
    __syncthreads();
    stage_tiles<NVT>(sV, VT0 + (size_t)l * NVT * 64);
    lds_dma_sync();
    f32x4 s[MTC], dg[MTC];
    if (act) {
      bf16x8 q0[KCQ];
      qload(0, q0);
      lds_rows<MTC, KCQ>(sV, KCQ, 0, q0, lane, [&](int mt, f32x4 d) {
#pragma unroll
        for (int r = 0; r < 4; ++r) { s[mt][r] = sigm(d[r]); dg[mt][r] = 0.f; }
      });
    }
    __syncthreads();
    stage_tiles<NU>(sU, (const bf16x8*)a.up[l]);
    stage_tiles<NVT>(sV, (const bf16x8*)a.vwt[l]);
    stage_tiles<D::NVW>(sP, (const bf16x8*)a.vw[l]);
    lds_dma_sync();
    if (act) {
      for (int m = 0; m < 2 * l + 1; ++m) {
        const int lm = l * l + m;
        // both rows' loads issued before the first product, so their latencies overlap
        bf16x8 ql[KCQ];
        qload(lm, ql);
        f32x4 hb[MTC];
        hbar_row(lm, hb);
        // z_lm consumed tile by tile: dgate += hbar z, zbar_lm = hbar sigmoid(gate) (in hb)
        lds_rows<MTC, KCQ>(sV, KCQ, 0, ql, lane, [&](int mt, f32x4 d) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            dg[mt][r] += hb[mt][r] * d[r];
            hb[mt][r] *= s[mt][r];
          }
        });
        bf16x8 zb[KCC];
#pragma unroll
        for (int kc = 0; kc < KCC; ++kc) zb[kc] = tiles_to_op(hb, kc);
        __bf16* dst = pdst(lm);
        PairStore ps;
        lds_rows<MTP, KCC>(sP, KCC, 0, zb, lane, [&](int mt, f32x4 d) {
          if (av) ps.put(mt, d, dst);
        });
      }
      // zbar of the gate block l: sum_m hbar_lm z_lm * sigmoid'
#pragma unroll
      for (int mt = 0; mt < MTC; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) dg[mt][r] *= s[mt][r] * (1.f - s[mt][r]);
#pragma unroll
      for (int kc = 0; kc < KCC; ++kc) z0b[l * KCC + kc] = tiles_to_op(dg, kc);
    }
  }
  // P_0 = zbar_0 (VW_0)^T in two halves of its row tiles
  __bf16* dst = pdst(0);
  PairStore ps;
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) {
    __syncthreads();
    stage_tiles<D::NP0>(sW, (const bf16x8*)a.vw[0] + (size_t)hf * D::NP0 * 64);
    lds_dma_sync();
    if (act)
      lds_rows<MTP / 2, NZC>(sW, NZC, 0, z0b, lane, [&](int mt, f32x4 d) {
        if (av) ps.put(hf * (MTP / 2) + mt, d, dst);
      });
  }
}

// The last layer's node update and its adjoint (BF16 form, only the scalar
// output live): per tile of 16 atoms, z_0 = W_down^T A (the scalar block),
// E_i = e0 + w_read . (h_0 + SiLU(z_0)), zbar_0 = w_read SiLU'(z_0) on root
// atoms, dE/dA = W_down zbar_0 written over A.  Both packings of W_down sit in
// LDS once per workgroup of 8 waves (128 atoms).
template <int C>
__global__ __launch_bounds__(64 * kN1Waves) __attribute__((amdgpu_waves_per_eu(4))) void k_nodeK(NodeKArgs a) {
  constexpr int MT = C / 16, KC = C / 32;
  __shared__ bf16x8 sDt[MT * KC * 64], sD[MT * KC * 64];
  stage_tiles<MT * KC>(sDt, (const bf16x8*)a.dt);
  stage_tiles<MT * KC>(sD, (const bf16x8*)a.d);
  lds_dma_sync();
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
  const int64_t a0 = ((int64_t)blockIdx.x * kN1Waves + (threadIdx.x >> 6)) * 16;
  if (a0 >= a.n) return;
  const bool av = a0 + n < a.n;
  const int64_t at = av ? a0 + n : a.n - 1;
  float* Ai = a.A + at * C;
  // B operand: this atom's messages, k-slot (kc, g, j) = channel 32 kc + 8 g + j
  bf16x8 ab[KC];
  if (a.msg) {
    // A_i = inv_n sum over row i's message slots, in edge order (each lane
    // sums its 8 channels of every chunk)
    float acc[KC][8];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[kc][j] = 0.f;
    const int e0 = a.row_ptr[at], e1 = av ? a.row_ptr[at + 1] : e0;
    const unsigned short* M = a.msg + 8 * g;
    auto add = [&](const uint4* u) {
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const unsigned w[4] = {u[kc].x, u[kc].y, u[kc].z, u[kc].w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          acc[kc][2 * t] += __uint_as_float(w[t] << 16);
          acc[kc][2 * t + 1] += __uint_as_float(w[t] & 0xffff0000u);
        }
      }
    };
    for (int e = e0; e < e1; ++e) {
      uint4 u0[KC];
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) u0[kc] = *(const uint4*)(M + (int64_t)e * C + 32 * kc);
      add(u0);
    }
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int j = 0; j < 8; ++j) ab[kc][j] = (__bf16)(a.inv_n * acc[kc][j]);
  } else {
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const float4 u = *(const float4*)(Ai + 32 * kc + 8 * g), v = *(const float4*)(Ai + 32 * kc + 8 * g + 4);
      const float x[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 8; ++j) ab[kc][j] = (__bf16)x[j];
    }
  }
  const bool own = a.owned_s[at] != 0;
  const float* h0 = a.h + at * (int64_t)a.nlm * C;
  double es = 0.0;
  f32x4 zb[MT];
  // D tile mt: z feature 16 mt + 4 g + r of atom n
  lds_rows<MT, KC>(sDt, KC, 0, ab, lane, [&](int mt, f32x4 d) {
    const float4 hv = *(const float4*)(h0 + 16 * mt + 4 * g);
    const float4 wv = *(const float4*)(a.w_read + 16 * mt + 4 * g);
    const float hh[4] = {hv.x, hv.y, hv.z, hv.w}, ww[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      es += (double)(hh[r] + silu(d[r])) * (double)ww[r];
      zb[mt][r] = own ? ww[r] * dsilu(d[r]) : 0.f;
    }
  });
  es += __shfl_xor(es, 16);
  es += __shfl_xor(es, 32);
  if (g == 0 && av) a.atom_e[at] = (double)a.e0[a.spec_s[at]] + es;
  bf16x8 zo[KC];
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) zo[kc] = tiles_to_op(zb, kc);
  // every lane has read its A row (or messages) above; the wave writes dE/dA over A
  lds_rows<MT, KC>(sD, KC, 0, zo, lane, [&](int mt, f32x4 d) {
    if (av) *(float4*)(Ai + 16 * mt + 4 * g) = make_float4(d[0], d[1], d[2], d[3]);
  });
}

void launch_nodeK(int C, const NodeKArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  const unsigned grid = (unsigned)((a.n + 16 * kN1Waves - 1) / (16 * kN1Waves));
  if (C == 64) k_nodeK<64><<<grid, 64 * kN1Waves, 0, s>>>(a);
  else k_nodeK<128><<<grid, 64 * kN1Waves, 0, s>>>(a);
}

template <int C, int L>
static void node1_c(bool fwd, int S, const Node1Args& a, hipStream_t s) {
  const unsigned grid = (unsigned)((a.n + 16 * kN1Waves - 1) / (16 * kN1Waves));
#define MPIP_N1(SS)                                                                 \
  if (fwd) k_node1_fwd<C, L, SS><<<grid, 64 * kN1Waves, 0, s>>>(a);                 \
  else k_node1_bwd<C, L, SS><<<grid, 64 * kN1Waves, 0, s>>>(a);
  switch (S) {
    case 1: MPIP_N1(1) break;
    case 2: MPIP_N1(2) break;
    case 3: MPIP_N1(3) break;
    default: MPIP_N1(4) break;
  }
#undef MPIP_N1
}

void launch_node1(bool fwd, int C, int L, int S, const Node1Args& a, hipStream_t s) {
  if (a.n <= 0) return;
  if (C == 64 && L == 1) node1_c<64, 1>(fwd, S, a, s);
  else if (C == 64) node1_c<64, 2>(fwd, S, a, s);
  else if (L == 1) node1_c<128, 1>(fwd, S, a, s);
  else node1_c<128, 2>(fwd, S, a, s);
}

}  // namespace mpip
