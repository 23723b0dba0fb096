// Specialised edge kernels for the first and the last message-passing layer
// (l_max <= 2, 64 or 128 channels) -- the layers of a depth-pruned model.
//
// First layer (input features depend on the sender's species only).
//   A_i[lm, c] = sum_e R_e[l, c] ht1[s_e, c] YC_e[lm] / n_avg with
//   R_e[l, c] = sum_k a2_e[k] W3[k, (l, c)], so
//   A_i[lm, c] = sum_{s,k} Q_i[lm, (s, k)] V_l[(s, k), c],
//   Q_i[lm, (s, k)] = sum_{e: s_e = s} a2_e[k] YC_e[lm],
//   V_l[(s, k), c]  = ht1[s, c] W3[k, (l, c)] / n_avg.
// The per-edge work drops to the radial MLP's hidden layers (in the BF16
// form read from the layer's radial table, edge_common.h rad_pos) plus a
// 16-edge MFMA contraction into Q; the channel dimension moves to one node
// GEMM per l.
// Its adjoint uses P_i = dA_i V^T: dE/da2_e[k] = sum_lm YC_e[lm] P_i[lm, (s_e, k)]
// and dE/dYC_e[lm] = sum_k a2_e[k] P_i[lm, (s_e, k)], both small MFMAs.
//
// Last layer (only scalars out, paths (l, l, 0)).
//   forward:  A_i[c] = sum_e sum_l R_e[l, c] <ht_j[l, :, c], YC_e[l, :]> / n_avg
//             with R in edges x channels MFMA layout (each lane: 4 edges x
//             C/16 contiguous channels), messages summed in registers.
//   adjoint a: channels x edges layout (each lane: one edge x C/4 channels):
//             dR, dE/dY, and the MLP adjoint (BF16: dE/dd from the radial
//             table's increments) fed straight from registers.
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

// four floats to a BF16 operand of the K = 16 MFMA, converted in pairs
__device__ __forceinline__ s16x4 pk4_bf16(f32x4 v) {
  typedef __attribute__((ext_vector_type(2))) float f32x2;
  typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
  const bf16x2 lo = __builtin_convertvector((f32x2){v[0], v[1]}, bf16x2);
  const bf16x2 hi = __builtin_convertvector((f32x2){v[2], v[3]}, bf16x2);
  const uint2 u = {__builtin_bit_cast(unsigned, lo), __builtin_bit_cast(unsigned, hi)};
  return __builtin_bit_cast(s16x4, u);
}

__device__ __forceinline__ f32x4 mfma_bf16_k16(s16x4 a, s16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Transposing LDS read of 16-bit data.  In each group of 16 lanes, lane m
// names 4 consecutive elements, which the group's 16 addresses take as row
// m / 4, columns 4 (m % 4) .. 4 (m % 4) + 3 of a 4 x 16 matrix T; lane i of
// the group receives column i, (T[0][i], T[1][i], T[2][i], T[3][i]).
__device__ __forceinline__ s16x4 lds_read_tr16(const void* p) {
  return __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s16x4*)p);
}

__device__ __forceinline__ bool fast_guard(const FastArgs& a) {
  return (int64_t)a.row_ptr[a.n] > a.capacity || a.status[ST_FLAGS] != 0;
}

// The couplings of the specialised layers are diagonal in m: a scalar with a
// degree-l harmonic to degree l (first layer, paths (0, l, l)) and two
// degree-l harmonics to a scalar (last layer, paths (l, l, 0)); the model is
// rejected otherwise when it is created.  Only the diagonal is used, read
// once per wave into scalar registers.
template <int L>
struct CgDiag {
  float c[(L + 1) * (L + 1)];
};
template <int L>
__device__ __forceinline__ CgDiag<L> cg_diag(const float* cg) {
  CgDiag<L> d;
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

// YC of the specialised layers' paths: YC[l^2 + m] = C[m][m] Y[l^2 + m] (diagonal of
// the coupling of path l)
template <int L>
__device__ __forceinline__ void yc_last(const CgDiag<L>& cd, const float* Y, float* yc) {
#pragma unroll
  for (int k = 0; k < (L + 1) * (L + 1); ++k) yc[k] = cd.c[k] * Y[k];
}

// adjoint of yc_last: Ybar[l^2 + m] = C[m][m] ycbar[l^2 + m]
template <int L>
__device__ __forceinline__ void yc_last_adj(const CgDiag<L>& cd, const float* ycb, float* Yb) {
#pragma unroll
  for (int k = 0; k < (L + 1) * (L + 1); ++k) Yb[k] = cd.c[k] * ycb[k];
}


// geometry backward: dE/dr_e = dbar u + (I - u u^T)/d (dP/du)^T Ybar, dbar = dE/dd
__device__ __forceinline__ float4 edge_grad_d(const Geo& geo, float dbar, const float* Yb) {
  float gu[3];
  sh_grad_contract(Yb, geo.u, gu);
  const float ud = gu[0] * geo.u[0] + gu[1] * geo.u[1] + gu[2] * geo.u[2];
  const float invd = __builtin_amdgcn_rcpf(geo.d);
  return make_float4(dbar * geo.u[0] + (gu[0] - ud * geo.u[0]) * invd, dbar * geo.u[1] + (gu[1] - ud * geo.u[1]) * invd,
                     dbar * geo.u[2] + (gu[2] - ud * geo.u[2]) * invd, 0.f);
}

// the same with dE/dd from the basis adjoint ebar
__device__ __forceinline__ float4 edge_grad(const Geo& geo, const float* ebar, const float* Yb) {
  float dbar = 0.f;
#pragma unroll
  for (int n = 0; n < kNB; ++n) dbar += ebar[n] * geo.dbasis[n];
  return edge_grad_d(geo, dbar, Yb);
}

// g_e += d (dE/dr_e)
__device__ __forceinline__ void add_grad(float4* g, int e, float4 d) {
  float4 acc = g[e];
  acc.x += d.x;
  acc.y += d.y;
  acc.z += d.z;
  g[e] = acc;
}

template <typename T, int NT>
__device__ __forceinline__ void stage_lds(T* dst, const void* src) {
  const T* s = (const T*)src;
  for (int t = threadIdx.x; t < NT; t += blockDim.x) dst[t] = s[t];
}

// ============================================================ first layer

// Workgroups of NW waves, each wave walking its own rows (row_walk).  The
// BF16 form reads the radial MLP's output from the layer's radial table
// (rad_pos); the FP32 form evaluates the MLP from row-major weight copies in
// LDS.  The per-tile harmonics and sender species are exchanged between the
// lanes of a wave through a wave-private LDS slice.
//
// Rows of Q and P: the (species s, degree-order lm) pairs, numbered
// q = lm S + s, so that Q_i[lm][s * 64 + k] = Q_i[q][k] (row q of 64 hidden
// values, contiguous).  S <= 4.
//
// Forward: Q_i[q][k] = sum_e Ysel_e[q] a2_e[k], as D tiles (hidden 16 nt +
// 4 g + r) x (q = 16 qt + lane % 16): the layer-2 activations in edges x
// features layout are directly the A operand (rows hidden, k = edges), and
// each lane stores 4 consecutive hidden values of one row q.
template <int PREC, int L, int S, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(PREC == 1 ? 3 : 1))) void k_l1_fwd(FastArgs a) {
  typedef Op<PREC> O;
  constexpr int NLM = (L + 1) * (L + 1), KQ = 64 * S, MROWS = S * NLM, MQ = (MROWS + 15) / 16;
  // FP32 form: W1, W2 as row-major copies (one copy serves both
  // orientations); the BF16 form reads the MLP's output from its radial table
  __shared__ float sR1[PREC == 0 ? 8 * 65 : 1], sR2[PREC == 0 ? 64 * 65 : 1];
  __shared__ float sY[NW][kTileE * NLM];
  __shared__ __align__(16) int sS[NW][kTileE];
  if (fast_guard(a)) return;
  const GeoK gk = geo_consts(a.rc, a.envelope_p);
  const CgDiag<L> cgd = cg_diag<L>(a.cg);
  if constexpr (PREC == 0) {
    stage_rows<8 * 65>(sR1, a.w1r);
    stage_rows<64 * 65>(sR2, a.w2r);
    __syncthreads();
  }
  const int lane = threadIdx.x & 63, g = lane >> 4, el = lane & 15, wv = threadIdx.x >> 6;
  float* syc = sY[wv];
  int* ssp = sS[wv];
  // the Q rows of this lane's columns: q = 16 qt + el = lm S + s
  int qlm[MQ], qs[MQ];
#pragma unroll
  for (int qt = 0; qt < MQ; ++qt) {
    const int q = 16 * qt + el;
    qlm[qt] = q < MROWS ? q / S : 0;
    qs[qt] = q < MROWS ? q - (q / S) * S : -2;   // -2 matches no sender (invalid edges carry -1)
  }
  const RowWalk rw = row_walk<NW>(a.n);
  // BF16 form: each tile's edge vectors are requested during the tile before
  // it, and the radial-table words of its edges once they have arrived (at
  // the end of that tile): tw[r][nt] = word (interval of edge 4 g + r,
  // hidden 16 nt + el), tt[r] its tau
  RowAhead ra(rw, a.row_ptr, nullptr);
  float4 pv = make_float4(1.f, 0.f, 0.f, 0.f);
  uint32_t tw[4][4] = {};
  float tt[4] = {};
  auto fetch = [&](int e, int end) {
    if constexpr (PREC == 1) pv = e < end ? a.e_vec[e] : make_float4(1.f, 0.f, 0.f, 0.f);
  };
  auto tab_fetch = [&]() {
    if constexpr (PREC == 1) {
      const RadPos rp = rad_pos(edge_length(pv), a.rtab_scale);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ke = __shfl(rp.k, 4 * g + r);
        tt[r] = __shfl(rp.tau, 4 * g + r);
        const uint32_t* row = a.rtab + (size_t)ke * 64 + el;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) tw[r][nt] = row[16 * nt];
      }
    }
  };
  if (ra.has_row()) {
    fetch(ra.e0 + el, ra.e1);
    tab_fetch();
  }
  for (int64_t i = rw.i; i < rw.end; i += rw.step, ra.advance(a.row_ptr, nullptr)) {
    const int e0 = ra.e0, e1 = ra.e1;
    if (e0 >= e1 && ra.has_next()) {
      fetch(ra.n0 + el, ra.n1);
      tab_fetch();
    }
    f32x4 q[4][MQ];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int qt = 0; qt < MQ; ++qt) q[nt][qt] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int t0 = e0; t0 < e1; t0 += kTileE) {
      const int e = t0 + el;
      const bool valid = e < e1;
      Geo geo;
      float4 v;
      if constexpr (PREC == 1) {
        v = pv;
        if (t0 + kTileE < e1) fetch(t0 + kTileE + el, e1);
        else if (ra.has_next()) fetch(ra.n0 + el, ra.n1);
        edge_direction(v, valid, geo);
      } else {
        v = valid ? a.e_vec[e] : make_float4(1.f, 0.f, 0.f, 0.f);
        edge_geometry(v, valid, gk, geo);
      }
      if (g == 0) {
        float yc[NLM];
        yc_last<L>(cgd, geo.Y, yc);
#pragma unroll
        for (int k = 0; k < NLM; ++k) syc[el * NLM + k] = yc[k];
        ssp[el] = valid ? __float_as_int(v.w) : -1;
      }
      // the MLP's second hidden layer, edges x features: a2[nt][r] = a(edge
      // 4 g + r)[hidden 16 nt + el]
      f32x4 a2[4];
      if constexpr (PREC == 1) {
        // from the radial-table words requested a tile ahead
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int nt = 0; nt < 4; ++nt)
            a2[nt][r] = fmaf(tt[r], __uint_as_float(tw[r][nt] & 0xffff0000u), __uint_as_float(tw[r][nt] << 16));
      } else {
        // layer 1 (features x edges), layer 2 (edges x features)
        f32x4 a1[4];
        const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          f32x4 acc = z;
#pragma unroll
          for (int qq = 0; qq < 2; ++qq) acc = O::mma(sR1[(4 * qq + g) * 65 + 16 * mt + el], geo.basis[4 * qq + g], acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) a1[mt][r] = silu(acc[r]);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          f32x4 acc = z;
#pragma unroll
          for (int kc = 0; kc < O::KC64; ++kc)   // B = W2 [h1][h2 = 16 nt + el]
            acc = O::mma(O::from_tiles(a1, kc), sR2[phi_f(kc, g) * 65 + 16 * nt + el], acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) a2[nt][r] = silu(acc[r]);
        }
      }
      wave_lds_sync();
      // Q[hidden][q] += sum_e a2[e][hidden] Ysel[e][q]: A = a2 tile nt (rows
      // hidden 16 nt + el, k = edges 4 g + r), B = Ysel (k = edges 4 g + r, column q)
      const int4 sp4 = *(const int4*)(ssp + 4 * g);
      const int spr[4] = {sp4.x, sp4.y, sp4.z, sp4.w};
      // A operands of the four hidden tiles, converted in pairs once per tile
      s16x4 av[4];
      if constexpr (PREC == 1) {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) av[nt] = pk4_bf16(a2[nt]);
      }
#pragma unroll
      for (int qt = 0; qt < MQ; ++qt) {
        f32x4 ys;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float y = syc[(4 * g + r) * NLM + qlm[qt]];
          ys[r] = (spr[r] == qs[qt]) ? y : 0.f;
        }
        if constexpr (PREC == 1) {
          const s16x4 bv = pk4_bf16(ys);
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) q[nt][qt] = mfma_bf16_k16(av[nt], bv, q[nt][qt]);
        } else {
#pragma unroll
          for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) q[nt][qt] = mfma_f32(a2[nt][r], ys[r], q[nt][qt]);
        }
      }
      tab_fetch();
      wave_lds_sync();
    }
    // row q = 16 qt + el, hidden 16 nt + 4 g + r: four consecutive values per store
#pragma unroll
    for (int qt = 0; qt < MQ; ++qt) {
      const int qq = 16 * qt + el;
      if (qq < MROWS) {
        const int64_t o = (int64_t)i * NLM * KQ + (int64_t)qq * 64 + 4 * g;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          if constexpr (PREC == 1) {
            *(s16x4*)((__bf16*)a.Q + o + 16 * nt) = pk4_bf16(q[nt][qt]);
          } else {
            *(float4*)(a.Q + o + 16 * nt) = make_float4(q[nt][qt][0], q[nt][qt][1], q[nt][qt][2], q[nt][qt][3]);
          }
        }
      }
    }
  }
}

// Adjoint.  dE/da2_e[k] = sum_q P_i[q][k] Ysel_e[q] and dE/dYC_e[lm] =
// sum_k P_i[(lm, s_e)][k] a2_e[k], both on MFMA with P_i as the A operand:
//   pa (rows hidden 16 mt + lane % 16, k-slot (g, j) of chunk c = species
//      4 (c / KCL) + g, lm = 8 (c % KCL) + j), against Ysel with the same
//      slots, whose lm is known at compile time;
//   pb (rows q = 16 mq + lane % 16, k = hidden in the operand permutation of
//      the MLP), against the activations a2.
// The row's P (BF16) is staged in a wave-private LDS slice, the next row's
// loaded into registers while this row's tiles run.
template <int PREC, int L, int S, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(PREC == 1 ? 3 : 1))) void k_l1_bwd(FastArgs a) {
  typedef Op<PREC> O;
  constexpr int NLM = (L + 1) * (L + 1), KQ = 64 * S, MROWS = S * NLM, MQ = (MROWS + 15) / 16;
  constexpr int KCL = (PREC == 1) ? (NLM + 7) / 8 : NLM;   // chunks over lm per species group
  constexpr int KCY = ((S + 3) / 4) * KCL;                  // chunks of the (s, lm) slots
  // FP32 form: W1, W2 as row-major copies (one copy serves forward and
  // adjoint); the BF16 form takes the MLP and its derivative from the radial table
  __shared__ float sR1[PREC == 0 ? 8 * 65 : 1], sR2[PREC == 0 ? 64 * 65 : 1];
  // dE/dYC rows of the tile: row el (edge), q = 16 mq + 4 g + r stored at
  // 16 g + 4 mq + r (sy_pos), row stride 65: a D-tile store's 64 lanes meet
  // each bank twice, the fewest for 64 words
  static_assert(MQ <= 4, "dE/dYC row layout");
  constexpr int SYB = 65;
  __shared__ float sYB[NW][kTileE * SYB];
  auto sy_pos = [](int q) { return 16 * ((q & 15) >> 2) + 4 * (q >> 4) + (q & 3); };
  if (fast_guard(a)) return;
  const GeoK gk = geo_consts(a.rc, a.envelope_p);
  const CgDiag<L> cgd = cg_diag<L>(a.cg);
  if constexpr (PREC == 0) {
    stage_rows<8 * 65>(sR1, a.w1r);
    stage_rows<64 * 65>(sR2, a.w2r);
    __syncthreads();
  }
  const int lane = threadIdx.x & 63, g = lane >> 4, el = lane & 15, wv = threadIdx.x >> 6;
  float* syb = sYB[wv];
  // BF16 form: P rows staged as [q][64] (q < 16 MQ, zero past MROWS) plus
  // 4 zero rows, which the pa reads of species >= S may reach; rows padded to
  // PRS = 80 elements (40 words), so the pb reads (16 rows x 4 lane groups of
  // 8 bytes) meet each bank 4 times and the pa reads (4 rows x 16 lanes) once
  constexpr int PRS = 80, PROWS = 16 * MQ + 4;
  constexpr int PW = (PREC == 1) ? PROWS * PRS : 8;         // BF16 elements
  constexpr int NPL = (PROWS * 8 + 63) / 64;                   // 16-byte pieces per lane (8 a row)
  __shared__ uint4 sPr[NW][PW / 8];
  const unsigned short* sPw = (const unsigned short*)sPr[wv];
  constexpr int pieces = NLM * KQ / 8;
  const RowWalk rw = row_walk<NW>(a.n);
  uint4 praw[NPL];
  auto p_fetch = [&](int64_t row) {
    if constexpr (PREC == 1) {
      const uint4* src = (const uint4*)((const __bf16*)a.P + row * NLM * KQ);
#pragma unroll
      for (int q = 0; q < NPL; ++q) {
        const int pc = q * 64 + lane;
        praw[q] = (row < rw.end && pc < pieces) ? src[pc] : make_uint4(0u, 0u, 0u, 0u);
      }
    }
  };
  auto p_stage = [&]() {
    if constexpr (PREC == 1) {
#pragma unroll
      for (int q = 0; q < NPL; ++q) {
        const int pc = q * 64 + lane;
        if (pc < PROWS * 8) sPr[wv][(pc >> 3) * (PRS / 8) + (pc & 7)] = praw[q];
      }
      wave_lds_sync();
    }
  };
  p_fetch(rw.i);
  // BF16 form: each tile's edge vectors are requested during the tile before
  // it (the FP32 form, short of registers, loads them at the tile's start)
  RowAhead ra(rw, a.row_ptr, nullptr);
  float4 pv = make_float4(1.f, 0.f, 0.f, 0.f);
  auto fetch = [&](int e, int end) {
    if constexpr (PREC == 1) pv = e < end ? a.e_vec[e] : make_float4(1.f, 0.f, 0.f, 0.f);
  };
  // BF16 form: the radial-table words of the edges in pv, requested once pv
  // has arrived (at the end of the tile before)
  RadRow rn{};
  auto tab_fetch = [&]() {
    if constexpr (PREC == 1) rn = rad_load(a.rtab, rad_pos(edge_length(pv), a.rtab_scale), g);
  };
  if (ra.has_row()) {
    fetch(ra.e0 + el, ra.e1);
    tab_fetch();
  }
  for (int64_t i = rw.i; i < rw.end; i += rw.step, ra.advance(a.row_ptr, nullptr)) {
    const int e0 = ra.e0, e1 = ra.e1;
    if (e0 >= e1 && ra.has_next()) {
      fetch(ra.n0 + el, ra.n1);
      tab_fetch();
    }
    p_stage();
    p_fetch(i + rw.step);
    const float* Pi = a.P + (int64_t)i * NLM * KQ;
    typename O::T pa[4][KCY];
    typename O::T pb[MQ][O::KC64];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int c = 0; c < KCY; ++c) {
        const int sg = c / KCL, lc = c % KCL;
        if constexpr (PREC == 1) {
          // species 4 sg + g, lm = 8 lc + j, hidden 16 mt + el
          const unsigned short* src = sPw + (4 * sg + g) * PRS + 16 * mt + el;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int lm = 8 * lc + j;
            pa[mt][c][j] = lm < NLM ? __builtin_bit_cast(__bf16, src[lm * S * PRS]) : (__bf16)0.f;
          }
        } else {
          const int sp_ = 4 * sg + g;
          pa[mt][c] = sp_ < S ? Pi[lc * KQ + sp_ * 64 + 16 * mt + el] : 0.f;
        }
      }
#pragma unroll
    for (int mq = 0; mq < MQ; ++mq) {
      const int qq = 16 * mq + el;
      if constexpr (PREC == 1) {
        const unsigned short* src = sPw + qq * PRS + 4 * g;
#pragma unroll
        for (int kc = 0; kc < O::KC64; ++kc) {
          const uint2 lo = *(const uint2*)(src + 32 * kc), hi = *(const uint2*)(src + 32 * kc + 16);
          pb[mq][kc] = __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
        }
      } else {
#pragma unroll
        for (int kc = 0; kc < O::KC64; ++kc)
          pb[mq][kc] = qq < MROWS ? Pi[qq * 64 + 16 * (kc / 4) + 4 * g + (kc % 4)] : 0.f;
      }
    }
    for (int t0 = e0; t0 < e1; t0 += kTileE) {
      const int e = t0 + el;
      const bool valid = e < e1;
      Geo geo;
      float4 v;
      if constexpr (PREC == 1) {
        v = pv;
        if (t0 + kTileE < e1) fetch(t0 + kTileE + el, e1);
        else if (ra.has_next()) fetch(ra.n0 + el, ra.n1);
      } else {
        v = valid ? a.e_vec[e] : make_float4(1.f, 0.f, 0.f, 0.f);
      }
      // BF16 form: the last layer's reverse-edge gradient of this edge, requested early
      float4 gq = make_float4(0.f, 0.f, 0.f, 0.f);
      if constexpr (PREC == 1) gq = (a.g2p && lane < kTileE && valid) ? a.g2p[e] : gq;
      if constexpr (PREC == 1) edge_direction(v, valid, geo);
      else edge_geometry(v, valid, gk, geo);
      const int sp = valid ? __float_as_int(v.w) : -1;
      float yc[NLM];
      yc_last<L>(cgd, geo.Y, yc);
      // the MLP's second hidden layer a2 (BF16 form: from the radial table,
      // with the increments sl for its derivative); FP32: p1, p2 kept for the adjoint
      f32x4 p1[4], p2[4], a2[4], ab2[4];
      f32x4 sl[4];
      if constexpr (PREC == 1) {
        rad_eval(rn, a2, sl);
      } else {
        f32x4 a1[4];
        mlp_fwd_rows(geo, lane, sR1, sR2, p1, a1, p2);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) a2[mt][r] = silu(p2[mt][r]);
      }
      // Ysel operand of this lane's edge (column el): slot (g, j) of chunk c
      // is species 4 (c / KCL) + g, lm = 8 (c % KCL) + j (FP32: lm = c % KCL)
      typename O::T yb[KCY];
#pragma unroll
      for (int c = 0; c < KCY; ++c) {
        const int sg = c / KCL, lc = c % KCL;
        const bool mine = (4 * sg + g) == sp;
        if constexpr (PREC == 1) {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int lm = 8 * lc + j;
            yb[c][j] = (__bf16)((lm < NLM && mine) ? yc[lm < NLM ? lm : 0] : 0.f);
          }
        } else {
          yb[c] = mine ? yc[lc] : 0.f;
        }
      }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < KCY; ++c) acc = O::mma(pa[mt][c], yb[c], acc);
        ab2[mt] = acc;
      }
      // dE/dYC^T rows q = 16 mq + 4 g + r of edge el, to LDS
#pragma unroll
      for (int mq = 0; mq < MQ; ++mq) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < O::KC64; ++kc) acc = O::mma(pb[mq][kc], O::from_tiles(a2, kc), acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) syb[el * SYB + 16 * g + 4 * mq + r] = acc[r];
      }
      float eb[kNB];
      float dbar = 0.f;
      if constexpr (PREC == 1) {
        dbar = rad_dbar(ab2, sl, a.rtab_scale);
        tab_fetch();
      } else {
        mlp_bwd_rows(ab2, p1, p2, lane, sR1, sR2, eb);
      }
      wave_lds_sync();
      if (lane < kTileE && valid) {
        float ycb[NLM], Yb[kMaxNlm];
#pragma unroll
        for (int k = 0; k < kMaxNlm; ++k) Yb[k] = 0.f;
#pragma unroll
        for (int k = 0; k < NLM; ++k) ycb[k] = syb[el * SYB + sy_pos(k * S + sp)];
        yc_last_adj<L>(cgd, ycb, Yb);
        float4 d;
        if constexpr (PREC == 1) d = edge_grad_d(geo, dbar, Yb);
        else d = edge_grad(geo, eb, Yb);
        if (a.g2p) {
          // h_e = (this layer's dE/dr_e) - g2p[e], where g2p[e] is the last
          // layer's dE/dr of the reverse edge: then F_i = sum_e h_e - h_rev(e)
          // and the virial is -sum_e r_e (x) h_e (r_rev(e) = -r_e), so the
          // outputs gather one array through the reverse edges instead of two
          if constexpr (PREC == 0) gq = a.g2p[e];
          a.g[e] = make_float4(d.x - gq.x, d.y - gq.y, d.z - gq.z, 0.f);
        } else {
          add_grad(a.g, e, d);
        }
      }
      wave_lds_sync();
    }
  }
}

// ============================================================ last layer

// Fused adjoint of the last layer (BF16 form).  Rows i are walked as in the
// pull; every edge e = (i <- j) stands for its reverse e' = (j <- i), whose
// sender is the row's own atom (same length, unit vector -u):
//   X_e'[l, c]    = sum_m YC_e'[lm] ht_i[lm, c]
//   dR_e'[l, c]   = dA_j[c] X_e'[l, c] / n_avg                 (MLP adjoint)
//   dE/dYC_e'[lm] = sum_c ht_i[lm, c] R_e'[l, c] dA_j[c] / n_avg
//   htbar_i[lm,c] = sum_{e in row i} YC_e'[lm] R_e'[l, c] dA_j[c] / n_avg
// so the only per-edge gather is dA_j, the radial MLP runs once per edge for
// both adjoints, and dE/dr_e' goes to g[rev(e)].  Layout per chunk (channels
// 32k + 8g + q of lane group g, edge el): R and X are D tiles (channels x
// edges); X is a 16x16x16 MFMA of the row's features (transposed through a
// wave-private LDS slice, one row per row) with YC masked to degree l; the
// products with dA_j feed the MLP adjoint (B operand) and dE/dYC (an MFMA
// against the row's features); for the pull, R dA is written to a wave-private
// LDS tile (edges x 32 channels), read back transposed (lds_read_tr16: lane
// (g, n) receives channel 16 tt + n of edges 4g .. 4g + 3, the B operand of a
// 16x16x16 MFMA over edges) and summed with YC^T over the tile's edges.
#ifndef MPIP_ADJ_WPF
#define MPIP_ADJ_WPF 2
#endif
constexpr int kAdjWPF = MPIP_ADJ_WPF;   // W3 tiles in flight in the fused adjoint's chunk loop
template <int C, int L, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2))) void k_l2_adj(FastArgs a) {
  typedef Op<1> O;
  typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
  constexpr int NLM = (L + 1) * (L + 1);
  constexpr int NK = C / 32, CN = C / 16, KCC = C / 32;
  constexpr int HT = (NLM + 3) / 4 * 4;    // channel stride of the transposed row (bf16)
  constexpr int NG = HT / 4;                // lane groups holding degrees in the X operand
  __shared__ bf16x8 sW[(L + 1) * CN * 2 * 64];
  __shared__ bf16x8 sWB[(L + 1) * 4 * KCC * 64];
  __shared__ unsigned sHT[NW][C * HT / 2];
  __shared__ __align__(16) float sY[NW][kTileE * 20];
  if (fast_guard(a)) return;
  const CgDiag<L> cgd = cg_diag<L>(a.cg);
  stage_lds<bf16x8, (L + 1) * CN * 2 * 64>(sW, a.w3t);
  stage_lds<bf16x8, (L + 1) * 4 * KCC * 64>(sWB, a.w3b);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, el = lane & 15, wv = threadIdx.x >> 6;
  unsigned* sh = sHT[wv];
  float* syc = sY[wv];
  // the pull's transposition tile (edges x 32 channels, BF16, rows padded to
  // 80 bytes against bank conflicts) reuses the YC slice, which is free once
  // the pull operands ya are formed
  constexpr int TRS = 40;
  unsigned short* str = (unsigned short*)syc;
  static_assert(kTileE * 20 * 4 >= kTileE * TRS * 2, "transposition tile fits the YC slice");
  const unsigned short* ht = (const unsigned short*)a.ht;
  const RowWalk rw = row_walk<NW>(a.n);
  // each tile's senders and edge vectors are requested during the tile before it
  RowAhead rah(rw, a.row_ptr, a.row_end);
  float4 pv = make_float4(-1.f, 0.f, 0.f, 0.f);
  int pj = 0;
  auto fetch = [&](int e, int end) {
    const bool ok = e < end;
    pj = ok ? a.e_src[e] : 0;
    pv = ok ? a.e_vec[e] : make_float4(-1.f, 0.f, 0.f, 0.f);
  };
  // the radial-table words of the edges in pv, requested once pv has
  // arrived (at the end of the tile before)
  RadRow rn{};
  auto tab_fetch = [&]() { rn = rad_load(a.rtab, rad_pos(edge_length(pv), a.rtab_scale), g); };
  if (rah.has_row()) {
    fetch(rah.e0 + el, rah.e1);
    tab_fetch();
  }
  for (int64_t i = rw.i; i < rw.end; i += rw.step, rah.advance(a.row_ptr, a.row_end)) {
    const int e0 = rah.e0, e1 = rah.e1;
    if (e0 >= e1 && rah.has_next()) {
      fetch(rah.n0 + el, rah.n1);
      tab_fetch();
    }
    const unsigned short* hi = ht + (int64_t)i * NLM * C;
    // the row's features, transposed: sh[c][lm] (degrees NLM .. HT-1 zero)
#pragma unroll
    for (int p0 = 0; p0 < C / 2; p0 += 64) {
      const int p = p0 + lane;
      if (p < C / 2) {
#pragma unroll
        for (int q = 0; q < HT / 2; ++q) {
          const unsigned u0 = (2 * q < NLM) ? *(const unsigned*)(hi + (2 * q) * C + 2 * p) : 0u;
          const unsigned u1 = (2 * q + 1 < NLM) ? *(const unsigned*)(hi + (2 * q + 1) * C + 2 * p) : 0u;
          sh[(2 * p) * (HT / 2) + q] = (u0 & 0xffffu) | (u1 << 16);
          sh[(2 * p + 1) * (HT / 2) + q] = (u0 >> 16) | (u1 & 0xffff0000u);
        }
      }
    }
    wave_lds_sync();
    // X operand of M-tile mt: row el -> channel 32(mt/2) + 8(el/4) + 4(mt%2) + el%4,
    // k-slot 4g + j -> degree lm
    auto hx_op = [&](int mt) -> s16x4 {
      const int ch = 32 * (mt / 2) + 8 * (el / 4) + 4 * (mt % 2) + (el % 4);
      const uint2 v = *(const uint2*)(sh + ch * (HT / 2) + 2 * (g < NG ? g : 0));
      return (g < NG) ? __builtin_bit_cast(s16x4, v) : (s16x4){0, 0, 0, 0};
    };
    f32x4 hb[NK][2];
#pragma unroll
    for (int k = 0; k < NK; ++k) hb[k][0] = hb[k][1] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int t0 = e0; t0 < e1; t0 += kTileE) {
      const int e = t0 + el;
      const bool valid = e < e1;
      const int j = pj;
      const float4 v = pv;
      if (t0 + kTileE < e1) fetch(t0 + kTileE + el, e1);
      else if (rah.has_next()) fetch(rah.n0 + el, rah.n1);
      const float* Aj = a.Abar + (int64_t)j * C + 8 * g;
      // dA_j of the first channel chunk, requested before the geometry
      float4 an0 = *(const float4*)Aj, an1 = *(const float4*)(Aj + 4);
      wave_lds_sync();   // the previous tile's transposition reads are done
      Geo geo;
      edge_direction(make_float4(-v.x, -v.y, -v.z, 0.f), valid, geo);
      float yc[NLM];
      yc_last<L>(cgd, geo.Y, yc);
      if (g == 0) {
#pragma unroll
        for (int k = 0; k < 16; ++k) syc[el * 17 + k] = k < NLM ? yc[k] : 0.f;
      }
      // X operands: B[k-slot 4g + j][edge el] = YC[4g + j] of degree l
      s16x4 yop[L + 1];
#pragma unroll
      for (int l = 0; l <= L; ++l)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          float w = 0.f;
#pragma unroll
          for (int gg = 0; gg < 4; ++gg) {
            const int lm = 4 * gg + jj;
            if (lm >= l * l && lm < (l + 1) * (l + 1)) w = (g == gg) ? yc[lm] : w;
          }
          yop[l][jj] = bfbits(w);
        }
      // the MLP's second hidden layer from the radial table (B operand of
      // R), with the increments sl for its derivative
      f32x4 ab2[4], sl[4];
      bf16x8 bop[2];
      {
        f32x4 a2[4];
        rad_eval(rn, a2, sl);
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) bop[kc] = O::from_tiles(a2, kc);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) ab2[mt] = (f32x4){0.f, 0.f, 0.f, 0.f};
      }
      wave_lds_sync();
      // pull operands: A[lm = el][k-slot 4g + j] = YC_{e'}[lm] of edge 4g + j
      // (1/n_avg is already in dA_j: the last-layer node kernel writes dA / n_avg)
      s16x4 ya[L + 1];
      {
        float yt[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) yt[r] = syc[(4 * g + r) * 17 + el];
#pragma unroll
        for (int l = 0; l <= L; ++l) {
          const bool mine = el >= l * l && el < (l + 1) * (l + 1);
          const bf16x4 v = {(__bf16)(mine ? yt[0] : 0.f), (__bf16)(mine ? yt[1] : 0.f), (__bf16)(mine ? yt[2] : 0.f),
                            (__bf16)(mine ? yt[3] : 0.f)};
          ya[l] = __builtin_bit_cast(s16x4, v);
        }
      }
      wave_lds_sync();
      // dE/dYC accumulated per degree (rows of the other degrees are discarded)
      f32x4 dy[L + 1];
#pragma unroll
      for (int l = 0; l <= L; ++l) dy[l] = (f32x4){0.f, 0.f, 0.f, 0.f};
      bf16x8 hn = *(const bf16x8*)(hi + (int64_t)(el < NLM ? el : 0) * C + 8 * g);
      // W3 operand tiles in the order the chunk loop uses them (per chunk k
      // and degree l: the four R tiles (hh, kc), then the four MLP-adjoint
      // tiles mt), read from LDS WPF steps ahead of their MFMA through a ring
      // of registers, so the LDS latency is not paid by each MFMA
      constexpr int WPL = 8, WPK = (L + 1) * WPL, NWS = NK * WPK;
      auto wtile = [&](auto sc) -> bf16x8 {
        constexpr int st = decltype(sc)::value, k = st / WPK, l = (st % WPK) / WPL, w = st % WPL;
        if constexpr (w < 4) return sW[((l * CN + 2 * k + (w >> 1)) * 2 + (w & 1)) * 64 + lane];
        else return sWB[((l * 4 + (w - 4)) * KCC + k) * 64 + lane];
      };
      bf16x8 wring[kAdjWPF];
      static_for<kAdjWPF>([&](auto pc) { wring[decltype(pc)::value] = wtile(pc); });
      auto wtake = [&](auto sc) -> bf16x8 {
        constexpr int st = decltype(sc)::value;
        const bf16x8 w = wring[st % kAdjWPF];
        if constexpr (st + kAdjWPF < NWS) wring[st % kAdjWPF] = wtile(std::integral_constant<int, st + kAdjWPF>{});
        return w;
      };
      static_for<NK>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        __builtin_amdgcn_sched_barrier(0);
        const float ai[8] = {an0.x, an0.y, an0.z, an0.w, an1.x, an1.y, an1.z, an1.w};
        const bf16x8 hr = hn;
        const s16x4 hx[2] = {hx_op(2 * k), hx_op(2 * k + 1)};
        if constexpr (k + 1 < NK) {
          an0 = *(const float4*)(Aj + 32 * (k + 1));
          an1 = *(const float4*)(Aj + 32 * (k + 1) + 4);
          hn = *(const bf16x8*)(hi + (int64_t)(el < NLM ? el : 0) * C + 32 * (k + 1) + 8 * g);
        }
        static_for<L + 1>([&](auto lc) {
          constexpr int l = decltype(lc)::value, s0 = k * WPK + l * WPL;
          float R8[8], X8[8];
          static_for<2>([&](auto hc) {
            constexpr int hh = decltype(hc)::value;
            f32x4 d = {0.f, 0.f, 0.f, 0.f};
            d = O::mma(wtake(std::integral_constant<int, s0 + 2 * hh>{}), bop[0], d);
            d = O::mma(wtake(std::integral_constant<int, s0 + 2 * hh + 1>{}), bop[1], d);
            const f32x4 x = mfma_bf16_k16(hx[hh], yop[l], (f32x4){0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int r = 0; r < 4; ++r) { R8[4 * hh + r] = d[r]; X8[4 * hh + r] = x[r]; }
          });
          bf16x8 rb, ra;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            rb[q] = (__bf16)(ai[q] * X8[q]);
            ra[q] = (__bf16)(ai[q] * R8[q]);
          }
          // MLP adjoint through layer 3
          static_for<4>([&](auto mc) {
            constexpr int mt = decltype(mc)::value;
            ab2[mt] = O::mma(wtake(std::integral_constant<int, s0 + 4 + mt>{}), rb, ab2[mt]);
          });
          // dE/dYC: D[lm][edge] += ht_i[lm][chunk] (R dA)[chunk][edge]
          dy[l] = O::mma(hr, ra, dy[l]);
          // pull: (R dA) through the LDS tile to edges x channels, summed over
          // the tile's edges.  The LDS executes a wave's accesses in order and
          // the write and the reads may alias, so they stay in program order
          // without a wave barrier, which would also hold back the weight reads.
          *(bf16x8*)(str + el * TRS + 8 * g) = ra;
#pragma unroll
          for (int tt = 0; tt < 2; ++tt) {
            const s16x4 tr = lds_read_tr16(str + (4 * g + el / 4) * TRS + 16 * tt + 4 * (el % 4));
            hb[k][tt] = mfma_bf16_k16(ya[l], tr, hb[k][tt]);
          }
        });
      });
      __builtin_amdgcn_sched_barrier(0);
      // dE/dYC of edge el: rows 4g + r live in lane el + 16 g
      float ycb[NLM];
#pragma unroll
      for (int lm = 0; lm < NLM; ++lm) {
        const int l = lm < 1 ? 0 : (lm < 4 ? 1 : (lm < 9 ? 2 : 3));
        ycb[lm] = __shfl(dy[l][lm % 4], el + 16 * (lm / 4));
      }
      const float dbar = rad_dbar(ab2, sl, a.rtab_scale);
      tab_fetch();
      if (lane < kTileE && valid) {
        float Yb[kMaxNlm];
#pragma unroll
        for (int k = 0; k < kMaxNlm; ++k) Yb[k] = 0.f;
        yc_last_adj<L>(cgd, ycb, Yb);
        if (a.g2p) {
          // dE/dr of the reverse edge, kept in this edge's slot (written once, coalesced)
          a.g2p[e] = edge_grad_d(geo, dbar, Yb);
        } else {
          const int rv = a.e_rev[e];
          if (rv >= 0) add_grad(a.g, rv, edge_grad_d(geo, dbar, Yb));
        }
      }
    }
    // htbar_i: D rows lm = 4g + r, column el of half tt = channel 32k + 16 tt + el
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lm = 4 * g + r;
      if (lm < NLM) {
        const int64_t o = ((int64_t)i * NLM + lm) * C + el;
#pragma unroll
        for (int k = 0; k < NK; ++k)
#pragma unroll
          for (int tt = 0; tt < 2; ++tt) {
            if (a.htbar_bf16) ((short*)a.htbar)[o + 32 * k + 16 * tt] = bfbits(hb[k][tt][r]);
            else a.htbar[o + 32 * k + 16 * tt] = hb[k][tt][r];
          }
      }
    }
    wave_lds_sync();
  }
}

// Forward of the last layer (BF16 form), sender side.  Rows j are walked as
// in the fused adjoint; each edge e' = (j <- i) of row j stands for its
// reverse e = (i <- j), whose sender is the row's own atom, and its message
//   m_e[c] = sum_l R_e[l, c] X_e[l, c],  X_e[l, c] = sum_m YC_e[lm] ht_j[lm, c]
// (X a 16x16x16 MFMA of the row's transposed features, as in the adjoint) is
// written in BF16 to the receiver-side slot M[rev(e')] in row i of the CSR.
// A_i = sum_{e in row i} m_e / n_avg is then a contiguous segmented sum.
template <int C, int L, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW / 4))) void k_l2_msg(FastArgs a) {
  typedef Op<1> O;
  constexpr int NLM = (L + 1) * (L + 1);
  constexpr int NK = C / 32, CN = C / 16;
  constexpr int HT = (NLM + 3) / 4 * 4, NG = HT / 4;
  __shared__ bf16x8 sW[(L + 1) * CN * 2 * 64];
  __shared__ unsigned sHT[NW][2][C * HT / 2];
  if (fast_guard(a)) return;
  const CgDiag<L> cgd = cg_diag<L>(a.cg);
  stage_lds<bf16x8, (L + 1) * CN * 2 * 64>(sW, a.w3t);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, el = lane & 15, wv = threadIdx.x >> 6;
  const unsigned short* ht = (const unsigned short*)a.ht;
  unsigned short* M = (unsigned short*)a.msg;
  const RowWalk rw = row_walk<NW>(a.n);
  auto rbeg = [&](int64_t r) { return a.row_ptr[r]; };
  auto rend = [&](int64_t r) { return a.row_end ? a.row_end[r] : a.row_ptr[r + 1]; };
  // a row's features, transposed into slot sl: sh[c][lm] (degrees NLM .. HT-1 zero)
  auto stage = [&](int sl, int64_t r) {
    unsigned* sh = sHT[wv][sl];
    const unsigned short* hr = ht + r * NLM * C;
#pragma unroll
    for (int p0 = 0; p0 < C / 2; p0 += 64) {
      const int p = p0 + lane;
      if (p < C / 2) {
#pragma unroll
        for (int q = 0; q < HT / 2; ++q) {
          const unsigned u0 = (2 * q < NLM) ? *(const unsigned*)(hr + (2 * q) * C + 2 * p) : 0u;
          const unsigned u1 = (2 * q + 1 < NLM) ? *(const unsigned*)(hr + (2 * q + 1) * C + 2 * p) : 0u;
          sh[(2 * p) * (HT / 2) + q] = (u0 & 0xffffu) | (u1 << 16);
          sh[(2 * p + 1) * (HT / 2) + q] = (u0 >> 16) | (u1 & 0xffff0000u);
        }
      }
    }
  };
  // X operand of M-tile mt from slot sl: row el -> channel 32(mt/2) + 8(el/4) + 4(mt%2) + el%4,
  // k-slot 4g + j -> degree lm
  auto hx_op = [&](int sl, int mt) -> s16x4 {
    const unsigned* sh = sHT[wv][sl];
    const int ch = 32 * (mt / 2) + 8 * (el / 4) + 4 * (mt % 2) + (el % 4);
    const uint2 v = *(const uint2*)(sh + ch * (HT / 2) + 2 * (g < NG ? g : 0));
    return (g < NG) ? __builtin_bit_cast(s16x4, v) : (s16x4){0, 0, 0, 0};
  };
  // Tiles are packed across rows: a tile takes the rest of the current row A
  // and, when that is shorter than 16 edges, the first edges of the wave's
  // next non-empty row B (features in the other slot), so partial tiles occur
  // only at the end of the walk.  X of a packed tile is two MFMAs, each row's
  // features against the YC columns of its own edges.
  int64_t ia = rw.i;
  int pa = 0, ea = 0, sa = 0;
  auto next_row = [&](int64_t r, int& b0, int& b1) -> int64_t {
    for (; r < rw.end; r += rw.step) {
      b0 = rbeg(r);
      b1 = rend(r);
      if (b0 < b1) return r;
    }
    return rw.end;
  };
  ia = next_row(ia, pa, ea);
  if (ia < rw.end) stage(sa, ia);
  wave_lds_sync();
  while (ia < rw.end) {
    const int nA = min(kTileE, ea - pa);
    int64_t ib = rw.end;
    int b0 = 0, b1 = 0, nB = 0;
    if (nA < kTileE) {
      ib = next_row(ia + rw.step, b0, b1);
      if (ib < rw.end) {
        nB = min(kTileE - nA, b1 - b0);
        stage(sa ^ 1, ib);
        wave_lds_sync();
      }
    }
    const bool inA = el < nA;
    const bool valid = el < nA + nB;
    const int e = inA ? pa + el : b0 + (el - nA);
    const int rv = valid ? a.e_rev[e] : -1;
    const float4 v = valid ? a.e_vec[e] : make_float4(-1.f, 0.f, 0.f, 0.f);
    Geo geo;
    edge_direction(make_float4(-v.x, -v.y, -v.z, 0.f), valid, geo);
    float yc[NLM];
    yc_last<L>(cgd, geo.Y, yc);
    // YC operands of degree l, split by the row of the lane's edge
    s16x4 yopA[L + 1], yopB[L + 1];
#pragma unroll
    for (int l = 0; l <= L; ++l)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        float w = 0.f;
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) {
          const int lm = 4 * gg + jj;
          if (lm >= l * l && lm < (l + 1) * (l + 1)) w = (g == gg) ? yc[lm] : w;
        }
        yopA[l][jj] = bfbits(inA ? w : 0.f);
        yopB[l][jj] = bfbits(inA ? 0.f : w);
      }
    // the MLP's second hidden layer from the radial table (B operand of R)
    bf16x8 bop[2];
    {
      f32x4 a2[4];
      rad_tiles(a.rtab, rad_pos(geo.d, a.rtab_scale), g, a2, nullptr);
#pragma unroll
      for (int kc = 0; kc < 2; ++kc) bop[kc] = O::from_tiles(a2, kc);
    }
    unsigned short* dst = M + (int64_t)(rv < 0 ? 0 : rv) * C + 8 * g;
    const bool packed = nB > 0;
    static_for<NK>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      __builtin_amdgcn_sched_barrier(0);
      const s16x4 hx[2] = {hx_op(sa, 2 * k), hx_op(sa, 2 * k + 1)};
      s16x4 hy[2] = {hx[0], hx[1]};
      if (packed) { hy[0] = hx_op(sa ^ 1, 2 * k); hy[1] = hx_op(sa ^ 1, 2 * k + 1); }
      float m8[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) m8[q] = 0.f;
#pragma unroll
      for (int l = 0; l <= L; ++l) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kc = 0; kc < 2; ++kc) d = O::mma(sW[((l * CN + 2 * k + hh) * 2 + kc) * 64 + lane], bop[kc], d);
          f32x4 x = mfma_bf16_k16(hx[hh], yopA[l], (f32x4){0.f, 0.f, 0.f, 0.f});
          if (packed) x = mfma_bf16_k16(hy[hh], yopB[l], x);
#pragma unroll
          for (int r = 0; r < 4; ++r) m8[4 * hh + r] += d[r] * x[r];
        }
      }
      typedef __attribute__((ext_vector_type(8))) float f32x8;
      f32x8 mv;
#pragma unroll
      for (int q = 0; q < 8; ++q) mv[q] = m8[q];
      if (rv >= 0) *(bf16x8*)(dst + 32 * k) = __builtin_convertvector(mv, bf16x8);
    });
    __builtin_amdgcn_sched_barrier(0);
    wave_lds_sync();   // this tile's reads of the slots are done before either is restaged
    if (packed) {
      // row A is done; row B's rest becomes the current row
      ia = ib;
      pa = b0 + nB;
      ea = b1;
      sa ^= 1;
      if (pa >= ea) {   // row B ended inside the tile too
        ia = next_row(ia + rw.step, pa, ea);
        if (ia < rw.end) { stage(sa, ia); wave_lds_sync(); }
      }
    } else if (nA < kTileE) {
      ia = rw.end;   // the last row of the walk, partial tile
    } else {
      pa += kTileE;
      if (pa >= ea) {
        ia = next_row(ia + rw.step, pa, ea);
        if (ia < rw.end) { stage(sa, ia); wave_lds_sync(); }
      }
    }
  }
}

// A_i[c] = sum_{e in row i} M[e][c] / n_avg: one wave per row, C/8 lanes per
// edge (8 channels each), 64/(C/8) edges per load, partial sums combined
// across the lane groups at the end.
template <int C>
__global__ __launch_bounds__(256) void k_l2_msum(FastArgs a) {
  constexpr int LPE = C / 8, EPI = 64 / LPE;
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (fast_guard(a) || i >= a.n) return;
  const int lane = threadIdx.x & 63, s = lane / LPE, c8 = lane % LPE;
  const int e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
  const unsigned short* M = (const unsigned short*)a.msg + 8 * c8;
  float acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.f;
  int e = e0 + s;
  for (; e + 3 * EPI < e1; e += 4 * EPI) {
    uint4 u[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) u[b] = *(const uint4*)(M + (int64_t)(e + b * EPI) * C);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const unsigned w[4] = {u[b].x, u[b].y, u[b].z, u[b].w};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        acc[2 * t] += __uint_as_float(w[t] << 16);
        acc[2 * t + 1] += __uint_as_float(w[t] & 0xffff0000u);
      }
    }
  }
  for (; e < e1; e += EPI) {
    const uint4 u = *(const uint4*)(M + (int64_t)e * C);
    const unsigned w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[2 * t] += __uint_as_float(w[t] << 16);
      acc[2 * t + 1] += __uint_as_float(w[t] & 0xffff0000u);
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int o = LPE; o < 64; o <<= 1) acc[q] += __shfl_xor(acc[q], o);
  if (s == 0) {
    float* dst = a.A + i * C + 8 * c8;
    *(float4*)dst = make_float4(a.inv_n * acc[0], a.inv_n * acc[1], a.inv_n * acc[2], a.inv_n * acc[3]);
    *(float4*)(dst + 4) = make_float4(a.inv_n * acc[4], a.inv_n * acc[5], a.inv_n * acc[6], a.inv_n * acc[7]);
  }
}

// ============================================================ dispatch


// persistent grids: a multiple of 8 workgroups (one row range per XCD), at
// most `per_xcd` workgroups per XCD and none without rows
static int l2_grid(int64_t n, int nw, int per_xcd) {
  const int64_t need = (n / 8 + nw - 1) / nw;
  const int64_t per = need < 1 ? 1 : (need < per_xcd ? need : per_xcd);
  return (int)(8 * per);
}

template <int PREC, int L>
static void l1_launch(bool fwd, int S, const FastArgs& a, hipStream_t s) {
  // 4 waves per workgroup; forward 4 waves per SIMD, adjoint 3 (BF16 form,
  // whose radial table leaves the tile's registers within 168 VGPRs)
  constexpr int NW = 4;
  const int gf = l2_grid(a.n, NW, 128), gb = l2_grid(a.n, NW, PREC == 1 ? 96 : 128);
#define MPIP_L1(SS)                                                        \
  if (fwd) k_l1_fwd<PREC, L, SS, NW><<<gf, 64 * NW, 0, s>>>(a);              \
  else k_l1_bwd<PREC, L, SS, NW><<<gb, 64 * NW, 0, s>>>(a);
  switch (S) {
    case 1: MPIP_L1(1) break;
    case 2: MPIP_L1(2) break;
    case 3: MPIP_L1(3) break;
    default: MPIP_L1(4) break;
  }
#undef MPIP_L1
}

// species-factorised first layer: n_species <= 4 (the engine checks)
void launch_l1(int prec, int L, bool fwd, const FastArgs& a, hipStream_t s) {
  if (prec == MPIP_BF16_MIXED) {
    if (L == 1) l1_launch<1, 1>(fwd, a.n_species, a, s); else l1_launch<1, 2>(fwd, a.n_species, a, s);
  } else {
    if (L == 1) l1_launch<0, 1>(fwd, a.n_species, a, s); else l1_launch<0, 2>(fwd, a.n_species, a, s);
  }
}

// BF16 form, sender side: which = 3 the fused adjoint (one workgroup of 8
// waves per CU: W3 in both packings and the MLP weights fill the LDS), 4 the
// messages (16 waves, 4 per SIMD sharing the LDS weights), 5 their sum
template <int C, int L>
static void l2_launch(int which, const FastArgs& a, hipStream_t s) {
  if (which == 3) k_l2_adj<C, L, 8><<<l2_grid(a.n, 8, 32), 64 * 8, 0, s>>>(a);
  else if (which == 4) k_l2_msg<C, L, 16><<<l2_grid(a.n, 16, C == 128 ? 32 : 64), 64 * 16, 0, s>>>(a);
  else k_l2_msum<C><<<(unsigned)((a.n + 3) / 4), 256, 0, s>>>(a);
}

void launch_l2(int prec, int C, int L, int which, const FastArgs& a, hipStream_t s) {
  (void)prec;   // BF16 form only (the FP32 form: launch_l2_32)
  if (C == 64 && L == 1) l2_launch<64, 1>(which, a, s);
  else if (C == 64 && L == 2) l2_launch<64, 2>(which, a, s);
  else if (C == 128 && L == 1) l2_launch<128, 1>(which, a, s);
  else l2_launch<128, 2>(which, a, s);
}

}  // namespace mpip
