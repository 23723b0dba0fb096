// Fused per-layer edge kernels: edge geometry, radial basis, real spherical
// harmonics, the radial MLP on MFMA, the coupling-tensor product on VALU and
// the segmented sum onto the receiving atom; and the hand-written adjoint of
// all of it (edge intermediates recomputed, never stored).
//
// One 64-lane wavefront owns one receiver row of the receiver-sorted CSR at a
// time and walks its edges in tiles of 16.  Per tile:
//   * every lane evaluates the geometry of edge (lane % 16) (4x redundant,
//     which lets each lane feed its own MFMA operand slots);
//   * radial MLP layers 1-2 run as features x edges MFMA products so that
//     each product's output registers are directly the next one's operand;
//   * layer 3 runs per coupling path as edges x channels products; the
//     result R_p[16][C] is staged in LDS and read back channel-per-lane;
//   * the tensor product accumulates the row's messages in registers, so the
//     segmented sum needs no atomics and is deterministic.
// The adjoint recomputes the same tile, forms dE/dR_p in LDS, feeds it to
// the transposed MLP products, and pulls the sender-side feature adjoint
// through the reverse edge: for e = (i, j, S) the reverse edge has the same
// length and Y_l(-u) = (-1)^l Y_l(u), so the contribution of atom i as a
// sender is computed while walking row i.
#include "edge_common.h"

namespace mpip {

// ------------------------------------------------------------ forward

// Weights and coupling coefficients are the same for every tile; left
// visible, their loads (the radial MLP and W3 of every path: hundreds of
// registers at l_max = 2) are hoisted ahead of the row loop and held there,
// which spills.  Hiding the pointers from the optimiser once per tile keeps
// each load next to its use, served from cache.
template <class T>
__device__ __forceinline__ T* opaque_ptr(T* p) {
  asm volatile("" : "+s"(p));
  return p;
}

template <int PREC, int C, int L, int KIND>
__global__ __launch_bounds__(64) void k_edge_fwd(EdgeArgs a) {
  typedef PathList<L, KIND> PL;
  constexpr int NP = PL::count();
  constexpr int NIN = PL::nin(), NOUT = PL::nout(), NYC = PL::nyc();
  constexpr int NLM = (L + 1) * (L + 1);
  // BF16 form: 16 lanes per edge group, 4 edges of the tile in flight, each
  // lane holding C/16 channels (16 lanes read 64 contiguous bytes of a
  // sender's row); the FP32 form (more registers per channel) keeps one or
  // two edges at a time
  constexpr int CW = PREC == 1 ? 16 : (C < 64 ? C : 64);   // lanes per edge group
  constexpr int CPL = C / CW;              // channels per lane
  constexpr int EPL = 64 / CW;             // edge groups
  constexpr int RS = C + 1;
  constexpr bool SPECIES_IN = (KIND == KIND_ONLY || KIND == KIND_FIRST);
  __shared__ float sR[kTileE * RS];
  __shared__ float syc[kTileE * NYC];
  __shared__ int sj[kTileE];
  if (edges_total(a) > a.capacity || a.status[ST_FLAGS] != 0) return;
  const GeoK gk = geo_consts(a.rc, a.envelope_p);
  const int lane = threadIdx.x;
  const int eg = lane / CW, cl = lane % CW;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    const int e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
    float acc[NOUT][CPL];
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
      for (int k = 0; k < CPL; ++k) acc[o][k] = 0.f;
    for (int t0 = e0; t0 < e1; t0 += kTileE) {
      const int el = lane & 15;
      const int e = t0 + el;
      const bool valid = e < e1;
      Geo geo;
      float4 v = valid ? a.e_vec[e] : make_float4(1.f, 0.f, 0.f, 0.f);
      edge_geometry(v, valid, gk, geo);
      if (lane < kTileE) {
        sj[el] = valid ? (SPECIES_IN ? __float_as_int(v.w) : a.e_src[e]) : -1;
        // YC[p][m1][m3] = sum_m2 C_p[m1][m2][m3] Y[l2 m2]
        static_for<NP>([&](auto PI) {
          constexpr int pi = decltype(PI)::value;
          constexpr P3 pp = PL::get(pi);
          constexpr int n1 = 2 * pp.l1 + 1, n2 = 2 * pp.l2 + 1, n3 = 2 * pp.l3 + 1;
          const float* cg = opaque_ptr(a.cg + PL::cg_off(pi));
#pragma unroll
          for (int m1 = 0; m1 < n1; ++m1)
            for (int m3 = 0; m3 < n3; ++m3) {
              float s = 0.f;
              for (int m2 = 0; m2 < n2; ++m2) s += cg[(m1 * n2 + m2) * n3 + m3] * geo.Y[pp.l2 * pp.l2 + m2];
              syc[el * NYC + PL::yc_off(pi) + m1 * n3 + m3] = s;
            }
        });
      }
      f32x4 p1[4], p2[4], a2[4];
      const void* w3f = opaque_ptr(a.w3f);
      mlp_forward<PREC>(geo, lane, opaque_ptr(a.w1a), opaque_ptr(a.w2a), p1, p2);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) a2[mt][r] = silu(p2[mt][r]);
      static_for<NP>([&](auto PI) {
        constexpr int pi = decltype(PI)::value;
        constexpr P3 pp = PL::get(pi);
        constexpr int n1 = 2 * pp.l1 + 1, n3 = 2 * pp.l3 + 1;
        __syncthreads();
        radial_out<PREC, C>(a2, lane, w3f, pi, sR, RS);
        __syncthreads();
        for (int ee = eg; ee < kTileE; ee += EPL) {
          if (t0 + ee >= e1) break;
          const int j = sj[ee];
          const float* yc = syc + ee * NYC + PL::yc_off(pi);
#pragma unroll
          for (int k = 0; k < CPL; ++k) {
            const int c = cl + k * CW;
            const float R = sR[ee * RS + c];
            float hj[5];
            for (int m1 = 0; m1 < n1; ++m1)
              hj[m1] = SPECIES_IN ? a.ht[(int64_t)j * C + c]
                                  : a.ht[((int64_t)j * NLM + pp.l1 * pp.l1 + m1) * C + c];
            for (int m3 = 0; m3 < n3; ++m3) {
              float s = 0.f;
              for (int m1 = 0; m1 < n1; ++m1) s += yc[m1 * n3 + m3] * hj[m1];
              const int o = (NOUT == 1) ? 0 : pp.l3 * pp.l3 + m3;
              acc[o][k] += R * s;
            }
          }
        }
      });
      __syncthreads();
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        float vv = acc[o][k];
#pragma unroll
        for (int off = 32; off >= CW; off >>= 1) vv += __shfl_xor(vv, off);
        if (eg == 0) a.A[((int64_t)i * NOUT + o) * C + cl + k * CW] = a.inv_n * vv;
      }
  }
}

// ------------------------------------------------------------ backward

// Paths [P0, P1) of the layer's path list (sorted by input degree l1), one
// launch per range in increasing order.  All paths of a middle layer in one
// kernel need more registers than a wave has (about 40 per path stay live),
// so the launches hand the two per-edge sums over paths (the MLP adjoint's
// input and dE/dY) on through a.part, and the last launch finishes the edge
// gradient (FIN; it may have no paths of its own).  A launch writes the
// htbar blocks of its paths' degrees, adding to a block an earlier launch
// began.  Default: all paths in one launch.
template <int PREC, int C, int L, int KIND, bool HTBAR, int P0 = 0, int P1 = 64, bool FIN = true>
__global__ __launch_bounds__(64) void k_edge_bwd(EdgeArgs a) {
  typedef PathList<L, KIND> PL;
  typedef Op<PREC> O;
  constexpr int NP = PL::count();
  constexpr int NIN = PL::nin(), NOUT = PL::nout(), NYC = PL::nyc();
  constexpr int NLM = (L + 1) * (L + 1);
  constexpr int CW = C < 64 ? C : 64;
  constexpr int CPL = C / CW;
  constexpr int EPL = 64 / CW;
  constexpr int RS = C + 1;
  constexpr bool SPECIES_IN = (KIND == KIND_ONLY || KIND == KIND_FIRST);
  constexpr int PE = P1 < NP ? P1 : NP;
  constexpr bool FROM_PART = P0 > 0, TO_PART = !FIN;
  // first path of each input degree: a launch starting after it adds to its block
  constexpr auto first_of = [](int l1) {
    for (int k = 0; k < PL::count(); ++k)
      if (PL::get(k).l1 == l1) return k;
    return PL::count();
  };
  __shared__ float sR[kTileE * RS];
  __shared__ float sRb[kTileE * RS];
  __shared__ float syc[kTileE * NYC];
  __shared__ float sAi[NOUT * C];
  __shared__ float seb[kTileE * kNB];
  __shared__ int sj[kTileE];
  if (edges_total(a) > a.capacity || a.status[ST_FLAGS] != 0) return;
  const GeoK gk = geo_consts(a.rc, a.envelope_p);
  const int lane = threadIdx.x;
  const int eg = lane / CW, cl = lane % CW;
  const int g = lane >> 4, el = lane & 15;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    const int e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];
    __syncthreads();
    for (int q = lane; q < NOUT * C; q += 64) sAi[q] = a.inv_n * a.Abar[(int64_t)i * NOUT * C + q];
    float Ai[NOUT][CPL];
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
      for (int k = 0; k < CPL; ++k) Ai[o][k] = a.inv_n * a.Abar[((int64_t)i * NOUT + o) * C + cl + k * CW];
    float hb[HTBAR ? NIN : 1][CPL];
#pragma unroll
    for (int o = 0; o < (HTBAR ? NIN : 1); ++o)
#pragma unroll
      for (int k = 0; k < CPL; ++k) hb[o][k] = 0.f;
    for (int t0 = e0; t0 < e1; t0 += kTileE) {
      const int e = t0 + el;
      const bool valid = e < e1;
      Geo geo;
      float4 v = valid ? a.e_vec[e] : make_float4(1.f, 0.f, 0.f, 0.f);
      edge_geometry(v, valid, gk, geo);
      const int jme = valid ? (SPECIES_IN ? __float_as_int(v.w) : a.e_src[e]) : -1;
      __syncthreads();
      if (lane < kTileE) {
        sj[el] = jme;
        static_for<NP>([&](auto PI) {
          constexpr int pi = decltype(PI)::value;
          constexpr P3 pp = PL::get(pi);
          if constexpr (pi < P0 || pi >= PE) return;
          constexpr int n1 = 2 * pp.l1 + 1, n2 = 2 * pp.l2 + 1, n3 = 2 * pp.l3 + 1;
          const float* cg = opaque_ptr(a.cg + PL::cg_off(pi));
#pragma unroll
          for (int m1 = 0; m1 < n1; ++m1)
            for (int m3 = 0; m3 < n3; ++m3) {
              float s = 0.f;
              for (int m2 = 0; m2 < n2; ++m2) s += cg[(m1 * n2 + m2) * n3 + m3] * geo.Y[pp.l2 * pp.l2 + m2];
              syc[el * NYC + PL::yc_off(pi) + m1 * n3 + m3] = s;
            }
        });
      }
      f32x4 p1[4], p2[4], a2[4], ab2[4];
      const void* w3f = opaque_ptr(a.w3f);
      const void* w3b = opaque_ptr(a.w3b);
      mlp_forward<PREC>(geo, lane, opaque_ptr(a.w1a), opaque_ptr(a.w2a), p1, p2);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) { a2[mt][r] = silu(p2[mt][r]); ab2[mt][r] = 0.f; }
      float Ybar[kMaxNlm];
#pragma unroll
      for (int k = 0; k < kMaxNlm; ++k) Ybar[k] = 0.f;
      // the sums over the earlier launches' paths (edge el; ab2 row 16 mt + 4 g + r)
      float* pe = (FROM_PART || TO_PART) ? a.part + (int64_t)(valid ? e : 0) * kPartStride : nullptr;
      if constexpr (FROM_PART) {
        if (valid) {
#pragma unroll
          for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) ab2[mt][r] = pe[16 * mt + 4 * g + r];
#pragma unroll
          for (int k = 0; k < NLM; ++k) Ybar[k] = pe[64 + k];
        }
      }
      static_for<NP>([&](auto PI) {
        constexpr int pi = decltype(PI)::value;
        constexpr P3 pp = PL::get(pi);
        if constexpr (pi < P0 || pi >= PE) return;
        constexpr int n1 = 2 * pp.l1 + 1, n2 = 2 * pp.l2 + 1, n3 = 2 * pp.l3 + 1;
        constexpr int ob = (NOUT == 1) ? 0 : pp.l3 * pp.l3;
        constexpr float sgn = (pp.l2 & 1) ? -1.f : 1.f;
        // one path at a time: interleaving the unrolled paths spills
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
        radial_out<PREC, C>(a2, lane, w3f, pi, sR, RS);
        __syncthreads();
        // pass A: lanes own channels, walk the edges (rolled: unrolled, the
        // loads of all 16 edges are hoisted and the registers spill)
#pragma unroll 1
        for (int ee = eg; ee < kTileE; ee += EPL) {
          const bool ok = (t0 + ee) < e1;
          const int j = sj[ee];
          const float* yc = syc + ee * NYC + PL::yc_off(pi);
#pragma unroll
          for (int k = 0; k < CPL; ++k) {
            const int c = cl + k * CW;
            float rb = 0.f;
            if (ok) {
              const float R = sR[ee * RS + c];
              float hj[5], Aj[5];
              for (int m1 = 0; m1 < n1; ++m1)
                hj[m1] = SPECIES_IN ? a.ht[(int64_t)j * C + c]
                                    : a.ht[((int64_t)j * NLM + pp.l1 * pp.l1 + m1) * C + c];
              if constexpr (HTBAR) {
                for (int m3 = 0; m3 < n3; ++m3)
                  Aj[m3] = a.inv_n * a.Abar[((int64_t)j * NOUT + ob + m3) * C + c];
              }
              for (int m1 = 0; m1 < n1; ++m1) {
                float T = 0.f, U = 0.f;
                for (int m3 = 0; m3 < n3; ++m3) {
                  T += yc[m1 * n3 + m3] * Ai[ob + m3][k];
                  if constexpr (HTBAR) U += yc[m1 * n3 + m3] * Aj[m3];
                }
                rb += T * hj[m1];
                if constexpr (HTBAR) hb[pp.l1 * pp.l1 + m1][k] += sgn * R * U;
              }
            }
            sRb[ee * RS + c] = rb;
          }
        }
        // pass B: lanes own (edge el, quarter g of every 16 channels); dE/dY
        // of the edge.  Lane g takes channels 16 q + 4 g .. + 3, so the four
        // lanes of an edge read 64 contiguous bytes of the sender's row.
        {
          const bool ok = valid;
          float W[5][5];
          for (int m1 = 0; m1 < n1; ++m1)
            for (int m3 = 0; m3 < n3; ++m3) W[m1][m3] = 0.f;
          if (ok) {
            // channels outermost (rolled), so only one float4 of features per
            // degree and one channel's dA are live at a time
            const float* hrow = SPECIES_IN ? a.ht + (int64_t)jme * C
                                           : a.ht + ((int64_t)jme * NLM + pp.l1 * pp.l1) * C;
#pragma unroll 1
            for (int q = 0; q < C / 16; ++q) {
              float4 hv4[n1];
#pragma unroll
              for (int m1 = 0; m1 < n1; ++m1)
                hv4[m1] = *(const float4*)(hrow + (SPECIES_IN ? 0 : m1 * C) + 16 * q + 4 * g);
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int c = 16 * q + 4 * g + u;
                const float R = sR[el * RS + c];
                float A3[n3];
#pragma unroll
                for (int m3 = 0; m3 < n3; ++m3) A3[m3] = sAi[(ob + m3) * C + c];
#pragma unroll
                for (int m1 = 0; m1 < n1; ++m1) {
                  const float hv = u == 0 ? hv4[m1].x : (u == 1 ? hv4[m1].y : (u == 2 ? hv4[m1].z : hv4[m1].w));
                  const float Rh = R * hv;
#pragma unroll
                  for (int m3 = 0; m3 < n3; ++m3) W[m1][m3] += Rh * A3[m3];
                }
              }
            }
          }
          for (int m1 = 0; m1 < n1; ++m1)
            for (int m3 = 0; m3 < n3; ++m3) {
              float w = W[m1][m3];
              w += __shfl_xor(w, 16);
              w += __shfl_xor(w, 32);
              W[m1][m3] = w;
            }
          const float* cg = opaque_ptr(a.cg + PL::cg_off(pi));
          for (int m2 = 0; m2 < n2; ++m2) {
            float s = 0.f;
            for (int m1 = 0; m1 < n1; ++m1)
              for (int m3 = 0; m3 < n3; ++m3) s += cg[(m1 * n2 + m2) * n3 + m3] * W[m1][m3];
            Ybar[pp.l2 * pp.l2 + m2] += s;
          }
        }
        __syncthreads();
        // MLP backward through layer 3: ab2^T += W3_p (hidden x C) x Rbar_p^T
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
          for (int kc = 0; kc < O::kch(C); ++kc)
            ab2[mt] = O::mma(O::ldt(w3b, (pi * 4 + mt) * O::kch(C) + kc, lane),
                             O::from_row(sRb + el * RS, kc, g), ab2[mt]);
        }
      });
      if constexpr (TO_PART) {
        if (valid) {
#pragma unroll
          for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) pe[16 * mt + 4 * g + r] = ab2[mt][r];
          if (g == 0) {
#pragma unroll
            for (int k = 0; k < NLM; ++k) pe[64 + k] = Ybar[k];
          }
        }
        continue;
      }
      // remaining MLP backward: silu'(p2) -> W2 -> silu'(p1) -> W1
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
          acc = O::mma(O::ldt(opaque_ptr(a.w2b), mt * O::KC64 + kc, lane), O::from_tiles(pb2, kc), acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) pb1[mt][r] = acc[r] * dsilu(p1[mt][r]);
      }
      {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < O::KC64; ++kc)
          acc = O::mma(O::ldt(opaque_ptr(a.w1b), kc, lane), O::from_tiles(pb1, kc), acc);
        __syncthreads();
        if (g < 2) {
#pragma unroll
          for (int r = 0; r < 4; ++r) seb[el * kNB + 4 * g + r] = acc[r];
        }
        __syncthreads();
      }
      if (lane < kTileE && valid) {
        float dbar = 0.f;
#pragma unroll
        for (int n = 0; n < kNB; ++n) dbar += seb[el * kNB + n] * geo.dbasis[n];
        float gu[3];
        sh_grad_contract(Ybar, geo.u, gu);
        const float ud = gu[0] * geo.u[0] + gu[1] * geo.u[1] + gu[2] * geo.u[2];
        const float invd = 1.0f / geo.d;
        float4 acc = a.g[e];
        acc.x += dbar * geo.u[0] + (gu[0] - ud * geo.u[0]) * invd;
        acc.y += dbar * geo.u[1] + (gu[1] - ud * geo.u[1]) * invd;
        acc.z += dbar * geo.u[2] + (gu[2] - ud * geo.u[2]) * invd;
        a.g[e] = acc;
      }
    }
    if constexpr (HTBAR) {
#pragma unroll
      for (int o = 0; o < NIN; ++o)
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
          const int lo = o < 1 ? 0 : (o < 4 ? 1 : 2);      // input degree of row o
          const int f = first_of(lo);
          // blocks of degrees with no path in this launch are left alone
          bool mine = false;
          for (int q = P0; q < PE; ++q) mine = mine || PL::get(q).l1 == lo;
          if ((P0 > 0 || PE < NP) && !mine) continue;
          float vv = hb[o][k];
          if constexpr (EPL == 2) vv += __shfl_down(vv, 32);
          float* dst = a.htbar + ((int64_t)i * NIN + o) * C + cl + k * CW;
          if (eg == 0) *dst = (f < P0) ? *dst + vv : vv;
        }
    }
  }
}

// ------------------------------------------------------------ dispatch

static int edge_grid(int64_t n) {
  int64_t g = n < 262144 ? n : 262144;
  return (int)(g < 1 ? 1 : g);
}

template <int PREC, int C, int L>
static void fwd_kind(int kind, const EdgeArgs& a, hipStream_t s) {
  const int gr = edge_grid(a.n);
  switch (kind) {
    case KIND_ONLY: k_edge_fwd<PREC, C, L, KIND_ONLY><<<gr, 64, 0, s>>>(a); break;
    case KIND_FIRST: k_edge_fwd<PREC, C, L, KIND_FIRST><<<gr, 64, 0, s>>>(a); break;
    case KIND_MID: k_edge_fwd<PREC, C, L, KIND_MID><<<gr, 64, 0, s>>>(a); break;
    default: k_edge_fwd<PREC, C, L, KIND_LAST><<<gr, 64, 0, s>>>(a); break;
  }
}

template <int PREC, int C, int L>
static void bwd_kind(int kind, const EdgeArgs& a, hipStream_t s) {
  const int gr = edge_grid(a.n);
  switch (kind) {
    case KIND_ONLY: k_edge_bwd<PREC, C, L, KIND_ONLY, false><<<gr, 64, 0, s>>>(a); break;
    case KIND_FIRST: k_edge_bwd<PREC, C, L, KIND_FIRST, false><<<gr, 64, 0, s>>>(a); break;
    case KIND_MID:
      // a few paths per launch (see k_edge_bwd); path order (l1, l2, l3):
      // l_max = 2: 000 011 022 | 101 110 | 112 121 | 202 211 | 220 | 222 | finish
      // l_max = 1: 000 011 | 101 110 (finishes)
      if constexpr (L >= 2) {
        k_edge_bwd<PREC, C, L, KIND_MID, true, 0, 3, false><<<gr, 64, 0, s>>>(a);
        k_edge_bwd<PREC, C, L, KIND_MID, true, 3, 5, false><<<gr, 64, 0, s>>>(a);
        k_edge_bwd<PREC, C, L, KIND_MID, true, 5, 7, false><<<gr, 64, 0, s>>>(a);
        k_edge_bwd<PREC, C, L, KIND_MID, true, 7, 9, false><<<gr, 64, 0, s>>>(a);
        k_edge_bwd<PREC, C, L, KIND_MID, true, 9, 10, false><<<gr, 64, 0, s>>>(a);
        k_edge_bwd<PREC, C, L, KIND_MID, true, 10, 11, false><<<gr, 64, 0, s>>>(a);
        k_edge_bwd<PREC, C, L, KIND_MID, true, 11, 11, true><<<gr, 64, 0, s>>>(a);
      } else {
        k_edge_bwd<PREC, C, L, KIND_MID, true, 0, 2, false><<<gr, 64, 0, s>>>(a);
        k_edge_bwd<PREC, C, L, KIND_MID, true, 2, 4, true><<<gr, 64, 0, s>>>(a);
      }
      break;
    default: k_edge_bwd<PREC, C, L, KIND_LAST, true><<<gr, 64, 0, s>>>(a); break;
  }
}

template <int PREC>
static void fwd_prec(int C, int L, int kind, const EdgeArgs& a, hipStream_t s) {
  if (C == 32 && L == 1) fwd_kind<PREC, 32, 1>(kind, a, s);
  else if (C == 32 && L == 2) fwd_kind<PREC, 32, 2>(kind, a, s);
  else if (C == 64 && L == 1) fwd_kind<PREC, 64, 1>(kind, a, s);
  else if (C == 64 && L == 2) fwd_kind<PREC, 64, 2>(kind, a, s);
  else if (C == 128 && L == 1) fwd_kind<PREC, 128, 1>(kind, a, s);
  else fwd_kind<PREC, 128, 2>(kind, a, s);
}

template <int PREC>
static void bwd_prec(int C, int L, int kind, const EdgeArgs& a, hipStream_t s) {
  if (C == 32 && L == 1) bwd_kind<PREC, 32, 1>(kind, a, s);
  else if (C == 32 && L == 2) bwd_kind<PREC, 32, 2>(kind, a, s);
  else if (C == 64 && L == 1) bwd_kind<PREC, 64, 1>(kind, a, s);
  else if (C == 64 && L == 2) bwd_kind<PREC, 64, 2>(kind, a, s);
  else if (C == 128 && L == 1) bwd_kind<PREC, 128, 1>(kind, a, s);
  else bwd_kind<PREC, 128, 2>(kind, a, s);
}

void launch_edge_fwd(int prec, int C, int L, int kind, const EdgeArgs& a, hipStream_t s) {
  if (prec == MPIP_BF16_MIXED) fwd_prec<1>(C, L, kind, a, s);
  else fwd_prec<0>(C, L, kind, a, s);
}

void launch_edge_bwd(int prec, int C, int L, int kind, const EdgeArgs& a, hipStream_t s) {
  if (prec == MPIP_BF16_MIXED) bwd_prec<1>(C, L, kind, a, s);
  else bwd_prec<0>(C, L, kind, a, s);
}

}  // namespace mpip
