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
#include <utility>

#include "kernels.h"

namespace mpip {

template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
// f(integral_constant<int, 0>), ..., f(integral_constant<int, N-1>), fully unrolled
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ------------------------------------------------------------ path lists

struct P3 { int l1, l2, l3; };

constexpr bool natural3(int a, int b, int c) {
  return ((a + b + c) % 2 == 0) && c >= (a > b ? a - b : b - a) && c <= a + b;
}

template <int L, int KIND>
struct PathList {
  static constexpr int l1max() { return (KIND == KIND_ONLY || KIND == KIND_FIRST) ? 0 : L; }
  static constexpr bool keep(int a, int b, int c) {
    if (!natural3(a, b, c)) return false;
    if (KIND == KIND_ONLY || KIND == KIND_LAST) return c == 0;
    return true;
  }
  static constexpr int count() {
    int n = 0;
    for (int a = 0; a <= l1max(); ++a)
      for (int b = 0; b <= L; ++b)
        for (int c = 0; c <= L; ++c)
          if (keep(a, b, c)) ++n;
    return n;
  }
  static constexpr P3 get(int i) {
    int n = 0;
    for (int a = 0; a <= l1max(); ++a)
      for (int b = 0; b <= L; ++b)
        for (int c = 0; c <= L; ++c)
          if (keep(a, b, c)) {
            if (n == i) return P3{a, b, c};
            ++n;
          }
    return P3{0, 0, 0};
  }
  static constexpr int yc_off(int i) {
    int o = 0;
    for (int k = 0; k < i; ++k) o += (2 * get(k).l1 + 1) * (2 * get(k).l3 + 1);
    return o;
  }
  static constexpr int cg_off(int i) {
    int o = 0;
    for (int k = 0; k < i; ++k) o += (2 * get(k).l1 + 1) * (2 * get(k).l2 + 1) * (2 * get(k).l3 + 1);
    return o;
  }
  static constexpr int nyc() { return yc_off(count()); }
  static constexpr int nin() { return (KIND == KIND_ONLY || KIND == KIND_FIRST) ? 1 : (L + 1) * (L + 1); }
  static constexpr int nout() { return (KIND == KIND_ONLY || KIND == KIND_LAST) ? 1 : (L + 1) * (L + 1); }
};

// ------------------------------------------------------------ geometry

struct Geo {
  float u[3];
  float d;
  float Y[kMaxNlm];
  float basis[kNB];
  float dbasis[kNB];
};

__device__ __forceinline__ void edge_geometry(float4 v, bool valid, float rc, int p, Geo& g) {
  if (!valid) {
    g.u[0] = g.u[1] = g.u[2] = 0.f;
    g.d = 1.f;
#pragma unroll
    for (int k = 0; k < kMaxNlm; ++k) g.Y[k] = 0.f;
#pragma unroll
    for (int k = 0; k < kNB; ++k) g.basis[k] = g.dbasis[k] = 0.f;
    return;
  }
  const float d = sqrtf(v.x * v.x + v.y * v.y + v.z * v.z);
  const float inv = 1.0f / d;
  const float x = v.x * inv, y = v.y * inv, z = v.z * inv;
  g.u[0] = x; g.u[1] = y; g.u[2] = z; g.d = d;
  const float s3 = 1.7320508075688772f, s5 = 2.23606797749979f, s15 = 3.872983346207417f;
  g.Y[0] = 1.f;
  g.Y[1] = s3 * y; g.Y[2] = s3 * z; g.Y[3] = s3 * x;
  g.Y[4] = s15 * x * y; g.Y[5] = s15 * y * z; g.Y[6] = 0.5f * s5 * (3.f * z * z - 1.f);
  g.Y[7] = s15 * x * z; g.Y[8] = 0.5f * s15 * (x * x - y * y);
  // polynomial envelope of order p
  const float xr = d / rc;
  float env = 0.f, denv = 0.f;
  if (xr < 1.f) {
    const float a = 0.5f * (p + 1) * (p + 2), b = (float)(p * (p + 2)), c = 0.5f * p * (p + 1);
    float xp1 = 1.f;  // x^(p-1)
    for (int k = 0; k < p - 1; ++k) xp1 *= xr;
    const float xp = xp1 * xr, xq = xp * xr, xs = xq * xr;
    env = 1.f - a * xp + b * xq - c * xs;
    denv = (-a * p * xp1 + b * (p + 1) * xp - c * (p + 2) * xq) / rc;
  }
  // Bessel basis via the Chebyshev recurrence for sin(n t), cos(n t)
  const float pref = sqrtf(2.0f / rc);
  const float th = 3.14159265358979f * d / rc;
  float s1, c1;
  sincosf(th, &s1, &c1);
  float sp = 0.f, cp = 1.f, sn = s1, cn = c1;
#pragma unroll
  for (int n = 1; n <= kNB; ++n) {
    const float kn = n * 3.14159265358979f / rc;
    const float B = pref * sn * inv;
    const float dB = pref * (kn * d * cn - sn) * inv * inv;
    g.basis[n - 1] = env * B;
    g.dbasis[n - 1] = denv * B + env * dB;
    const float sx = 2.f * c1 * sn - sp, cx = 2.f * c1 * cn - cp;
    sp = sn; cp = cn; sn = sx; cn = cx;
  }
}

// gu = (dP/du)^T Ybar for the polynomials above
__device__ __forceinline__ void sh_grad_contract(const float* Yb, const float* u, float* gu) {
  const float s3 = 1.7320508075688772f, s5 = 2.23606797749979f, s15 = 3.872983346207417f;
  const float x = u[0], y = u[1], z = u[2];
  gu[0] = s3 * Yb[3] + s15 * (y * Yb[4] + z * Yb[7] + x * Yb[8]);
  gu[1] = s3 * Yb[1] + s15 * (x * Yb[4] + z * Yb[5] - y * Yb[8]);
  gu[2] = s3 * Yb[2] + s15 * (y * Yb[5] + x * Yb[7]) + 3.f * s5 * z * Yb[6];
}

// ------------------------------------------------------------ MFMA helpers

template <int PREC> struct Op;

template <> struct Op<1> {  // BF16 operands, K = 32 per instruction
  typedef bf16x8 T;
  static constexpr int KC64 = 2;   // k-chunks for K = 64
  __device__ static f32x4 mma(T a, T b, f32x4 c) { return mfma_bf16(a, b, c); }
  // operand of k-chunk kc from four D tiles (hidden 16*t + 4*g + r)
  __device__ static T from_tiles(const f32x4* t, int kc) {
    T v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (__bf16)t[2 * kc + j / 4][j % 4];
    return v;
  }
  __device__ static T load(const void* base, int idx) { return ((const T*)base)[idx]; }
  // operand of channels 32*kc + 8*g + j from an LDS row
  __device__ static T from_row(const float* row, int kc, int g) {
    T v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (__bf16)row[32 * kc + 8 * g + j];
    return v;
  }
  static constexpr int kch(int K) { return K / 32; }
};

template <> struct Op<0> {  // FP32 operands, K = 4 per instruction
  typedef float T;
  static constexpr int KC64 = 16;
  __device__ static f32x4 mma(T a, T b, f32x4 c) { return mfma_f32(a, b, c); }
  __device__ static T from_tiles(const f32x4* t, int q) { return t[q / 4][q % 4]; }
  __device__ static T load(const void* base, int idx) { return ((const T*)base)[idx]; }
  __device__ static T from_row(const float* row, int q, int g) { return row[4 * q + g]; }
  static constexpr int kch(int K) { return K / 4; }
};

// basis operand (K = n_basis = 8 padded): bf16: group 0 holds basis[j];
// f32: chunk q, group g holds basis[4q + g]
__device__ __forceinline__ bf16x8 basis_op_bf16(const float* b, int g) {
  bf16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = (__bf16)(g == 0 ? b[j] : 0.f);
  return v;
}

template <int PREC>
__device__ __forceinline__ void mlp_forward(const Geo& geo, int lane, const void* w1a, const void* w2a,
                                            f32x4* p1, f32x4* p2) {
  typedef Op<PREC> O;
  const int g = lane >> 4;
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = z;
    if constexpr (PREC == 1) {
      acc = O::mma(O::load(w1a, mt * 64 + lane), basis_op_bf16(geo.basis, g), acc);
    } else {
#pragma unroll
      for (int q = 0; q < 2; ++q) acc = O::mma(O::load(w1a, (mt * 2 + q) * 64 + lane), geo.basis[4 * q + g], acc);
    }
    p1[mt] = acc;
  }
  f32x4 a1[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) a1[mt][r] = silu(p1[mt][r]);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = z;
#pragma unroll
    for (int kc = 0; kc < O::KC64; ++kc)
      acc = O::mma(O::load(w2a, (mt * O::KC64 + kc) * 64 + lane), O::from_tiles(a1, kc), acc);
    p2[mt] = acc;
  }
}

// R_p for one path: D[nt] tiles (edges 4g + r, channels 16 nt + lane%16) -> LDS
template <int PREC, int C>
__device__ __forceinline__ void radial_out(const f32x4* a2, int lane, const void* w3f, int p, float* sR,
                                           int RS) {
  typedef Op<PREC> O;
  const int g = lane >> 4, n = lane & 15;
  typename O::T aop[O::KC64];
#pragma unroll
  for (int kc = 0; kc < O::KC64; ++kc) aop[kc] = O::from_tiles(a2, kc);
#pragma unroll
  for (int nt = 0; nt < C / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < O::KC64; ++kc)
      acc = O::mma(aop[kc], O::load(w3f, ((p * (C / 16) + nt) * O::KC64 + kc) * 64 + lane), acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) sR[(4 * g + r) * RS + 16 * nt + n] = acc[r];
  }
}

__device__ __forceinline__ int64_t edges_total(const EdgeArgs& a) { return (int64_t)a.row_ptr[a.n]; }

// ------------------------------------------------------------ forward

template <int PREC, int C, int L, int KIND>
__global__ __launch_bounds__(64) void k_edge_fwd(EdgeArgs a) {
  typedef PathList<L, KIND> PL;
  constexpr int NP = PL::count();
  constexpr int NIN = PL::nin(), NOUT = PL::nout(), NYC = PL::nyc();
  constexpr int NLM = (L + 1) * (L + 1);
  constexpr int CW = C < 64 ? C : 64;      // lanes per edge group
  constexpr int CPL = C / CW;              // channels per lane
  constexpr int EPL = 64 / CW;             // edge groups
  constexpr int RS = C + 1;
  constexpr bool SPECIES_IN = (KIND == KIND_ONLY || KIND == KIND_FIRST);
  __shared__ float sR[kTileE * RS];
  __shared__ float syc[kTileE * NYC];
  __shared__ int sj[kTileE];
  if (edges_total(a) > a.capacity || a.status[ST_FLAGS] != 0) return;
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
      edge_geometry(v, valid, a.rc, a.envelope_p, geo);
      if (lane < kTileE) {
        sj[el] = valid ? (SPECIES_IN ? __float_as_int(v.w) : a.e_src[e]) : -1;
        // YC[p][m1][m3] = sum_m2 C_p[m1][m2][m3] Y[l2 m2]
        static_for<NP>([&](auto PI) {
          constexpr int pi = decltype(PI)::value;
          constexpr P3 pp = PL::get(pi);
          constexpr int n1 = 2 * pp.l1 + 1, n2 = 2 * pp.l2 + 1, n3 = 2 * pp.l3 + 1;
          const float* cg = a.cg + PL::cg_off(pi);
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
      mlp_forward<PREC>(geo, lane, a.w1a, a.w2a, p1, p2);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) a2[mt][r] = silu(p2[mt][r]);
      static_for<NP>([&](auto PI) {
        constexpr int pi = decltype(PI)::value;
        constexpr P3 pp = PL::get(pi);
        constexpr int n1 = 2 * pp.l1 + 1, n3 = 2 * pp.l3 + 1;
        __syncthreads();
        radial_out<PREC, C>(a2, lane, a.w3f, pi, sR, RS);
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
        if constexpr (EPL == 2) vv += __shfl_down(vv, 32);
        if (eg == 0) a.A[((int64_t)i * NOUT + o) * C + cl + k * CW] = a.inv_n * vv;
      }
  }
}

// ------------------------------------------------------------ backward

template <int PREC, int C, int L, int KIND, bool HTBAR>
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
  constexpr int CB = C / 4;                // channel block of pass B
  constexpr bool SPECIES_IN = (KIND == KIND_ONLY || KIND == KIND_FIRST);
  __shared__ float sR[kTileE * RS];
  __shared__ float sRb[kTileE * RS];
  __shared__ float syc[kTileE * NYC];
  __shared__ float sAi[NOUT * C];
  __shared__ float seb[kTileE * kNB];
  __shared__ int sj[kTileE];
  if (edges_total(a) > a.capacity || a.status[ST_FLAGS] != 0) return;
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
      edge_geometry(v, valid, a.rc, a.envelope_p, geo);
      const int jme = valid ? (SPECIES_IN ? __float_as_int(v.w) : a.e_src[e]) : -1;
      __syncthreads();
      if (lane < kTileE) {
        sj[el] = jme;
        static_for<NP>([&](auto PI) {
          constexpr int pi = decltype(PI)::value;
          constexpr P3 pp = PL::get(pi);
          constexpr int n1 = 2 * pp.l1 + 1, n2 = 2 * pp.l2 + 1, n3 = 2 * pp.l3 + 1;
          const float* cg = a.cg + PL::cg_off(pi);
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
      mlp_forward<PREC>(geo, lane, a.w1a, a.w2a, p1, p2);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) { a2[mt][r] = silu(p2[mt][r]); ab2[mt][r] = 0.f; }
      float Ybar[kMaxNlm];
#pragma unroll
      for (int k = 0; k < kMaxNlm; ++k) Ybar[k] = 0.f;
      static_for<NP>([&](auto PI) {
        constexpr int pi = decltype(PI)::value;
        constexpr P3 pp = PL::get(pi);
        constexpr int n1 = 2 * pp.l1 + 1, n2 = 2 * pp.l2 + 1, n3 = 2 * pp.l3 + 1;
        constexpr int ob = (NOUT == 1) ? 0 : pp.l3 * pp.l3;
        constexpr float sgn = (pp.l2 & 1) ? -1.f : 1.f;
        __syncthreads();
        radial_out<PREC, C>(a2, lane, a.w3f, pi, sR, RS);
        __syncthreads();
        // pass A: lanes own channels, walk the edges
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
        // pass B: lanes own (edge el, channel block g); dE/dY of the edge
        {
          const bool ok = valid;
          float W[5][5];
          for (int m1 = 0; m1 < n1; ++m1)
            for (int m3 = 0; m3 < n3; ++m3) W[m1][m3] = 0.f;
          if (ok) {
            for (int cc = 0; cc < CB; ++cc) {
              const int c = g * CB + cc;
              const float R = sR[el * RS + c];
              for (int m1 = 0; m1 < n1; ++m1) {
                const float hv = SPECIES_IN ? a.ht[(int64_t)jme * C + c]
                                            : a.ht[((int64_t)jme * NLM + pp.l1 * pp.l1 + m1) * C + c];
                const float Rh = R * hv;
                for (int m3 = 0; m3 < n3; ++m3) W[m1][m3] += Rh * sAi[(ob + m3) * C + c];
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
          const float* cg = a.cg + PL::cg_off(pi);
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
            ab2[mt] = O::mma(O::load(a.w3b, ((pi * 4 + mt) * O::kch(C) + kc) * 64 + lane),
                             O::from_row(sRb + el * RS, kc, g), ab2[mt]);
        }
      });
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
          acc = O::mma(O::load(a.w2b, (mt * O::KC64 + kc) * 64 + lane), O::from_tiles(pb2, kc), acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) pb1[mt][r] = acc[r] * dsilu(p1[mt][r]);
      }
      {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < O::KC64; ++kc)
          acc = O::mma(O::load(a.w1b, kc * 64 + lane), O::from_tiles(pb1, kc), acc);
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
          float vv = hb[o][k];
          if constexpr (EPL == 2) vv += __shfl_down(vv, 32);
          if (eg == 0) a.htbar[((int64_t)i * NIN + o) * C + cl + k * CW] = vv;
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
    case KIND_MID: k_edge_bwd<PREC, C, L, KIND_MID, true><<<gr, 64, 0, s>>>(a); break;
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
