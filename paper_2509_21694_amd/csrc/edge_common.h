// Device helpers shared by the edge kernels: compile-time path lists, edge
// geometry (radial basis, envelope, real harmonics), MFMA operand helpers
// and the radial-MLP forward in features x edges orientation.
#pragma once
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

// sin t and cos t for t in [0, pi]: Taylor polynomials (through x^13 and
// x^14) of the reduced argument x = min(t, pi - t) in [0, pi/2], whose
// truncation error is below 1e-9; sin(pi - x) = sin x, cos(pi - x) = -cos x.
__device__ __forceinline__ void sincos_0pi(float t, float* s, float* c) {
  const bool up = t > 1.5707963267948966f;
  const float x = up ? 3.14159265358979f - t : t, x2 = x * x;
  float ps = 1.f / 6227020800.f;
  ps = fmaf(ps, x2, -1.f / 39916800.f);
  ps = fmaf(ps, x2, 1.f / 362880.f);
  ps = fmaf(ps, x2, -1.f / 5040.f);
  ps = fmaf(ps, x2, 1.f / 120.f);
  ps = fmaf(ps, x2, -1.f / 6.f);
  ps = fmaf(ps, x2, 1.f);
  float pc = -1.f / 87178291200.f;
  pc = fmaf(pc, x2, 1.f / 479001600.f);
  pc = fmaf(pc, x2, -1.f / 3628800.f);
  pc = fmaf(pc, x2, 1.f / 40320.f);
  pc = fmaf(pc, x2, -1.f / 720.f);
  pc = fmaf(pc, x2, 1.f / 24.f);
  pc = fmaf(pc, x2, -0.5f);
  pc = fmaf(pc, x2, 1.f);
  *s = x * ps;
  *c = up ? -pc : pc;
}

// Per-kernel constants of the geometry (cutoff, basis normalisation,
// envelope polynomial), formed once per wave from r_c and p and kept in
// scalar registers.
struct GeoK {
  float irc;        // 1 / r_c
  float pi_irc;     // pi / r_c
  float pref;       // sqrt(2 / r_c)
  float ea, eb, ec; // envelope 1 - ea x^p + eb x^(p+1) - ec x^(p+2)
  float da, db, dc; // its derivative in d: (-da x^(p-1) + db x^p - dc x^(p+1))
  int p;
};

__device__ __forceinline__ float sgpr_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

__device__ __forceinline__ GeoK geo_consts(float rc, int p) {
  GeoK k;
  const float irc = 1.0f / rc;
  const float a = 0.5f * (p + 1) * (p + 2), b = (float)(p * (p + 2)), c = 0.5f * p * (p + 1);
  k.irc = sgpr_f(irc);
  k.pi_irc = sgpr_f(3.14159265358979f * irc);
  k.pref = sgpr_f(sqrtf(2.0f * irc));
  k.ea = sgpr_f(a); k.eb = sgpr_f(b); k.ec = sgpr_f(c);
  k.da = sgpr_f(a * p * irc); k.db = sgpr_f(b * (p + 1) * irc); k.dc = sgpr_f(c * (p + 2) * irc);
  k.p = __builtin_amdgcn_readfirstlane(p);
  return k;
}

// Tail lanes of a tile (valid == false) evaluate a unit vector along x and
// are zeroed at the end, so the code has no divergent branch.  The Bessel
// argument pi d / r_c lies in [0, pi] for every edge; sin(n t), cos(n t)
// follow from the Chebyshev recurrence, and with A = sqrt(2/r_c) / d
//   basis_n  = f A sin(n t)
//   dbasis_n = f' A sin(n t) + f A (n pi / r_c cos(n t) - sin(n t) / d)
//            = A (f' - f / d) sin(n t) + n (f A pi / r_c) cos(n t).
__device__ __forceinline__ void edge_geometry(float4 v, bool valid, const GeoK& k, Geo& g) {
  const float vx = valid ? v.x : 1.f, vy = valid ? v.y : 0.f, vz = valid ? v.z : 0.f;
  // |v| and 1/|v| from the hardware reciprocal square root (about 1 ulp)
  const float d2 = vx * vx + vy * vy + vz * vz;
  const float inv = __builtin_amdgcn_rsqf(d2);
  const float d = d2 * inv;
  const float x = vx * inv, y = vy * inv, z = vz * inv;
  const float msk = valid ? 1.f : 0.f;
  g.u[0] = msk * x; g.u[1] = msk * y; g.u[2] = msk * z; g.d = d;
  const float s3 = 1.7320508075688772f, s5 = 2.23606797749979f, s15 = 3.872983346207417f;
  g.Y[0] = msk;
  g.Y[1] = msk * s3 * y; g.Y[2] = msk * s3 * z; g.Y[3] = msk * s3 * x;
  g.Y[4] = msk * s15 * x * y; g.Y[5] = msk * s15 * y * z; g.Y[6] = msk * 0.5f * s5 * (3.f * z * z - 1.f);
  g.Y[7] = msk * s15 * x * z; g.Y[8] = msk * 0.5f * s15 * (x * x - y * y);
  // polynomial envelope of order p (zero from r_c on)
  const float xr = d * k.irc;
  float xp1 = 1.f;  // x^(p-1)
  for (int q = 0; q < k.p - 1; ++q) xp1 *= xr;
  const float xp = xp1 * xr, xq = xp * xr, xs = xq * xr;
  const float in = (valid && xr < 1.f) ? 1.f : 0.f;
  const float env = in * (1.f - k.ea * xp + k.eb * xq - k.ec * xs);
  const float denv = in * (-k.da * xp1 + k.db * xp - k.dc * xq);
  const float th = fminf(d * k.pi_irc, 3.14159265358979f);
  float s1, c1;
  sincos_0pi(th, &s1, &c1);
  const float A = k.pref * inv;
  const float E1 = env * A;
  const float F1 = A * (denv - env * inv);
  const float F2 = E1 * k.pi_irc;
  const float tc = 2.f * c1;
  float sp = 0.f, cp = 1.f, sn = s1, cn = c1, nF2 = F2;
#pragma unroll
  for (int n = 1; n <= kNB; ++n) {
    g.basis[n - 1] = E1 * sn;
    g.dbasis[n - 1] = fmaf(F1, sn, nF2 * cn);
    const float sx = fmaf(tc, sn, -sp), cx = fmaf(tc, cn, -cp);
    sp = sn; cp = cn; sn = sx; cn = cx;
    nF2 += F2;
  }
}

// Direction, length and harmonics only (the kernels that take the radial
// MLP's output from its table need no basis): the same u, d and Y as
// edge_geometry, basis and dbasis left unset.
__device__ __forceinline__ void edge_direction(float4 v, bool valid, Geo& g) {
  const float vx = valid ? v.x : 1.f, vy = valid ? v.y : 0.f, vz = valid ? v.z : 0.f;
  const float d2 = vx * vx + vy * vy + vz * vz;
  const float inv = __builtin_amdgcn_rsqf(d2);
  const float d = d2 * inv;
  const float x = vx * inv, y = vy * inv, z = vz * inv;
  const float msk = valid ? 1.f : 0.f;
  g.u[0] = msk * x; g.u[1] = msk * y; g.u[2] = msk * z; g.d = d;
  const float s3 = 1.7320508075688772f, s5 = 2.23606797749979f, s15 = 3.872983346207417f;
  g.Y[0] = msk;
  g.Y[1] = msk * s3 * y; g.Y[2] = msk * s3 * z; g.Y[3] = msk * s3 * x;
  g.Y[4] = msk * s15 * x * y; g.Y[5] = msk * s15 * y * z; g.Y[6] = msk * 0.5f * s5 * (3.f * z * z - 1.f);
  g.Y[7] = msk * s15 * x * z; g.Y[8] = msk * 0.5f * s15 * (x * x - y * y);
}

// Tabulated radial MLP (BF16 form).  The second hidden layer a(d) in R^64
// of one layer's radial MLP is a function of the edge length alone; the
// table holds, for the kRadTab intervals [d_k, d_k+1) of [0, r_c]
// (d_k = k r_c / kRadTab), a(d_k) and the increment a(d_k+1) - a(d_k) as a
// BF16 pair per hidden unit (value in the low half), [kRadTab][64] words.
// Between the knots a is interpolated linearly:
//   a(d) = a(d_k) + tau (a(d_k+1) - a(d_k)),  tau = d kRadTab / r_c - k,
// and its derivative is the interval's slope, (a(d_k+1) - a(d_k)) kRadTab / r_c.
// Lengths at or past r_c take the last interval at tau = 1 (a = 0 there).
struct RadPos {
  int k;
  float tau;
};
__device__ __forceinline__ RadPos rad_pos(float d, float scale) {
  const float t = fminf(d * scale, (float)kRadTab);
  const int k = min((int)t, kRadTab - 1);
  return {k, fminf(t - (float)k, 1.f)};
}
// The table words of a lane's four D tiles in the features x edges layout
// (lane (g, el): hidden 16 mt + 4 g + r of the lane's edge), with tau
struct RadRow {
  uint4 w[4];
  float tau;
};
__device__ __forceinline__ RadRow rad_load(const uint32_t* tab, RadPos rp, int g) {
  const uint4* row = (const uint4*)(tab + (size_t)rp.k * 64) + g;
  RadRow rr;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) rr.w[mt] = row[4 * mt];
  rr.tau = rp.tau;
  return rr;
}
// a(d) in that layout and, when sl is given, the increments
__device__ __forceinline__ void rad_eval(const RadRow& rr, f32x4* a2, f32x4* sl) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const unsigned w[4] = {rr.w[mt].x, rr.w[mt].y, rr.w[mt].z, rr.w[mt].w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float v = __uint_as_float(w[r] << 16), inc = __uint_as_float(w[r] & 0xffff0000u);
      a2[mt][r] = fmaf(rr.tau, inc, v);
      if (sl) sl[mt][r] = inc;
    }
  }
}
__device__ __forceinline__ void rad_tiles(const uint32_t* tab, RadPos rp, int g, f32x4* a2, f32x4* sl) {
  rad_eval(rad_load(tab, rp, g), a2, sl);
}
// |v| as edge_direction forms it (tail lanes carry a unit vector)
__device__ __forceinline__ float edge_length(float4 v) {
  const float d2 = v.x * v.x + v.y * v.y + v.z * v.z;
  return d2 * __builtin_amdgcn_rsqf(d2);
}
// dE/dd of the lane's edge from dE/da (ab2, same layout) and the increments:
// sum over the 64 hidden units, the four lane groups of an edge combined
__device__ __forceinline__ float rad_dbar(const f32x4* ab2, const f32x4* sl, float scale) {
  float s = 0.f;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) s = fmaf(ab2[mt][r], sl[mt][r], s);
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  return s * scale;
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
  // operand tile `tile` (64 lanes) of a packed array in global memory: the
  // tile base is kept scalar and formed at its use, the lane adds a 32-bit offset
  __device__ static T ldt(const void* base, int tile, int lane) {
    const T* b = (const T*)base + (size_t)tile * 64;
    asm volatile("" : "+s"(b));
    return *(const T*)((const char*)b + (unsigned)lane * sizeof(T));
  }
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
  __device__ static T ldt(const void* base, int tile, int lane) {
    const T* b = (const T*)base + (size_t)tile * 64;
    asm volatile("" : "+s"(b));
    return *(const T*)((const char*)b + (unsigned)lane * sizeof(T));
  }
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

// W1, W2: operand arrays in global memory or LDS (same packing)
template <int PREC, typename WT>
__device__ __forceinline__ void mlp_forward_w(const Geo& geo, int lane, const WT* W1, const WT* W2, f32x4* p1,
                                              f32x4* p2) {
  typedef Op<PREC> O;
  const int g = lane >> 4;
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = z;
    if constexpr (PREC == 1) {
      acc = O::mma(W1[mt * 64 + lane], basis_op_bf16(geo.basis, g), acc);
    } else {
#pragma unroll
      for (int q = 0; q < 2; ++q) acc = O::mma(W1[(mt * 2 + q) * 64 + lane], geo.basis[4 * q + g], acc);
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
    for (int kc = 0; kc < O::KC64; ++kc) acc = O::mma(W2[(mt * O::KC64 + kc) * 64 + lane], O::from_tiles(a1, kc), acc);
    p2[mt] = acc;
  }
}

template <int PREC>
__device__ __forceinline__ void mlp_forward(const Geo& geo, int lane, const void* w1a, const void* w2a,
                                            f32x4* p1, f32x4* p2) {
  typedef typename Op<PREC>::T T;
  mlp_forward_w<PREC, T>(geo, lane, (const T*)w1a, (const T*)w2a, p1, p2);
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
      acc = O::mma(aop[kc], O::ldt(w3f, (p * (C / 16) + nt) * O::KC64 + kc, lane), acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) sR[(4 * g + r) * RS + 16 * nt + n] = acc[r];
  }
}

__device__ __forceinline__ int64_t edges_total(const EdgeArgs& a) { return (int64_t)a.row_ptr[a.n]; }

// ---- FP32 radial MLP from row-major LDS copies (W1 [8][65], W2 [64][65],
// rows the layer input), 16x16x4 MFMA: D tile row 4 g + r, column lane % 16;
// A operand of lane (g, l16) = A[l16][g], B operand = B[g][l16]

// hidden index of k-chunk q, lane group g (the D -> B operand order of the MLP)
__device__ __forceinline__ int phi_f(int q, int g) { return 16 * (q / 4) + 4 * g + (q % 4); }

// layers 1 and 2: p1, p2 (and a1 = silu(p1)) as D tiles (hidden 16 mt + 4 g + r) x (edge)
__device__ __forceinline__ void mlp_fwd_rows(const Geo& geo, int lane, const float* sW1, const float* sW2, f32x4* p1,
                                             f32x4* a1, f32x4* p2) {
  const int g = lane >> 4, el = lane & 15;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 2; ++q) acc = mfma_f32(sW1[(4 * q + g) * 65 + 16 * mt + el], geo.basis[4 * q + g], acc);
    p1[mt] = acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) a1[mt][r] = silu(acc[r]);
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < 16; ++kc) acc = mfma_f32(sW2[phi_f(kc, g) * 65 + 16 * mt + el], a1[kc / 4][kc % 4], acc);
    p2[mt] = acc;
  }
}

// backward from ab2 = dE/da2 (features x edges): pb2 = ab2 silu'(p2) -> W2 ->
// silu'(p1) -> W1 -> dE/de; lane el (< 16) receives dE/de of edge el in eb
__device__ __forceinline__ void mlp_bwd_rows(const f32x4* ab2, const f32x4* p1, const f32x4* p2, int lane,
                                             const float* sW1, const float* sW2, float* eb) {
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
    for (int kc = 0; kc < 16; ++kc) acc = mfma_f32(sW2[(16 * mt + el) * 65 + phi_f(kc, g)], pb2[kc / 4][kc % 4], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) pb1[mt][r] = acc[r] * dsilu(p1[mt][r]);
  }
  f32x4 eacc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kc = 0; kc < 16; ++kc)
    eacc = mfma_f32(el < kNB ? sW1[(el < kNB ? el : 0) * 65 + phi_f(kc, g)] : 0.f, pb1[kc / 4][kc % 4], eacc);
  const int src = el + 16;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    eb[r] = eacc[r];
    eb[4 + r] = __shfl(eacc[r], src);
  }
}

// stage n floats of a row-major weight copy into LDS (whole workgroup)
template <int NF>
__device__ __forceinline__ void stage_rows(float* dst, const float* src) {
  for (int t = threadIdx.x; t < NF; t += blockDim.x) dst[t] = src[t];
}


// Rows of the calling wave.  Workgroups are dispatched to the 8 XCDs in
// round-robin order, so workgroup b runs on XCD b % 8: each XCD takes a
// contiguous eighth of the spatially sorted rows and its waves walk that
// range side by side, so the sender rows they gather stay within one L2.
// The grid is a multiple of 8 workgroups.
struct RowWalk {
  int64_t i, end, step;
};
template <int NW>
__device__ __forceinline__ RowWalk row_walk(int64_t n) {
  const int b = blockIdx.x, x = b & 7, lb = b >> 3, BX = gridDim.x >> 3;
  const int64_t r0 = n * x / 8, r1 = n * (x + 1) / 8;
  return {r0 + (int64_t)lb * NW + (threadIdx.x >> 6), r1, (int64_t)BX * NW};
}

// Edge ranges of a wave's current row and of its next row along a RowWalk
// (the next row's bounds are read a row ahead), so that a tile loop can
// request the first tile of the next row while it works on its last one.
// row_end: the walked prefix of each row (receptive-field trimming), or null.
struct RowAhead {
  int64_t i, end, step;
  int e0, e1, n0, n1;
  __device__ __forceinline__ RowAhead(const RowWalk& rw, const int32_t* row_ptr, const int32_t* row_end)
      : i(rw.i), end(rw.end), step(rw.step), e0(0), e1(0), n0(0), n1(0) {
    if (i < end) { e0 = row_ptr[i]; e1 = row_end ? row_end[i] : row_ptr[i + 1]; }
    if (i + step < end) { n0 = row_ptr[i + step]; n1 = row_end ? row_end[i + step] : row_ptr[i + step + 1]; }
  }
  __device__ __forceinline__ bool has_row() const { return i < end; }
  __device__ __forceinline__ bool has_next() const { return i + step < end; }
  __device__ __forceinline__ void advance(const int32_t* row_ptr, const int32_t* row_end) {
    i += step;
    e0 = n0;
    e1 = n1;
    if (i + step < end) { n0 = row_ptr[i + step]; n1 = row_end ? row_end[i + step] : row_ptr[i + step + 1]; }
  }
};


}  // namespace mpip
