// Molecular dynamics around the evaluation: the integrator kernels of
// mpip_md_run.  One step is the BAOAB splitting of Langevin dynamics
// (Leimkuhler and Matthews): half kick B, half drift A, the exact
// Ornstein-Uhlenbeck velocity update O over the full step, half drift A,
// new forces, half kick B.  With zero friction O is the identity and the
// step is velocity Verlet.  Units: Angstrom, fs, eV, amu, K.  The Gaussian
// numbers of O come from Philox4x32-10 (Salmon et al., SC'11) keyed by the
// seed, with the counter (atom, step), through the Box-Muller transform.
#include "kernels.h"

namespace mpip {

namespace {

// (eV / Angstrom) / amu in Angstrom / fs^2: e [C] / amu [kg] gives (J / m) / kg = m / s^2 per
// (V / m); times 1e10 (per Angstrom instead of per metre) and 1e-20 (m / s^2 in Angstrom / fs^2)
constexpr double kAccel = 1.602176634e-19 / 1.66053906660e-27 * 1e10 * 1e-20;
constexpr double kBoltzmann = 8.617333262e-5;  // eV / K

// one Philox4x32 round: products of the even words by the multipliers, the
// high halves mixed with the odd words and the key
__device__ __forceinline__ void philox_round(uint32_t* c, const uint32_t* k) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0, hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0], n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

__device__ __forceinline__ void philox4x32_10(uint32_t* c, uint64_t seed) {
  uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k);
    k[0] += 0x9E3779B9u;
    k[1] += 0xBB67AE85u;
  }
}

// three standard normal numbers for (atom, step)
__device__ __forceinline__ void normals3(uint64_t seed, int64_t atom, int64_t step, double* xi) {
  uint32_t c[4] = {(uint32_t)atom, (uint32_t)((uint64_t)atom >> 32), (uint32_t)step, (uint32_t)((uint64_t)step >> 32)};
  philox4x32_10(c, seed);
  const double two32 = 4294967296.0, two_pi = 6.283185307179586;
  const double u0 = ((double)c[0] + 1.0) / two32, u1 = ((double)c[1] + 0.5) / two32;
  const double u2 = ((double)c[2] + 1.0) / two32, u3 = ((double)c[3] + 0.5) / two32;
  const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
  xi[0] = r0 * cos(two_pi * u1);
  xi[1] = r0 * sin(two_pi * u1);
  xi[2] = r1 * cos(two_pi * u3);
}

// B, A, O, A of one step (everything before the new forces)
// (with a reference: flags an atom that has moved more than sqrt(thr2) since the list was built)
__global__ void k_md_first(int64_t n, double* __restrict__ x, double* __restrict__ v, const double* __restrict__ f,
                           const int32_t* __restrict__ spec, const double* __restrict__ masses, double dt, double c1,
                           double c2, double kT, uint64_t seed, int64_t step, const double* __restrict__ xref,
                           double thr2, int64_t* __restrict__ moved) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double m = masses[spec[i]];
  const double ak = kAccel / m;
  double vi[3], xi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    vi[d] = v[3 * i + d] + 0.5 * dt * ak * f[3 * i + d];
    xi[d] = x[3 * i + d] + 0.5 * dt * vi[d];
  }
  if (c1 != 1.0) {
    double z[3];
    normals3(seed, i, step, z);
    const double sig = sqrt(kT * kAccel / m);
#pragma unroll
    for (int d = 0; d < 3; ++d) vi[d] = c1 * vi[d] + c2 * sig * z[d];
  }
  double d2 = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double xn = xi[d] + 0.5 * dt * vi[d];
    x[3 * i + d] = xn;
    v[3 * i + d] = vi[d];
    if (xref) d2 += (xn - xref[3 * i + d]) * (xn - xref[3 * i + d]);
  }
  if (xref && d2 > thr2) atomicOr((unsigned long long*)moved, 1ull);
}

// the positions the neighbour list was built for
__global__ void k_md_reference(int64_t n, const double* __restrict__ x, double* __restrict__ xref,
                               int64_t* __restrict__ moved) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i == 0) *moved = 0;
  if (i >= 3 * n) return;
  xref[i] = x[i];
}

// B with the new forces; per-block sums of the kinetic energy (eV), fixed order
__global__ __launch_bounds__(256) void k_md_second(int64_t n, double* __restrict__ v, const double* __restrict__ f,
                                                   const int32_t* __restrict__ spec, const double* __restrict__ masses,
                                                   double dt, double* __restrict__ partials) {
  __shared__ double sh[256];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double ke = 0.0;
  if (i < n) {
    const double m = masses[spec[i]];
    const double ak = kAccel / m;
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double vd = v[3 * i + d] + 0.5 * dt * ak * f[3 * i + d];
      v[3 * i + d] = vd;
      s += vd * vd;
    }
    ke = 0.5 * m * s / kAccel;
  }
  sh[threadIdx.x] = ke;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

// the step's kinetic and potential energy; the evaluation's error flags
// are kept across steps (each evaluation clears its own status word)
__global__ void k_md_record(const double* __restrict__ partials, int nblocks, const double* __restrict__ energy,
                            const int64_t* __restrict__ status, double* __restrict__ epot, double* __restrict__ ekin,
                            int64_t* __restrict__ sticky) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) s += partials[b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (ekin) *ekin = sh[0];
    if (epot) *epot = *energy;
    *sticky |= status[ST_FLAGS];
  }
}

__global__ void k_md_flags(const int64_t* __restrict__ sticky, int64_t* __restrict__ status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) status[ST_FLAGS] |= *sticky;
}

}  // namespace

void md_first(int64_t n, double* x, double* v, const double* f, const int32_t* spec, const double* masses, double dt,
              double friction, double temperature, uint64_t seed, int64_t step, const double* xref, double thr2,
              int64_t* moved, hipStream_t s) {
  const double c1 = exp(-friction * dt), c2 = sqrt(1.0 - c1 * c1);
  k_md_first<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, x, v, f, spec, masses, dt, c1, c2,
                                                          kBoltzmann * temperature, seed, step, xref, thr2, moved);
}

void md_reference(int64_t n, const double* x, double* xref, int64_t* moved, hipStream_t s) {
  k_md_reference<<<(unsigned)((3 * n + 255) / 256), 256, 0, s>>>(n, x, xref, moved);
}

void md_second(int64_t n, double* v, const double* f, const int32_t* spec, const double* masses, double dt,
               double* partials, hipStream_t s) {
  k_md_second<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, v, f, spec, masses, dt, partials);
}

void md_record(const double* partials, int nblocks, const double* energy, const int64_t* status, double* epot,
               double* ekin, int64_t* sticky, hipStream_t s) {
  k_md_record<<<1, 256, 0, s>>>(partials, nblocks, energy, status, epot, ekin, sticky);
}

void md_flags(const int64_t* sticky, int64_t* status, hipStream_t s) { k_md_flags<<<1, 64, 0, s>>>(sticky, status); }

}  // namespace mpip
