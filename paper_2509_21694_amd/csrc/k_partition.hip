// Graph partitioning on the GPU: stage-1 spatial grid along one axis and the
// halo of periodic images within `halo` of the slab (Methods, "Graph
// Partitioning"), and the accumulation of a partition's force rows into the
// full structure (Methods, "Global Output Integration").
//
// Arithmetic of the membership tests (FP64, one rounding per operation):
//   x  = p - floor(p / Lx) * Lx          wrapped coordinate along the axis
//   b  = min(floor((x / Lx) * P), P - 1) stage-1 bin
//   lo = part * Lx / P, hi = (part + 1) * Lx / P
//   image s of atom a is a halo atom iff xs = x + s * Lx lies in
//   [lo - halo, lo) or [hi, hi + halo), and (s != 0 or b != part).
// Local order: root atoms by increasing index, then halo images by
// increasing s, then by increasing index.
#include "kernels.h"

namespace mpip {

#pragma clang fp contract(off)
__device__ __forceinline__ void slab_wrap(double p, double Lx, int P, double* x, int* b) {
  const double fl = floor(__ddiv_rn(p, Lx));
  const double xw = __dsub_rn(p, __dmul_rn(fl, Lx));
  int bb = (int)floor(__dmul_rn(__ddiv_rn(xw, Lx), (double)P));
  bb = bb < 0 ? 0 : (bb > P - 1 ? P - 1 : bb);
  *x = xw;
  *b = bb;
}

// flags[c * n + a] = 1 iff atom a belongs to category c (0: root, 1 + k: image s = k - nimg)
__global__ void k_slab_flags(const double* __restrict__ pos, int64_t n, SlabArgs sa, int32_t* __restrict__ flags) {
  const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  double x;
  int b;
  slab_wrap(pos[3 * a + sa.axis], sa.L, sa.P, &x, &b);
  const double lo = __ddiv_rn(__dmul_rn((double)sa.part, sa.L), (double)sa.P);
  const double hi = __ddiv_rn(__dmul_rn((double)(sa.part + 1), sa.L), (double)sa.P);
  flags[a] = (b == sa.part) ? 1 : 0;
  for (int k = 0; k < 2 * sa.nimg + 1; ++k) {
    const int s = k - sa.nimg;
    const double xs = __dadd_rn(x, __dmul_rn((double)s, sa.L));
    bool in = ((xs >= __dsub_rn(lo, sa.halo)) && (xs < lo)) || ((xs >= hi) && (xs < __dadd_rn(hi, sa.halo)));
    if (s == 0 && b == sa.part) in = false;
    if (sa.hop && sa.hop[a] > sa.max_hop) in = false;
    flags[(int64_t)(1 + k) * n + a] = in ? 1 : 0;
  }
}

__global__ void k_slab_write(const double* __restrict__ pos, const int32_t* __restrict__ spec, int64_t n,
                             SlabArgs sa, const int32_t* __restrict__ flags, const int32_t* __restrict__ offs,
                             const int64_t* __restrict__ base, double* __restrict__ out_pos,
                             int32_t* __restrict__ out_spec, int32_t* __restrict__ out_idx) {
  const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  double x;
  int b;
  slab_wrap(pos[3 * a + sa.axis], sa.L, sa.P, &x, &b);
  for (int c = 0; c < 2 * sa.nimg + 2; ++c) {
    if (!flags[(int64_t)c * n + a]) continue;
    const int64_t slot = base[c] + offs[(int64_t)c * (n + 1) + a];
    if (slot >= sa.capacity) continue;
    const double xs = (c == 0) ? x : __dadd_rn(x, __dmul_rn((double)(c - 1 - sa.nimg), sa.L));
    for (int d = 0; d < 3; ++d) out_pos[3 * slot + d] = (d == sa.axis) ? xs : pos[3 * a + d];
    out_spec[slot] = spec[a];
    out_idx[slot] = (int32_t)a;
  }
}

void slab_share_launch(const double* pos, const int32_t* spec, int64_t n, const SlabArgs& sa, int32_t* flags,
                       int32_t* offs, int32_t* scan_tmp, hipStream_t s) {
  const int g = (int)((n + 255) / 256);
  k_slab_flags<<<g, 256, 0, s>>>(pos, n, sa, flags);
  for (int c = 0; c < 2 * sa.nimg + 2; ++c)
    exclusive_scan(flags + (int64_t)c * n, n, offs + (int64_t)c * (n + 1), scan_tmp, s);
}

void slab_write_launch(const double* pos, const int32_t* spec, int64_t n, const SlabArgs& sa, const int32_t* flags,
                       const int32_t* offs, const int64_t* base, double* out_pos, int32_t* out_spec,
                       int32_t* out_idx, hipStream_t s) {
  const int g = (int)((n + 255) / 256);
  k_slab_write<<<g, 256, 0, s>>>(pos, spec, n, sa, flags, offs, base, out_pos, out_spec, out_idx);
}

// dst[index[k]] += src[k] (rows of 3 doubles)
__global__ void k_accumulate_rows(const double* __restrict__ src, const int32_t* __restrict__ index, int64_t n,
                                  int64_t n_dst, double* __restrict__ dst) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t o = index[k];
  if (o < 0 || o >= n_dst) return;
  for (int d = 0; d < 3; ++d) atomicAdd(&dst[3 * o + d], src[3 * k + d]);
}

void accumulate_rows_launch(const double* src, const int32_t* index, int64_t n, int64_t n_dst, double* dst,
                            hipStream_t s) {
  if (n <= 0) return;
  k_accumulate_rows<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, index, n, n_dst, dst);
}

// graph halo (Methods "Graph Partitioning", stage 2 as a breadth-first
// expansion): hop 0 on the atoms of slab sa.part, K + 1 elsewhere (sorted rows)
__global__ void k_bfs_roots(const double* __restrict__ pos_s, int64_t n, SlabArgs sa, int K, int32_t* __restrict__ hop) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  double x;
  int b;
  slab_wrap(pos_s[3 * r + sa.axis], sa.L, sa.P, &x, &b);
  hop[r] = (b == sa.part) ? 0 : K + 1;
}

__global__ void k_hop_to_input(int64_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ hop_sorted,
                               int32_t* __restrict__ hop_in) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r < n) hop_in[perm[r]] = hop_sorted[r];
}

void bfs_hops_launch(const NbrBuffers& b, int64_t n, const SlabArgs& sa, int K, int64_t capacity, int32_t* hop_sorted,
                     int32_t* hop_in, hipStream_t s) {
  const unsigned g = (unsigned)((n + 255) / 256);
  k_bfs_roots<<<g, 256, 0, s>>>(b.pos_s, n, sa, K, hop_sorted);
  for (int h = 0; h < K; ++h) hop_sweep_launch(b, n, h, capacity, hop_sorted, s);
  k_hop_to_input<<<g, 256, 0, s>>>(n, b.perm, hop_sorted, hop_in);
}

// E += e, W += w: one partition's root energy and virial into the totals
__global__ void k_add_energy_virial(const double* __restrict__ e, const double* __restrict__ w, double* __restrict__ E,
                                    double* __restrict__ W) {
  const int k = threadIdx.x;
  if (k == 0) E[0] += e[0];
  if (k < 9) W[k] += w[k];
}

void add_energy_virial_launch(const double* e, const double* w, double* E, double* W, hipStream_t s) {
  k_add_energy_virial<<<1, 64, 0, s>>>(e, w, E, W);
}

// dst[index[k]] = src[k] for the first n rows (root-atom energies)
__global__ void k_scatter_scalars(const double* __restrict__ src, const int32_t* __restrict__ index, int64_t n,
                                  int64_t n_dst, double* __restrict__ dst) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t o = index[k];
  if (o >= 0 && o < n_dst) dst[o] = src[k];
}

void scatter_scalars_launch(const double* src, const int32_t* index, int64_t n, int64_t n_dst, double* dst,
                            hipStream_t s) {
  if (n <= 0) return;
  k_scatter_scalars<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, index, n, n_dst, dst);
}

}  // namespace mpip
