// Batched evaluation of many small independent structures in one pass: the
// structures' atoms are concatenated and the neighbour list is built per
// structure, so the CSR is block diagonal and every per-layer kernel runs
// once over all rows of all structures.  Each receiver scans its
// structure's atoms and, per sender, only the periodic images that can lie
// within the cutoff (|S_k| <= img_k); the membership test is the same FP64
// expression as for single structures.  A row lists its edges by sender,
// then image.
#include "kernels.h"

namespace mpip {

__global__ void k_batch_index(const int64_t* __restrict__ ptr, int B, int32_t* __restrict__ sidx) {
  const int b = blockIdx.x;
  if (b >= B) return;
  for (int64_t i = ptr[b] + threadIdx.x; i < ptr[b + 1]; i += blockDim.x) sidx[i] = b;
}

// per atom: image index n_d = floor(x_d / L_d) along periodic axes (0 otherwise);
// validity flags as in the single-structure path
__global__ void k_batch_prep(const double* __restrict__ pos, const int32_t* __restrict__ spec, int64_t n,
                             const int32_t* __restrict__ sidx, const BatchCell* __restrict__ cells, int n_species,
                             int4* __restrict__ info, int32_t* __restrict__ spec_s, uint8_t* __restrict__ owned_s,
                             int32_t* __restrict__ perm, int64_t* __restrict__ status) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const BatchCell c = cells[sidx[i]];
  int nimg[3];
  int bad = 0;
  for (int d = 0; d < 3; ++d) {
    const double x = pos[3 * i + d];
    if (!isfinite(x)) bad |= FL_NONFINITE;
    nimg[d] = (c.pbc[d] && isfinite(x)) ? (int)floor(x / c.L[d]) : 0;
  }
  int sp = spec[i];
  if (sp < 0 || sp >= n_species) bad |= FL_SPECIES;
  spec_s[i] = sp < 0 ? 0 : (sp >= n_species ? n_species - 1 : sp);
  info[i] = make_int4(nimg[0], nimg[1], nimg[2], 0);
  owned_s[i] = 1;
  perm[i] = (int32_t)i;
  if (bad) atomicOr((unsigned long long*)&status[ST_FLAGS], (unsigned long long)bad);
}

#pragma clang fp contract(off)
__device__ __forceinline__ bool batch_pair(const double* xi, const double* xj, const BatchCell& c, int S0, int S1,
                                           int S2, double rc2, double* dxo) {
  double dx[3];
  for (int k = 0; k < 3; ++k) {
    const double s = __dadd_rn(__dadd_rn(__dmul_rn((double)S0, c.cell[0 * 3 + k]), __dmul_rn((double)S1, c.cell[1 * 3 + k])),
                               __dmul_rn((double)S2, c.cell[2 * 3 + k]));
    dx[k] = __dadd_rn(__dsub_rn(xj[k], xi[k]), s);
  }
  const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx[0], dx[0]), __dmul_rn(dx[1], dx[1])), __dmul_rn(dx[2], dx[2]));
  dxo[0] = dx[0]; dxo[1] = dx[1]; dxo[2] = dx[2];
  return d2 < rc2;
}

template <bool FILL>
__global__ void k_batch_nbr(int64_t n, const double* __restrict__ pos, const int4* __restrict__ info,
                            const int32_t* __restrict__ spec_s, const int32_t* __restrict__ sidx,
                            const int64_t* __restrict__ ptr, const BatchCell* __restrict__ cells, double rc,
                            int32_t* __restrict__ cnt, const int32_t* __restrict__ row_ptr, int64_t capacity,
                            int32_t* __restrict__ e_src, uint32_t* __restrict__ e_shift, float4* __restrict__ e_vec,
                            int64_t* __restrict__ status) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (FILL && row_ptr[n] > capacity) return;
  const int b = sidx[i];
  const BatchCell c = cells[b];
  const int64_t j0 = ptr[b], j1 = ptr[b + 1];
  const int4 me = info[i];
  const double xi[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  const double rc2 = rc * rc;
  int count = 0, coincident = 0;
  const int64_t out = FILL ? row_ptr[i] : 0;
  // wrapped coordinates of the receiver, for the image ranges only (the
  // membership test below is the FP64 expression of the full search)
  const int mi[3] = {me.x, me.y, me.z};
  double yi[3], invL[3];
  for (int d = 0; d < 3; ++d) {
    yi[d] = c.pbc[d] ? xi[d] - (double)mi[d] * c.L[d] : 0.0;
    invL[d] = c.pbc[d] ? 1.0 / c.L[d] : 0.0;
  }
  // per sender: along each periodic axis only the images o with
  // |y_j - y_i + o L| < r_c can hold a pair (one or two of -img..img),
  // widened by a slack far above the rounding of the wrapped coordinates
  for (int64_t j = j0; j < j1; ++j) {
    const int4 oj = info[j];
    const double xj[3] = {pos[3 * j], pos[3 * j + 1], pos[3 * j + 2]};
    const int ojn[3] = {oj.x, oj.y, oj.z};
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      if (c.pbc[d]) {
        const double dy = (xj[d] - (double)ojn[d] * c.L[d]) - yi[d];
        lo[d] = max(-c.img[d], (int)ceil((-rc - dy) * invL[d] - 1e-6));
        hi[d] = min(c.img[d], (int)floor((rc - dy) * invL[d] + 1e-6));
      } else {
        lo[d] = 0;
        hi[d] = 0;
      }
    }
    for (int oz = lo[2]; oz <= hi[2]; ++oz)
      for (int oy = lo[1]; oy <= hi[1]; ++oy)
        for (int ox = lo[0]; ox <= hi[0]; ++ox) {
          const int S0 = c.pbc[0] ? ox - oj.x + me.x : 0;
          const int S1 = c.pbc[1] ? oy - oj.y + me.y : 0;
          const int S2 = c.pbc[2] ? oz - oj.z + me.z : 0;
          if (j == i && S0 == 0 && S1 == 0 && S2 == 0) continue;
          double dx[3];
          if (batch_pair(xi, xj, c, S0, S1, S2, rc2, dx)) {
            if (dx[0] == 0.0 && dx[1] == 0.0 && dx[2] == 0.0) coincident = 1;
            if (FILL) {
              const int64_t e = out + count;
              e_src[e] = (int32_t)j;
              e_shift[e] = (uint32_t)(S0 & 0xff) | ((uint32_t)(S1 & 0xff) << 8) | ((uint32_t)(S2 & 0xff) << 16);
              e_vec[e] = make_float4((float)dx[0], (float)dx[1], (float)dx[2], __int_as_float(spec_s[j]));
            }
            ++count;
          }
        }
  }
  if (!FILL) cnt[i] = count;
  if (coincident) atomicOr((unsigned long long*)&status[ST_FLAGS], (unsigned long long)FL_COINCIDENT);
}

__global__ void k_batch_capacity(const int32_t* __restrict__ row_ptr, int64_t n, int64_t capacity,
                                 int64_t* __restrict__ status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int64_t E = row_ptr[n];
    status[ST_NEDGES] = E;
    if (E > capacity) atomicOr((unsigned long long*)&status[ST_FLAGS], (unsigned long long)FL_CAPACITY);
  }
}

void build_neighbors_batch(const NbrBuffers& b, const BatchBuffers& bb, int B, const double* pos,
                           const int32_t* spec, int64_t n, int n_species, double rc, int64_t capacity, hipStream_t s) {
  const int ga = (int)((n + 255) / 256);
  k_batch_index<<<B, 256, 0, s>>>(bb.ptr, B, bb.sidx);
  k_batch_prep<<<ga, 256, 0, s>>>(pos, spec, n, bb.sidx, bb.cells, n_species, b.info_s, b.spec_s, b.owned_s,
                                  b.perm, b.status);
  k_batch_nbr<false><<<ga, 256, 0, s>>>(n, pos, b.info_s, b.spec_s, bb.sidx, bb.ptr, bb.cells, rc, b.cnt, nullptr,
                                        capacity, nullptr, nullptr, nullptr, b.status);
  exclusive_scan(b.cnt, n, b.row_ptr, b.scan_tmp, s);
  k_batch_capacity<<<1, 64, 0, s>>>(b.row_ptr, n, capacity, b.status);
  k_batch_nbr<true><<<ga, 256, 0, s>>>(n, pos, b.info_s, b.spec_s, bb.sidx, bb.ptr, bb.cells, rc, nullptr,
                                       b.row_ptr, capacity, b.e_src, b.e_shift, b.e_vec, b.status);
  reverse_edges(b, n, capacity, false, s);
}

// one block per structure: forces of its atoms, its energy and virial (FP64,
// fixed order); 16 atoms at a time, 16 lanes over each atom's edges
__global__ __launch_bounds__(256) void k_batch_out(int64_t n, const int32_t* __restrict__ row_ptr,
                                                   const float4* __restrict__ e_vec, const float4* __restrict__ g,
                                                   const int32_t* __restrict__ e_rev, const double* __restrict__ atom_e,
                                                   const int64_t* __restrict__ ptr, int64_t capacity,
                                                   const int64_t* __restrict__ status, double* __restrict__ forces,
                                                   double* __restrict__ energy, double* __restrict__ virial) {
  __shared__ double sh[4][10];
  const int b = blockIdx.x, l16 = threadIdx.x & 15, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double loc[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) loc[k] = 0.0;
  const bool run = (status[ST_FLAGS] == 0) && ((int64_t)row_ptr[n] <= capacity);
  if (run) {
    for (int64_t i0 = ptr[b]; i0 < ptr[b + 1]; i0 += 16) {
      const int64_t i = i0 + (threadIdx.x >> 4);
      double F[3] = {0.0, 0.0, 0.0};
      if (i < ptr[b + 1]) {
        for (int e = row_ptr[i] + l16; e < row_ptr[i + 1]; e += 16) {
          const int rv = e_rev[e];
          const float4 ge = g[e];
          const float4 gr = rv >= 0 ? g[rv] : make_float4(0.f, 0.f, 0.f, 0.f);
          const float4 r = e_vec[e];
          F[0] += (double)ge.x - (double)gr.x;
          F[1] += (double)ge.y - (double)gr.y;
          F[2] += (double)ge.z - (double)gr.z;
          const double rr[3] = {r.x, r.y, r.z}, gg[3] = {ge.x, ge.y, ge.z};
#pragma unroll
          for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q) loc[1 + 3 * p + q] += rr[p] * gg[q];
        }
      }
#pragma unroll
      for (int off = 8; off > 0; off >>= 1)
#pragma unroll
        for (int d = 0; d < 3; ++d) F[d] += __shfl_xor(F[d], off);
      if (l16 == 0 && i < ptr[b + 1]) {
        forces[3 * i + 0] = F[0];
        forces[3 * i + 1] = F[1];
        forces[3 * i + 2] = F[2];
        loc[0] += atom_e[i];
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < 10; ++k) loc[k] += __shfl_xor(loc[k], off);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 10; ++k) sh[w][k] = loc[k];
  __syncthreads();
  if (threadIdx.x < 10) {
    const double t = ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) + sh[3][threadIdx.x];
    if (threadIdx.x == 0) energy[b] = t;
    else virial[9 * b + threadIdx.x - 1] = -t;
  }
}

void launch_batch_outputs(int64_t n, int B, const NbrBuffers& nb, const float4* g,
                          const double* atom_e, const BatchBuffers& bb, int64_t capacity, double* forces,
                          double* energy, double* virial, hipStream_t s) {
  k_batch_out<<<B, 256, 0, s>>>(n, nb.row_ptr, nb.e_vec, g, nb.e_rev, atom_e, bb.ptr, capacity, nb.status, forces,
                                energy, virial);
}

}  // namespace mpip
