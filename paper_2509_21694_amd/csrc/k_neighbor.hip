// Cell list and neighbour list (CSR, receiver-sorted) for gfx950.
//
// Atoms are binned by their wrapped position, counting-sorted by bin (ties
// broken by input index, so the order is deterministic), and every later
// kernel works in this spatially sorted order.  Each atom scans the 27
// neighbouring bins (or, along periodic directions too thin for three bins,
// a range of periodic images) and keeps (i, j, S) iff the FP64 test
//   s_k = (S0*cell[0][k] + S1*cell[1][k]) + S2*cell[2][k]
//   dx_k = (x_j[k] - x_i[k]) + s_k,  d2 = (dx0*dx0 + dx1*dx1) + dx2*dx2 < rc*rc
// holds, evaluated on the raw input positions with one rounding per
// operation (no contraction), so the edge set is reproducible bit for bit.
#include "kernels.h"

namespace mpip {

// ---------------------------------------------------------------- scans

// Exclusive scan of n int32 values into out[0..n] (out[n] = total).
// Three launches: per-block sums, one-block scan of the sums, local scans.
static constexpr int kScanBlock = 256, kScanPer = 4, kScanTile = kScanBlock * kScanPer;

__global__ void k_scan_partials(const int32_t* __restrict__ in, int64_t n, int32_t* __restrict__ sums) {
  __shared__ int32_t sh[kScanBlock];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int32_t s = 0;
  for (int k = 0; k < kScanPer; ++k) {
    int64_t idx = base + threadIdx.x * kScanPer + k;
    if (idx < n) s += in[idx];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = kScanBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = sh[0];
}

__global__ void k_scan_sums(int32_t* __restrict__ sums, int64_t nblocks) {
  // single block of kScanBlock threads; sequential carry over chunks
  __shared__ int32_t sh[kScanBlock];
  int32_t carry = 0;
  for (int64_t c0 = 0; c0 < nblocks; c0 += kScanBlock) {
    int64_t idx = c0 + threadIdx.x;
    int32_t v = idx < nblocks ? sums[idx] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
      int32_t t = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (idx < nblocks) sums[idx] = carry + sh[threadIdx.x] - v;  // exclusive
    int32_t tot = sh[kScanBlock - 1];
    __syncthreads();
    carry += tot;
  }
}

__global__ void k_scan_local(const int32_t* __restrict__ in, int64_t n, const int32_t* __restrict__ sums,
                             int32_t* __restrict__ out) {
  __shared__ int32_t sh[kScanBlock];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int32_t v[kScanPer];
  int32_t s = 0;
  for (int k = 0; k < kScanPer; ++k) {
    int64_t idx = base + threadIdx.x * kScanPer + k;
    v[k] = idx < n ? in[idx] : 0;
    s += v[k];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int32_t t = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t run = sums[blockIdx.x] + sh[threadIdx.x] - s;
  for (int k = 0; k < kScanPer; ++k) {
    int64_t idx = base + threadIdx.x * kScanPer + k;
    if (idx < n) out[idx] = run;
    run += v[k];
    if (idx == n - 1) out[n] = run;
  }
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void exclusive_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* tmp, hipStream_t s) {
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) {
    launch_zero(out, sizeof(int32_t), s);
    return;
  }
  k_scan_partials<<<nb, kScanBlock, 0, s>>>(in, n, tmp);
  k_scan_sums<<<1, kScanBlock, 0, s>>>(tmp, nb);
  k_scan_local<<<nb, kScanBlock, 0, s>>>(in, n, tmp, out);
}

// ---------------------------------------------------------------- binning

__global__ void k_bounds(const double* __restrict__ pos, const int32_t* __restrict__ spec, int64_t n,
                         int n_species, double* __restrict__ part, int64_t* __restrict__ status) {
  __shared__ double sh[6][256];
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    for (int d = 0; d < 3; ++d) {
      double x = pos[3 * i + d];
      if (!isfinite(x)) bad |= FL_NONFINITE;
      else { mn[d] = fmin(mn[d], x); mx[d] = fmax(mx[d], x); }
    }
    int sp = spec[i];
    if (sp < 0 || sp >= n_species) bad |= FL_SPECIES;
  }
  if (bad) atomicOr((unsigned long long*)&status[ST_FLAGS], (unsigned long long)bad);
  for (int d = 0; d < 3; ++d) { sh[d][threadIdx.x] = mn[d]; sh[3 + d][threadIdx.x] = mx[d]; }
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + off]);
        sh[3 + d][threadIdx.x] = fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + off]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_grid(const double* __restrict__ part, int nparts, CellInfo ci, int max_bins,
                       GridParams* __restrict__ gp, int64_t* __restrict__ status) {
  // min / max over the partial bounds: lane-strided, then a butterfly (exact in any order)
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (int b = threadIdx.x; b < nparts; b += 64)
    for (int d = 0; d < 3; ++d) {
      mn[d] = fmin(mn[d], part[b * 6 + d]);
      mx[d] = fmax(mx[d], part[b * 6 + 3 + d]);
    }
  for (int off = 32; off > 0; off >>= 1)
    for (int d = 0; d < 3; ++d) {
      mn[d] = fmin(mn[d], __shfl_xor(mn[d], off));
      mx[d] = fmax(mx[d], __shfl_xor(mx[d], off));
    }
  if (threadIdx.x != 0) return;
  const double wmin = ci.rc * (1.0 + 1e-6);
  GridParams g;
  for (int d = 0; d < 3; ++d) {
    g.img[d] = 0;
    if (ci.pbc[d]) {
      double L = ci.L[d];
      int nb = (int)floor(L / wmin);
      g.lo[d] = 0.0;
      g.len[d] = L;
      if (nb >= 3) {
        g.nb[d] = nb; g.stencil[d] = 1; g.inv_bin[d] = (double)nb / L;
      } else {
        g.nb[d] = 1; g.stencil[d] = 0; g.inv_bin[d] = 0.0;
        g.img[d] = (int)ceil(ci.rc / L + 1e-6);   // wrapped positions: |S| < r_c / L + 1
      }
    } else {
      double ext = (mx[d] >= mn[d]) ? (mx[d] - mn[d]) : 0.0;
      int nb = (int)floor(ext / wmin);
      if (nb < 1) nb = 1;
      g.lo[d] = mn[d];
      g.len[d] = ext;
      g.nb[d] = nb; g.stencil[d] = 1;
      g.inv_bin[d] = ext > 0.0 ? (double)nb / ext : 0.0;
    }
  }
  // keep the total bin count within the workspace: widen bins (still >= rc)
  while ((int64_t)g.nb[0] * g.nb[1] * g.nb[2] > max_bins) {
    int d = 0;
    for (int k = 1; k < 3; ++k) if (g.nb[k] > g.nb[d]) d = k;
    int nb = g.nb[d] / 2;
    if (ci.pbc[d] && nb < 3) {
      g.nb[d] = 1; g.stencil[d] = 0; g.inv_bin[d] = 0.0; g.img[d] = (int)ceil(ci.rc / ci.L[d] + 1e-6);
    } else {
      if (nb < 1) nb = 1;
      g.nb[d] = nb;
      g.inv_bin[d] = g.len[d] > 0.0 ? (double)nb / g.len[d] : 0.0;
    }
  }
  g.nbins = g.nb[0] * g.nb[1] * g.nb[2];
  int tot = 0;
  for (int d = 0; d < 3; ++d) {
    int bits = 0;
    while ((1 << bits) < g.nb[d]) ++bits;
    g.mbits[d] = bits;
    tot += bits;
  }
  g.nrank = 1 << tot;
  // FP32 prefilter of the stencil search (orthorhombic cells): with the
  // wrapped positions y (|y| <= Y per component) and per-block shifts s
  // (|s| <= S) rounded to FP32 (unit roundoff u), each component of the FP32
  // difference is within du = u (2Y + 2S + 2|d|) of the exact one, so for
  // |d| <= sqrt(2) r_c the FP32 |d|^2 is within E = du (2 sqrt(6) r_c + 3 du)
  // + 7 u r_c^2 of the exact (and of the FP64) value.  Outside a band of
  // half-width 2E around r_c^2, and above 2E, the FP32 decision is the FP64
  // one; the band (and near-coincident pairs) take the FP64 predicate.
  {
    bool ortho = true;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        if (a != b && ci.cell[3 * a + b] != 0.0) ortho = false;
    double Y = 0.0, S = 0.0;
    for (int d = 0; d < 3; ++d) {
      if (ci.pbc[d]) {
        Y = fmax(Y, fabs(ci.cell[4 * d]) * (1.0 + 1e-6));
        S = fmax(S, fabs(ci.cell[4 * d]));
      } else {
        Y = fmax(Y, fmax(fabs(mn[d]), fabs(mx[d])));
      }
    }
    const double u = 1.0 / 8388608.0;   // 2^-23, twice FP32's unit roundoff
    const double rc = ci.rc;
    const double du = u * (2.0 * Y + 2.0 * S + 2.0 * 1.4142135623730951 * rc);
    const double E = du * (2.0 * 2.449489742783178 * rc + 3.0 * du) + 7.0 * u * rc * rc + 1e-12 * rc * rc;
    const bool finite = isfinite(Y) && Y < 1e7;
    g.pf_rc2 = (float)(rc * rc);
    g.pf_margin = (ortho && finite && 2.0 * E < 0.25 * rc * rc) ? (float)(2.0 * E * 1.01) : -1.0f;
  }
  *gp = g;
  (void)status;
}

// image index n_d (periodic: x = w + n*L with w in [0, L)) and bin id
__global__ void k_bin_assign(const double* __restrict__ pos, int64_t n, CellInfo ci,
                             const GridParams* __restrict__ gp, int4* __restrict__ info,
                             int32_t* __restrict__ bin_count) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  GridParams g = *gp;
  int nimg[3], b[3];
  for (int d = 0; d < 3; ++d) {
    double x = pos[3 * i + d];
    double w;
    if (ci.pbc[d]) {
      double L = ci.L[d];
      double fl = floor(x / L);
      w = x - fl * L;
      nimg[d] = (int)fl;
    } else {
      w = x - g.lo[d];
      nimg[d] = 0;
    }
    int bb = (int)floor(w * g.inv_bin[d]);
    bb = bb < 0 ? 0 : (bb >= g.nb[d] ? g.nb[d] - 1 : bb);
    b[d] = bb;
  }
  int bin = (b[2] * g.nb[1] + b[1]) * g.nb[0] + b[0];
  info[i] = make_int4(nimg[0], nimg[1], nimg[2], bin);
  atomicAdd(&bin_count[bin], 1);
}

// Position of a bin on a Morton (Z-order) curve over the bin grid: the bits of
// the three bin coordinates interleaved from the lowest level up, a dimension
// dropping out once its bits are used.  Sorting atoms by this rank makes any
// contiguous range of rows a compact 3-D region, so the sender rows gathered
// by rows processed together stay within one L2.
__device__ __forceinline__ int bin_rank(int bin, const GridParams& g) {
  const int c[3] = {bin % g.nb[0], (bin / g.nb[0]) % g.nb[1], bin / (g.nb[0] * g.nb[1])};
  int r = 0, pos = 0;
  const int kmax = max(g.mbits[0], max(g.mbits[1], g.mbits[2]));
  for (int k = 0; k < kmax; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (k < g.mbits[d]) {
        r |= ((c[d] >> k) & 1) << pos;
        ++pos;
      }
  return r;
}

__global__ void k_rank_count(const GridParams* __restrict__ gp, const int32_t* __restrict__ bin_count,
                             int32_t* __restrict__ rank_count) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const GridParams g = *gp;
  if (b >= g.nbins) return;
  rank_count[bin_rank(b, g)] = bin_count[b];
}

__global__ void k_bin_start(const GridParams* __restrict__ gp, const int32_t* __restrict__ rank_start,
                            int32_t* __restrict__ bin_start) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const GridParams g = *gp;
  if (b >= g.nbins) return;
  bin_start[b] = rank_start[bin_rank(b, g)];
}

__global__ void k_bin_fill(const int4* __restrict__ info, int64_t n, const int32_t* __restrict__ bin_start,
                           int32_t* __restrict__ cursor, int32_t* __restrict__ bin_atoms) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int bin = info[i].w;
  int slot = atomicAdd(&cursor[bin], 1);
  bin_atoms[bin_start[bin] + slot] = (int32_t)i;
}

// insertion sort of each bin's atoms by input index (deterministic order)
__global__ void k_bin_sort(const GridParams* __restrict__ gp, const int32_t* __restrict__ bin_start,
                           const int32_t* __restrict__ bin_count, int32_t* __restrict__ bin_atoms) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= gp->nbins) return;
  int s = bin_start[b], e = s + bin_count[b];
  for (int k = s + 1; k < e; ++k) {
    int v = bin_atoms[k];
    int q = k - 1;
    while (q >= s && bin_atoms[q] > v) { bin_atoms[q + 1] = bin_atoms[q]; --q; }
    bin_atoms[q + 1] = v;
  }
}

__global__ void k_gather_sorted(const int32_t* __restrict__ perm, int64_t n, const double* __restrict__ pos,
                                const int32_t* __restrict__ spec, const int4* __restrict__ info,
                                int64_t n_owned, int n_species, CellInfo ci, double* __restrict__ pos_s,
                                int4* __restrict__ info_s, float4* __restrict__ ypos_s,
                                int32_t* __restrict__ spec_s, int32_t* __restrict__ inv_perm,
                                uint8_t* __restrict__ owned_s) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  int o = perm[k];
  const double x[3] = {pos[3 * (int64_t)o + 0], pos[3 * (int64_t)o + 1], pos[3 * (int64_t)o + 2]};
  pos_s[3 * k + 0] = x[0];
  pos_s[3 * k + 1] = x[1];
  pos_s[3 * k + 2] = x[2];
  const int4 io = info[o];
  info_s[k] = io;
  // y = x - sum_d image_d cell_d (the image counts are 0 in open dimensions)
  const int im[3] = {io.x, io.y, io.z};
  float y[3];
  for (int c = 0; c < 3; ++c) {
    double v = x[c];
    for (int d = 0; d < 3; ++d)
      if (im[d] != 0) v -= (double)im[d] * ci.cell[3 * d + c];
    y[c] = (float)v;
  }
  ypos_s[k] = make_float4(y[0], y[1], y[2], 0.f);
  int sp = spec[o];  // out-of-range species are flagged by k_bounds; clamp so reads stay in bounds
  spec_s[k] = sp < 0 ? 0 : (sp >= n_species ? n_species - 1 : sp);
  inv_perm[o] = (int32_t)k;
  owned_s[k] = (uint8_t)(o < n_owned ? 1 : 0);
}

// ---------------------------------------------------------------- neighbours

#pragma clang fp contract(off)
__device__ __forceinline__ bool pair_test(const double* __restrict__ xi, const double* __restrict__ xj,
                                          const CellInfo& ci, int S0, int S1, int S2, double rc2,
                                          double* dxo) {
  double dx[3];
  for (int k = 0; k < 3; ++k) {
    double s = __dadd_rn(__dadd_rn(__dmul_rn((double)S0, ci.cell[0 * 3 + k]),
                                   __dmul_rn((double)S1, ci.cell[1 * 3 + k])),
                         __dmul_rn((double)S2, ci.cell[2 * 3 + k]));
    dx[k] = __dadd_rn(__dsub_rn(xj[k], xi[k]), s);
  }
  double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx[0], dx[0]), __dmul_rn(dx[1], dx[1])), __dmul_rn(dx[2], dx[2]));
  dxo[0] = dx[0]; dxo[1] = dx[1]; dxo[2] = dx[2];
  return d2 < rc2;
}

template <bool FILL>
__global__ void k_nbr(int64_t n, const double* __restrict__ pos_s, const int4* __restrict__ info_s,
                      const int32_t* __restrict__ spec_s, CellInfo ci, const GridParams* __restrict__ gp,
                      const int32_t* __restrict__ bin_start, const int32_t* __restrict__ bin_count,
                      int32_t* __restrict__ blk, int32_t* __restrict__ cnt,
                      const int32_t* __restrict__ row_ptr, int64_t capacity, int32_t* __restrict__ e_src,
                      uint32_t* __restrict__ e_shift, float4* __restrict__ e_vec, int64_t* __restrict__ status) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (FILL && row_ptr[n] > capacity) return;
  const GridParams g = *gp;
  if (g.stencil[0] && g.stencil[1] && g.stencil[2]) return;   // k_nbr_w
  const int4 me = info_s[i];
  int bi[3];
  {
    int bin = me.w;
    bi[0] = bin % g.nb[0];
    bi[1] = (bin / g.nb[0]) % g.nb[1];
    bi[2] = bin / (g.nb[0] * g.nb[1]);
  }
  const int ni[3] = {me.x, me.y, me.z};
  double xi[3] = {pos_s[3 * i], pos_s[3 * i + 1], pos_s[3 * i + 2]};
  const double rc2 = ci.rc * ci.rc;
  // stencil dimensions: the bins -1..1 around the atom's; dimensions
  // thinner than three bins (periodic, one bin): per sender, only the
  // images o with |y_j - y_i + o L| < r_c (y the wrapped coordinates), which
  // are one or two of -img..img, widened by a slack far above the rounding
  int lo[3], hi[3];
  double yi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = g.stencil[d] ? -1 : 0;
    hi[d] = g.stencil[d] ? 1 : 0;
    yi[d] = g.stencil[d] ? 0.0 : xi[d] - (double)ni[d] * ci.L[d];
  }
  int count = 0;
  int64_t out = FILL ? row_ptr[i] : 0;
  int coincident = 0;
  const bool stencil3 = false;   // the all-stencil case runs in k_nbr_w
  for (int oz = lo[2]; oz <= hi[2]; ++oz)
    for (int oy = lo[1]; oy <= hi[1]; ++oy)
      for (int ox = lo[0]; ox <= hi[0]; ++ox) {
        int o[3] = {ox, oy, oz};
        int c[3], Sp[3];
        bool skip = false;
        for (int d = 0; d < 3; ++d) {
          if (g.stencil[d]) {
            int cc = bi[d] + o[d];
            Sp[d] = 0;
            if (ci.pbc[d]) {
              if (g.nb[d] < 3) { skip = true; break; }
              if (cc < 0) { cc += g.nb[d]; Sp[d] = -1; }
              else if (cc >= g.nb[d]) { cc -= g.nb[d]; Sp[d] = 1; }
            } else if (cc < 0 || cc >= g.nb[d]) { skip = true; break; }
            c[d] = cc;
          } else {
            c[d] = 0;
            Sp[d] = 0;
          }
        }
        if (skip) continue;
        int bin = (c[2] * g.nb[1] + c[1]) * g.nb[0] + c[0];
        int s = bin_start[bin], e = s + bin_count[bin];
        for (int j = s; j < e; ++j) {
          int4 oj = info_s[j];
          double xj[3] = {pos_s[3 * (int64_t)j], pos_s[3 * (int64_t)j + 1], pos_s[3 * (int64_t)j + 2]};
          const int nj[3] = {oj.x, oj.y, oj.z};
          int ilo[3], ihi[3];
          for (int d = 0; d < 3; ++d) {
            if (g.stencil[d]) {
              ilo[d] = ihi[d] = 0;
            } else {
              const double dy = (xj[d] - (double)nj[d] * ci.L[d]) - yi[d], invL = 1.0 / ci.L[d];
              ilo[d] = max(-g.img[d], (int)ceil((-ci.rc - dy) * invL - 1e-6));
              ihi[d] = min(g.img[d], (int)floor((ci.rc - dy) * invL + 1e-6));
            }
          }
          for (int pz = ilo[2]; pz <= ihi[2]; ++pz)
            for (int py = ilo[1]; py <= ihi[1]; ++py)
              for (int px = ilo[0]; px <= ihi[0]; ++px) {
                int S[3];
                S[0] = ci.pbc[0] ? Sp[0] + px - oj.x + ni[0] : 0;
                S[1] = ci.pbc[1] ? Sp[1] + py - oj.y + ni[1] : 0;
                S[2] = ci.pbc[2] ? Sp[2] + pz - oj.z + ni[2] : 0;
                if (j == i && S[0] == 0 && S[1] == 0 && S[2] == 0) continue;
                double dx[3];
                if (pair_test(xi, xj, ci, S[0], S[1], S[2], rc2, dx)) {
                  if (dx[0] == 0.0 && dx[1] == 0.0 && dx[2] == 0.0) coincident = 1;
                  if (FILL) {
                    int64_t eidx = out + count;
                    e_src[eidx] = j;
                    e_shift[eidx] = (uint32_t)(S[0] & 0xff) | ((uint32_t)(S[1] & 0xff) << 8) |
                                    ((uint32_t)(S[2] & 0xff) << 16);
                    e_vec[eidx] = make_float4((float)dx[0], (float)dx[1], (float)dx[2], __int_as_float(spec_s[j]));
                  }
                  ++count;
                }
              }
        }
      }
  if (!FILL) cnt[i] = count;
  if (FILL && stencil3) blk[28 * i + 27] = count;
  if (coincident) atomicOr((unsigned long long*)&status[ST_FLAGS], (unsigned long long)FL_COINCIDENT);
}

// The same search with one wave per atom when all three dimensions use the
// 27-bin stencil (the bulk case): the candidates of the 27 bins are laid end
// to end and spread over the lanes (a lane finds its bin by a binary search
// in the wave's LDS prefix of bin sizes), tested with the same FP64
// predicate, and the passing ones are compacted with a ballot so each row
// is written contiguously.  Edge order (stencil block, then bin order) and
// the per-block offsets blk are those of k_nbr.
// sShift code of the stencil's central block (Sp = 0)
constexpr int kCenterShift = 1 | (1 << 2) | (1 << 4);

// position of the r-th (from 0) set bit of x; x has more than r set bits
__device__ __forceinline__ int nth_set_bit(unsigned long long x, int r) {
  int pos = 0;
#pragma unroll
  for (int sh = 32; sh > 0; sh >>= 1) {
    const unsigned long long lo = x & ((1ull << sh) - 1ull);
    const int c = __popcll(lo);
    if (r >= c) {
      r -= c;
      x >>= sh;
      pos += sh;
    } else {
      x = lo;
    }
  }
  return pos;
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_nbr_w(int64_t n, const double* __restrict__ pos_s,
                                               const int4* __restrict__ info_s, const float4* __restrict__ ypos_s,
                                               const int32_t* __restrict__ spec_s,
                                               CellInfo ci, const GridParams* __restrict__ gp,
                                               const int32_t* __restrict__ bin_start,
                                               const int32_t* __restrict__ bin_count, int32_t* __restrict__ blk,
                                               int32_t* __restrict__ cnt, const int32_t* __restrict__ row_ptr,
                                               int64_t capacity, int32_t* __restrict__ e_src,
                                               uint32_t* __restrict__ e_shift, float4* __restrict__ e_vec,
                                               uint64_t* __restrict__ cmask, uint32_t* __restrict__ cand,
                                               int64_t* __restrict__ status) {
  __shared__ int sPre[4][28], sStart[4][27], sShift[4][27], sCnt[4][27];
  __shared__ float4 sSf[4][27];   // the blocks' shifts Sp . cell, rounded to FP32 (prefilter)
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * 4 + wv;
  const GridParams g = *gp;
  if (!(g.stencil[0] && g.stencil[1] && g.stencil[2])) return;
  if (i >= n) return;
  if (FILL && row_ptr[n] > capacity) return;
  const int4 me = info_s[i];
  const int bi[3] = {me.w % g.nb[0], (me.w / g.nb[0]) % g.nb[1], me.w / (g.nb[0] * g.nb[1])};
  if (FILL && cand && row_ptr[i + 1] - row_ptr[i] <= kCandList) {
    // the counting pass listed this row's passing candidates (sender, stencil
    // block) in scan order: lane q writes edge q after the FP64 difference
    const int npass = row_ptr[i + 1] - row_ptr[i];
    const int64_t out = row_ptr[i];
    if (lane < 27) sCnt[wv][lane] = 0;
    wave_lds_sync();
    const double xi[3] = {pos_s[3 * i], pos_s[3 * i + 1], pos_s[3 * i + 2]};
    int coincident = 0;
    if (lane < npass) {
      const uint32_t c = cand[i * kCandList + lane];
      const int j = (int)(c >> 5), k = (int)(c & 31u);
      const int o[3] = {k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1};
      const int4 oj = info_s[j];
      const int nj[3] = {oj.x, oj.y, oj.z}, ni[3] = {me.x, me.y, me.z};
      int S[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int cc = bi[d] + o[d];
        const int Sp = cc < 0 ? -1 : (cc >= g.nb[d] ? 1 : 0);
        S[d] = ci.pbc[d] ? Sp - nj[d] + ni[d] : 0;
      }
      const double xj[3] = {pos_s[3 * (int64_t)j], pos_s[3 * (int64_t)j + 1], pos_s[3 * (int64_t)j + 2]};
      double dx[3];
      pair_test(xi, xj, ci, S[0], S[1], S[2], ci.rc * ci.rc, dx);
      if (dx[0] == 0.0 && dx[1] == 0.0 && dx[2] == 0.0) coincident = 1;
      const int64_t eidx = out + lane;
      e_src[eidx] = j;
      e_shift[eidx] = (uint32_t)(S[0] & 0xff) | ((uint32_t)(S[1] & 0xff) << 8) | ((uint32_t)(S[2] & 0xff) << 16);
      e_vec[eidx] = make_float4((float)dx[0], (float)dx[1], (float)dx[2], __int_as_float(spec_s[j]));
      atomicAdd(&sCnt[wv][k], 1);
    }
    wave_lds_sync();
    int cb = lane < 27 ? sCnt[wv][lane] : 0;
    int wsum = cb;
#pragma unroll
    for (int oo = 1; oo < 32; oo <<= 1) {
      const int t = __shfl_up(wsum, oo);
      if (lane >= oo) wsum += t;
    }
    if (lane < 27) blk[28 * i + lane] = wsum - cb;
    if (lane == 0) blk[28 * i + 27] = npass;
    if (__any(coincident) && lane == 0) atomicOr((unsigned long long*)&status[ST_FLAGS], (unsigned long long)FL_COINCIDENT);
    return;
  }
  // lane k < 27: stencil block k = ((oz+1)*3 + (oy+1))*3 + (ox+1)
  int bc = 0;
  if (lane < 27) {
    const int o[3] = {lane % 3 - 1, (lane / 3) % 3 - 1, lane / 9 - 1};
    int c[3], Sp[3];
    bool skip = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int cc = bi[d] + o[d];
      Sp[d] = 0;
      if (ci.pbc[d]) {
        if (g.nb[d] < 3) skip = true;
        if (cc < 0) { cc += g.nb[d]; Sp[d] = -1; }
        else if (cc >= g.nb[d]) { cc -= g.nb[d]; Sp[d] = 1; }
      } else if (cc < 0 || cc >= g.nb[d]) {
        skip = true;
      }
      c[d] = cc;
    }
    int bs = 0;
    if (!skip) {
      const int bin = (c[2] * g.nb[1] + c[1]) * g.nb[0] + c[0];
      bs = bin_start[bin];
      bc = bin_count[bin];
    }
    sStart[wv][lane] = bs;
    sShift[wv][lane] = (Sp[0] + 1) | ((Sp[1] + 1) << 2) | ((Sp[2] + 1) << 4);
    float sf[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      double v = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (Sp[d] != 0) v += (double)Sp[d] * ci.cell[3 * d + cc];
      sf[cc] = (float)v;
    }
    sSf[wv][lane] = make_float4(sf[0], sf[1], sf[2], 0.f);
    sCnt[wv][lane] = 0;
  }
  // exclusive prefix of the bin sizes over lanes 0..26
  int v = bc;
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) {
    const int t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  if (lane < 27) sPre[wv][lane] = v - bc;
  if (lane == 26) sPre[wv][27] = v;
  const int total = __shfl(v, 26);
  wave_lds_sync();
  const double xi[3] = {pos_s[3 * i], pos_s[3 * i + 1], pos_s[3 * i + 2]};
  const double rc2 = ci.rc * ci.rc;
  const bool pf_on = g.pf_margin >= 0.f;
  const float4 yi = ypos_s[i];
  const int64_t out = FILL ? row_ptr[i] : 0;
  int count = 0, coincident = 0;
  // candidate f: stencil block k (last with pre[k] <= f; empty bins share the
  // prefix of the next one), atom j, shift S; pass / dx from the FP64 test
  auto candidate = [&](int f, int& j, int& k, int* S, double* dx) -> bool {
    k = 0;
#pragma unroll
    for (int step = 16; step > 0; step >>= 1)
      if (k + step < 27 && sPre[wv][k + step] <= f) k += step;
    j = sStart[wv][k] + (f - sPre[wv][k]);
    const int sc = sShift[wv][k];
    const int Sp[3] = {(sc & 3) - 1, ((sc >> 2) & 3) - 1, ((sc >> 4) & 3) - 1};
    const int4 oj = info_s[j];
    S[0] = ci.pbc[0] ? Sp[0] - oj.x + me.x : 0;
    S[1] = ci.pbc[1] ? Sp[1] - oj.y + me.y : 0;
    S[2] = ci.pbc[2] ? Sp[2] - oj.z + me.z : 0;
    if (j == i && S[0] == 0 && S[1] == 0 && S[2] == 0) return false;
    const double xj[3] = {pos_s[3 * (int64_t)j], pos_s[3 * (int64_t)j + 1], pos_s[3 * (int64_t)j + 2]};
    return pair_test(xi, xj, ci, S[0], S[1], S[2], rc2, dx);
  };
  if (FILL && total <= 64 * kCandWords) {
    // the counting pass kept which candidates passed: lane q takes the q-th
    // passing candidate (ascending f, the order of the full scan) and only
    // the passing pairs are evaluated again (for their FP64 difference)
    const int nw = (total + 63) >> 6;
    const unsigned long long mine = lane < nw ? cmask[(int64_t)i * kCandWords + lane] : 0ull;
    int incl = __popcll(mine);
#pragma unroll
    for (int o = 1; o < kCandWords; o <<= 1) {
      const int t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    unsigned long long wd[kCandWords];
    int ex[kCandWords];
#pragma unroll
    for (int t = 0; t < kCandWords; ++t) {
      wd[t] = __shfl(mine, t);
      ex[t] = __shfl(incl, t) - __popcll(wd[t]);
    }
    const int npass = __shfl(incl, kCandWords - 1);
    for (int q0 = 0; q0 < npass; q0 += 64) {
      const int q = q0 + lane;
      bool pass = false;
      int j = 0, k = 0, S[3] = {0, 0, 0};
      double dx[3] = {0.0, 0.0, 0.0};
      if (q < npass) {
        int w = 0;
        unsigned long long word = wd[0];
        int rank = q - ex[0];
#pragma unroll
        for (int t = 1; t < kCandWords; ++t)
          if (t < nw && ex[t] <= q) { w = t; word = wd[t]; rank = q - ex[t]; }
        pass = candidate(64 * w + nth_set_bit(word, rank), j, k, S, dx);
        if (pass && dx[0] == 0.0 && dx[1] == 0.0 && dx[2] == 0.0) coincident = 1;
      }
      if (pass) {
        const int64_t eidx = out + q;
        e_src[eidx] = j;
        e_shift[eidx] = (uint32_t)(S[0] & 0xff) | ((uint32_t)(S[1] & 0xff) << 8) | ((uint32_t)(S[2] & 0xff) << 16);
        e_vec[eidx] = make_float4((float)dx[0], (float)dx[1], (float)dx[2], __int_as_float(spec_s[j]));
        atomicAdd(&sCnt[wv][k], 1);
      }
    }
    count = npass;
  } else
  for (int base = 0; base < total; base += 64) {
    const int f = base + lane;
    bool pass = false;
    int j = 0, k = 0, S[3] = {0, 0, 0};
    double dx[3] = {0.0, 0.0, 0.0};
    if (f < total) {
      // largest k with pre[k] <= f (empty bins share the prefix of the next one)
#pragma unroll
      for (int step = 16; step > 0; step >>= 1)
        if (k + step < 27 && sPre[wv][k + step] <= f) k += step;
      j = sStart[wv][k] + (f - sPre[wv][k]);
      const int sc = sShift[wv][k];
      // counting pass: the FP32 prefilter decides outside its band
      int decided = 0;   // 1 pass, -1 fail, 0 FP64 predicate
      if (!FILL && pf_on) {
        const float4 yj = ypos_s[j], sf = sSf[wv][k];
        const float d0 = (yj.x - yi.x) + sf.x, d1 = (yj.y - yi.y) + sf.y, d2 = (yj.z - yi.z) + sf.z;
        const float q = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
        if (j == i && sc == kCenterShift) decided = -1;   // the atom itself (S = 0)
        else if (q > g.pf_rc2 + g.pf_margin) decided = -1;
        else if (q < g.pf_rc2 - g.pf_margin && q > g.pf_margin) decided = 1;
      }
      if (decided != 0) {
        pass = decided > 0;
      } else {
        const int Sp[3] = {(sc & 3) - 1, ((sc >> 2) & 3) - 1, ((sc >> 4) & 3) - 1};
        const int4 oj = info_s[j];
        S[0] = ci.pbc[0] ? Sp[0] - oj.x + me.x : 0;
        S[1] = ci.pbc[1] ? Sp[1] - oj.y + me.y : 0;
        S[2] = ci.pbc[2] ? Sp[2] - oj.z + me.z : 0;
        if (!(j == i && S[0] == 0 && S[1] == 0 && S[2] == 0)) {
          const double xj[3] = {pos_s[3 * (int64_t)j], pos_s[3 * (int64_t)j + 1], pos_s[3 * (int64_t)j + 2]};
          pass = pair_test(xi, xj, ci, S[0], S[1], S[2], rc2, dx);
          if (pass && dx[0] == 0.0 && dx[1] == 0.0 && dx[2] == 0.0) coincident = 1;
        }
      }
    }
    const unsigned long long m = __ballot(pass);
    if (!FILL && lane == 0 && (base >> 6) < kCandWords) cmask[(int64_t)i * kCandWords + (base >> 6)] = m;
    if (!FILL && cand && pass) {
      const int slot = count + __popcll(m & ((1ull << lane) - 1ull));
      if (slot < kCandList) cand[i * kCandList + slot] = ((uint32_t)j << 5) | (uint32_t)k;
    }
    if (FILL && pass) {
      const int64_t eidx = out + count + __popcll(m & ((1ull << lane) - 1ull));
      e_src[eidx] = j;
      e_shift[eidx] = (uint32_t)(S[0] & 0xff) | ((uint32_t)(S[1] & 0xff) << 8) | ((uint32_t)(S[2] & 0xff) << 16);
      e_vec[eidx] = make_float4((float)dx[0], (float)dx[1], (float)dx[2], __int_as_float(spec_s[j]));
      atomicAdd(&sCnt[wv][k], 1);
    }
    count += __popcll(m);
  }
  if (FILL) {
    wave_lds_sync();
    // blk: edges of the row before each stencil block, then the row total
    int c = lane < 27 ? sCnt[wv][lane] : 0;
    int w = c;
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
      const int t = __shfl_up(w, o);
      if (lane >= o) w += t;
    }
    if (lane < 27) blk[28 * i + lane] = w - c;
    if (lane == 0) blk[28 * i + 27] = count;
  } else if (lane == 0) {
    cnt[i] = count;
  }
  if (__any(coincident) && lane == 0) atomicOr((unsigned long long*)&status[ST_FLAGS], (unsigned long long)FL_COINCIDENT);
}

__global__ void k_check_capacity(const int32_t* __restrict__ row_ptr, int64_t n, int64_t capacity,
                                 int64_t* __restrict__ status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int64_t E = row_ptr[n];
    status[ST_NEDGES] = E;
    if (E > capacity) atomicOr((unsigned long long*)&status[ST_FLAGS], (unsigned long long)FL_CAPACITY);
  }
}

// Reverse edges, one search per pair: of the two edges (i, j, S) and
// (j, i, -S), the one whose sender index is larger (for an atom's own image,
// the one whose first nonzero shift component is positive) finds its partner
// in the sender's row and writes both entries (e_rev starts at -1).  16
// lanes per row.
__global__ __launch_bounds__(256) void k_nbr_rev(int64_t n, const int32_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ e_src,
                                                 const uint32_t* __restrict__ e_shift, const int4* __restrict__ info_s,
                                                 const GridParams* __restrict__ gp, const int32_t* __restrict__ blk,
                                                 int64_t capacity, int32_t* __restrict__ e_rev) {
  const int64_t i = blockIdx.x * 16 + (threadIdx.x >> 4);
  const int l16 = threadIdx.x & 15;
  if (i >= n) return;
  if (row_ptr[n] > capacity) return;
  // gp null (batched lists): no stencil blocks, the whole row j is searched
  GridParams g{};
  if (gp) g = *gp;
  const bool stencil3 = gp && g.stencil[0] && g.stencil[1] && g.stencil[2];
  int bi[3] = {0, 0, 0};
  if (stencil3) {
    const int bin = info_s[i].w;
    bi[0] = bin % g.nb[0]; bi[1] = (bin / g.nb[0]) % g.nb[1]; bi[2] = bin / (g.nb[0] * g.nb[1]);
  }
  for (int e = row_ptr[i] + l16; e < row_ptr[i + 1]; e += 16) {
    const int j = e_src[e];
    const uint32_t sh = e_shift[e];
    const int S0 = (int8_t)(sh & 0xff), S1 = (int8_t)((sh >> 8) & 0xff), S2 = (int8_t)((sh >> 16) & 0xff);
    const bool owner = (j != (int)i) ? (j > (int)i) : (S0 != 0 ? S0 > 0 : (S1 != 0 ? S1 > 0 : S2 > 0));
    if (!owner) continue;
    const uint32_t want = (uint32_t)((-S0) & 0xff) | ((uint32_t)((-S1) & 0xff) << 8) | ((uint32_t)((-S2) & 0xff) << 16);
    int f0 = row_ptr[j], f1 = row_ptr[j + 1];
    if (stencil3) {
      // the reverse edge sits in row j's block of stencil offset -o, o = bin(j) - bin(i)
      const int bin = info_s[j].w;
      const int bj[3] = {bin % g.nb[0], (bin / g.nb[0]) % g.nb[1], bin / (g.nb[0] * g.nb[1])};
      int k = 0;
#pragma unroll
      for (int d = 2; d >= 0; --d) {
        int o = bj[d] - bi[d];
        if (o > 1) o -= g.nb[d];        // periodic wrap (nb >= 3 with a stencil)
        else if (o < -1) o += g.nb[d];
        k = 3 * k + (1 - o);
      }
      f1 = f0 + blk[28 * (int64_t)j + k + 1];
      f0 = f0 + blk[28 * (int64_t)j + k];
    }
    int r = -1;
    for (int f = f0; f < f1; ++f)
      if (e_src[f] == (int)i && e_shift[f] == want) { r = f; break; }
    e_rev[e] = r;
    if (r >= 0) e_rev[r] = e;
  }
}

// export in input indices
__global__ void k_nbr_export(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ e_src,
                             const uint32_t* __restrict__ e_shift, const int32_t* __restrict__ perm, int64_t capacity,
                             int32_t* __restrict__ oi, int32_t* __restrict__ oj, int32_t* __restrict__ os) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (row_ptr[n] > capacity) return;
  for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    uint32_t sh = e_shift[e];
    oi[e] = perm[i];
    oj[e] = perm[e_src[e]];
    os[3 * (int64_t)e + 0] = (int8_t)(sh & 0xff);
    os[3 * (int64_t)e + 1] = (int8_t)((sh >> 8) & 0xff);
    os[3 * (int64_t)e + 2] = (int8_t)((sh >> 16) & 0xff);
  }
}

// ---------------------------------------------------------------- list reuse
// A list built with a larger radius r_c + skin (the "superset": rows sup_row,
// senders sup_src, shifts sup_shift, reverse edges sup_rev) stays valid while
// no atom has moved more than skin/2: every pair now closer than r_c is in it
// with the same image shift.  Each evaluation then re-applies the FP64
// predicate d < r_c to the superset's (i, j, S) at the current positions and
// compacts the kept edges, in superset order, into the working list.

// sorted positions from the input positions (the permutation of the build)
__global__ void k_refresh_sorted(const double* __restrict__ pos, const int32_t* __restrict__ perm, int64_t n,
                                 double* __restrict__ pos_s) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t o = perm[k];
  pos_s[3 * k] = pos[3 * o];
  pos_s[3 * k + 1] = pos[3 * o + 1];
  pos_s[3 * k + 2] = pos[3 * o + 2];
}

// one wave per row: keep flag of every superset edge (in map) and the row's count
__global__ __launch_bounds__(256) void k_skin_count(int64_t n, const double* __restrict__ pos_s, CellInfo ci,
                                                    const int32_t* __restrict__ sup_row,
                                                    const int32_t* __restrict__ sup_src,
                                                    const uint32_t* __restrict__ sup_shift, int64_t sup_cap,
                                                    int32_t* __restrict__ map, int32_t* __restrict__ cnt,
                                                    int64_t* __restrict__ status) {
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n || sup_row[n] > sup_cap) return;
  const double xi[3] = {pos_s[3 * i], pos_s[3 * i + 1], pos_s[3 * i + 2]};
  const double rc2 = ci.rc * ci.rc;
  int count = 0, coincident = 0;
  for (int e0 = sup_row[i]; e0 < sup_row[i + 1]; e0 += 64) {
    const int e = e0 + lane;
    bool keep = false;
    if (e < sup_row[i + 1]) {
      const int64_t j = sup_src[e];
      const uint32_t sh = sup_shift[e];
      const double xj[3] = {pos_s[3 * j], pos_s[3 * j + 1], pos_s[3 * j + 2]};
      double dx[3];
      keep = pair_test(xi, xj, ci, (int8_t)(sh & 0xff), (int8_t)((sh >> 8) & 0xff), (int8_t)((sh >> 16) & 0xff), rc2, dx);
      if (keep && dx[0] == 0.0 && dx[1] == 0.0 && dx[2] == 0.0) coincident = 1;
      map[e] = keep ? 1 : 0;
    }
    count += __popcll(__ballot(keep));
  }
  if (lane == 0) cnt[i] = count;
  if (__any(coincident) && lane == 0) atomicOr((unsigned long long*)&status[ST_FLAGS], (unsigned long long)FL_COINCIDENT);
}

// one wave per row: kept edges written in superset order; map[e] becomes the
// working index of superset edge e (or -1)
__global__ __launch_bounds__(256) void k_skin_fill(int64_t n, const double* __restrict__ pos_s,
                                                   const int32_t* __restrict__ spec_s, CellInfo ci,
                                                   const int32_t* __restrict__ sup_row,
                                                   const int32_t* __restrict__ sup_src,
                                                   const uint32_t* __restrict__ sup_shift, int64_t sup_cap,
                                                   const int32_t* __restrict__ row_ptr, int64_t capacity,
                                                   int32_t* __restrict__ map, int32_t* __restrict__ e_src,
                                                   uint32_t* __restrict__ e_shift, float4* __restrict__ e_vec) {
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n || sup_row[n] > sup_cap || row_ptr[n] > capacity) return;
  const double xi[3] = {pos_s[3 * i], pos_s[3 * i + 1], pos_s[3 * i + 2]};
  int64_t out = row_ptr[i];
  for (int e0 = sup_row[i]; e0 < sup_row[i + 1]; e0 += 64) {
    const int e = e0 + lane;
    const bool in = e < sup_row[i + 1];
    const bool keep = in && map[e] != 0;
    const unsigned long long m = __ballot(keep);
    if (keep) {
      const int64_t k = out + __popcll(m & ((1ull << lane) - 1ull));
      const int32_t j = sup_src[e];
      const uint32_t sh = sup_shift[e];
      const int S0 = (int8_t)(sh & 0xff), S1 = (int8_t)((sh >> 8) & 0xff), S2 = (int8_t)((sh >> 16) & 0xff);
      const double xj[3] = {pos_s[3 * (int64_t)j], pos_s[3 * (int64_t)j + 1], pos_s[3 * (int64_t)j + 2]};
      double dx[3];
      pair_test(xi, xj, ci, S0, S1, S2, 0.0, dx);
      e_src[k] = j;
      e_shift[k] = sh;
      e_vec[k] = make_float4((float)dx[0], (float)dx[1], (float)dx[2], __int_as_float(spec_s[j]));
      map[e] = (int32_t)k;
    } else if (in) {
      map[e] = -1;
    }
    out += __popcll(m);
  }
}

// reverse edges of the working list through the superset's
__global__ void k_skin_rev(int64_t n, const int32_t* __restrict__ sup_row, const int32_t* __restrict__ sup_rev,
                           int64_t sup_cap, const int32_t* __restrict__ map, const int32_t* __restrict__ row_ptr,
                           int64_t capacity, int32_t* __restrict__ e_rev) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (sup_row[n] > sup_cap || row_ptr[n] > capacity || e >= sup_row[n]) return;
  const int k = map[e];
  if (k < 0) return;
  const int r = sup_rev[e];
  e_rev[k] = r >= 0 ? map[r] : -1;
}

void refresh_sorted(const NbrBuffers& b, const double* pos, int64_t n, hipStream_t s) {
  k_refresh_sorted<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(pos, b.perm, n, b.pos_s);
}

void compact_list(const NbrBuffers& b, const NbrBuffers& sup, int64_t sup_cap, int32_t* map, const CellInfo& ci,
                  int64_t n, int64_t capacity, hipStream_t s) {
  const unsigned gw = (unsigned)((n + 3) / 4);
  k_skin_count<<<gw, 256, 0, s>>>(n, b.pos_s, ci, sup.row_ptr, sup.e_src, sup.e_shift, sup_cap, map, b.cnt, b.status);
  exclusive_scan(b.cnt, n, b.row_ptr, b.scan_tmp, s);
  k_check_capacity<<<1, 64, 0, s>>>(b.row_ptr, n, capacity, b.status);
  k_skin_fill<<<gw, 256, 0, s>>>(n, b.pos_s, b.spec_s, ci, sup.row_ptr, sup.e_src, sup.e_shift, sup_cap, b.row_ptr,
                                 capacity, map, b.e_src, b.e_shift, b.e_vec);
  k_skin_rev<<<(unsigned)((sup_cap + 255) / 256), 256, 0, s>>>(n, sup.row_ptr, sup.e_rev, sup_cap, map, b.row_ptr,
                                                               capacity, b.e_rev);
}

// ---------------------------------------------------------------- driver

void build_neighbors(const NbrBuffers& b, const mpip_system& sys, const CellInfo& ci, int64_t capacity,
                     hipStream_t s) {
  const int64_t n = sys.n_atoms;
  const int nblk = 256;
  int nparts = (int)((n + 255) / 256);
  if (nparts > kBoundsParts) nparts = kBoundsParts;
  k_bounds<<<nparts, 256, 0, s>>>(sys.positions, sys.species, n, ci.n_species, b.bounds, b.status);
  k_grid<<<1, 64, 0, s>>>(b.bounds, nparts, ci, b.max_bins, b.grid, b.status);
  launch_zero(b.bin_count, sizeof(int32_t) * (b.max_bins + 1), s);
  launch_zero(b.bin_cursor, sizeof(int32_t) * (b.max_bins + 1), s);
  const int ga = (int)((n + nblk - 1) / nblk);
  k_bin_assign<<<ga, nblk, 0, s>>>(sys.positions, n, ci, b.grid, b.info, b.bin_count);
  // bins laid out along a Morton curve: counts in rank order, scan, back to bins
  const int64_t nr = 8 * (int64_t)b.max_bins;
  launch_zero(b.rank_count, sizeof(int32_t) * (nr + 1), s);
  const unsigned gb = (unsigned)((b.max_bins + 255) / 256);
  k_rank_count<<<gb, 256, 0, s>>>(b.grid, b.bin_count, b.rank_count);
  exclusive_scan(b.rank_count, nr, b.rank_start, b.scan_tmp, s);
  k_bin_start<<<gb, 256, 0, s>>>(b.grid, b.rank_start, b.bin_start);
  k_bin_fill<<<ga, nblk, 0, s>>>(b.info, n, b.bin_start, b.bin_cursor, b.perm);
  k_bin_sort<<<gb, 256, 0, s>>>(b.grid, b.bin_start, b.bin_count, b.perm);
  k_gather_sorted<<<ga, nblk, 0, s>>>(b.perm, n, sys.positions, sys.species, b.info, sys.n_owned, ci.n_species, ci,
                                      b.pos_s, b.info_s, b.ypos_s, b.spec_s, b.inv_perm, b.owned_s);
  // one of each pair does the work: k_nbr_w when all dimensions use the 27-bin stencil, else k_nbr
  const unsigned gw = (unsigned)((n + 3) / 4);
  k_nbr_w<false><<<gw, 256, 0, s>>>(n, b.pos_s, b.info_s, b.ypos_s, b.spec_s, ci, b.grid, b.bin_start, b.bin_count, nullptr, b.cnt,
                                    nullptr, capacity, nullptr, nullptr, nullptr, b.cmask, b.cand, b.status);
  k_nbr<false><<<ga, nblk, 0, s>>>(n, b.pos_s, b.info_s, b.spec_s, ci, b.grid, b.bin_start, b.bin_count, nullptr, b.cnt, nullptr,
                                   capacity, nullptr, nullptr, nullptr, b.status);
  exclusive_scan(b.cnt, n, b.row_ptr, b.scan_tmp, s);
  k_check_capacity<<<1, 64, 0, s>>>(b.row_ptr, n, capacity, b.status);
  k_nbr_w<true><<<gw, 256, 0, s>>>(n, b.pos_s, b.info_s, b.ypos_s, b.spec_s, ci, b.grid, b.bin_start, b.bin_count, b.blk, nullptr,
                                   b.row_ptr, capacity, b.e_src, b.e_shift, b.e_vec, b.cmask, b.cand, b.status);
  k_nbr<true><<<ga, nblk, 0, s>>>(n, b.pos_s, b.info_s, b.spec_s, ci, b.grid, b.bin_start, b.bin_count, b.blk, nullptr, b.row_ptr,
                                  capacity, b.e_src, b.e_shift, b.e_vec, b.status);
  reverse_edges(b, n, capacity, true, s);
}

void reverse_edges(const NbrBuffers& b, int64_t n, int64_t capacity, bool blocks, hipStream_t s) {
  launch_fill32(b.e_rev, 0xffffffffu, sizeof(int32_t) * (size_t)capacity, s);
  k_nbr_rev<<<(unsigned)((n + 15) / 16), 256, 0, s>>>(n, b.row_ptr, b.e_src, b.e_shift, b.info_s,
                                                       blocks ? b.grid : nullptr, b.blk, capacity, b.e_rev);
}

void export_neighbors(const NbrBuffers& b, int64_t n, int64_t capacity, int32_t* oi, int32_t* oj, int32_t* os,
                      hipStream_t s) {
  const int ga = (int)((n + 255) / 256);
  k_nbr_export<<<ga, 256, 0, s>>>(n, b.row_ptr, b.e_src, b.e_shift, b.perm, capacity, oi, oj, os);
}

}  // namespace mpip
