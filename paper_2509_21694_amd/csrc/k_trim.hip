// Receptive-field trimming of a partition share (Methods "Graph
// Partitioning": a root atom's energy after K message-passing layers depends
// only on its K-hop neighbourhood).
//
// With hop(i) the number of edges from atom i to the nearest root atom, layer
// t needs updated features only on atoms with hop <= K - t: layer K only on
// the roots, layer 1 on everything within K - 1 hops.  The share's rows are
// re-ordered so that hop classes are contiguous (class 0 = roots, then hop 1,
// ..., class K = K or more hops, each class in the previous, cell-sorted
// order), which turns "atoms with hop <= K - t" into the row prefix
// [0, n_t) of the receiver CSR; the layer kernels then run over prefixes.
//
// Inside every row the edges whose neighbour is a root are put first, so the
// sender-side last layer (only messages into roots matter) walks a prefix.
//
// Scratch: the per-row stencil blocks (dead once the list is built) hold the
// old node arrays, hop classes and new indices; the rank-count arrays hold
// the per-block class counts; the edge-gradient buffer stages the old edge
// arrays and the receiver array the new edge positions.
#include "kernels.h"

namespace mpip {

namespace {

constexpr int kMaxClass = 17;   // K <= 16 layers: classes 0..K

struct TrimScratch {
  int4* info_o;
  double* pos_o;
  int32_t* spec_o;
  int32_t* perm_o;
  int32_t* rp_o;      // [n + 1]
  uint8_t* own_o;
  int32_t* hop;       // [n] hop class per (old) row
  int32_t* newidx;    // [n] old row -> new row
};

// byte layout inside the [n][28] int32 stencil-block array (112 bytes per row)
TrimScratch trim_scratch(const NbrBuffers& b, int64_t n) {
  char* base = (char*)b.blk;
  TrimScratch t;
  size_t o = 0;
  auto take = [&](size_t bytes) { char* p = base + o; o += (bytes + 15) & ~(size_t)15; return p; };
  t.info_o = (int4*)take(sizeof(int4) * n);
  t.pos_o = (double*)take(sizeof(double) * 3 * n);
  t.spec_o = (int32_t*)take(sizeof(int32_t) * n);
  t.perm_o = (int32_t*)take(sizeof(int32_t) * n);
  t.rp_o = (int32_t*)take(sizeof(int32_t) * (n + 1));
  t.hop = (int32_t*)take(sizeof(int32_t) * n);
  t.newidx = (int32_t*)take(sizeof(int32_t) * n);
  t.own_o = (uint8_t*)take(n);
  return t;
}

__device__ __forceinline__ bool list_bad(const int32_t* row_ptr, int64_t n, int64_t capacity, const int64_t* status) {
  return status[ST_FLAGS] != 0 || (int64_t)row_ptr[n] > capacity;
}

// hop 0 on root atoms, K ("K or more") elsewhere
__global__ void k_hop_init(int64_t n, const uint8_t* __restrict__ owned_s, int K, int32_t* __restrict__ hop) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) hop[i] = owned_s[i] ? 0 : K;
}

// one level of the breadth-first expansion: the neighbours of atoms at hop h
// get hop h + 1 unless they are closer already.  16 lanes per row.  Several
// lanes may store the same value h + 1 into one entry; an entry at hop h is
// never written in this level, so the frontier test is not disturbed.
__global__ __launch_bounds__(256) void k_hop_sweep(int64_t n, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ e_src, int64_t capacity,
                                                   const int64_t* __restrict__ status, int h, int32_t* hop) {
  const int64_t i = blockIdx.x * 16 + (threadIdx.x >> 4);
  if (i >= n || list_bad(row_ptr, n, capacity, status)) return;
  if (hop[i] != h) return;
  for (int e = row_ptr[i] + (threadIdx.x & 15); e < row_ptr[i + 1]; e += 16) {
    const int j = e_src[e];
    if (hop[j] > h + 1) hop[j] = h + 1;
  }
}

// per block of 256 rows, the number of rows of each class: cnt[c * nb + block]
__global__ __launch_bounds__(256) void k_class_count(int64_t n, const int32_t* __restrict__ hop, int K, int64_t nb,
                                                     int32_t* __restrict__ cnt) {
  __shared__ int32_t sc[kMaxClass];
  if (threadIdx.x <= K) sc[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) atomicAdd(&sc[hop[i]], 1);
  __syncthreads();
  if (threadIdx.x <= K) cnt[threadIdx.x * nb + blockIdx.x] = sc[threadIdx.x];
}

// stable partition by class: new row = first slot of (class, block) from the
// class-major exclusive scan of the block counts + rank within the block
__global__ __launch_bounds__(256) void k_class_rank(int64_t n, const int32_t* __restrict__ hop, int K, int64_t nb,
                                                    const int32_t* __restrict__ start, int32_t* __restrict__ newidx) {
  __shared__ int32_t sw[4][kMaxClass];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = blockIdx.x * 256 + threadIdx.x;
  const int c = i < n ? hop[i] : -1;
  int rank = 0;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int q = 0; q <= K; ++q) {
    const uint64_t m = __ballot(c == q);
    if (lane == 0) sw[w][q] = __popcll(m);
    if (c == q) rank = __popcll(m & lt);
  }
  __syncthreads();
  if (i < n) {
    int base = start[c * nb + blockIdx.x];
    for (int v = 0; v < w; ++v) base += sw[v][c];
    newidx[i] = base + rank;
  }
}

// first row of every class (bounds[c], c = 0..K, bounds[K + 1] = n) and
// whether the list is unusable (bounds[K + 2])
__global__ void k_class_bounds(const int32_t* __restrict__ start, int64_t nb, int K, int64_t n,
                               const int32_t* __restrict__ row_ptr, int64_t capacity,
                               const int64_t* __restrict__ status, int64_t* __restrict__ bounds) {
  const int c = threadIdx.x;
  if (c <= K) bounds[c] = (int64_t)start[c * nb];
  if (c == 0) {
    bounds[K + 1] = n;
    bounds[K + 2] = list_bad(row_ptr, n, capacity, status) ? 1 : 0;
  }
}

__global__ void k_save_nodes(int64_t n, const double* __restrict__ pos_s, const int4* __restrict__ info_s,
                             const int32_t* __restrict__ spec_s, const uint8_t* __restrict__ owned_s,
                             const int32_t* __restrict__ perm, const int32_t* __restrict__ row_ptr, TrimScratch t) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i > n) return;
  t.rp_o[i] = row_ptr[i];
  if (i == n) return;
  t.pos_o[3 * i] = pos_s[3 * i];
  t.pos_o[3 * i + 1] = pos_s[3 * i + 1];
  t.pos_o[3 * i + 2] = pos_s[3 * i + 2];
  t.info_o[i] = info_s[i];
  t.spec_o[i] = spec_s[i];
  t.own_o[i] = owned_s[i];
  t.perm_o[i] = perm[i];
}

// node arrays scattered to the new rows; cnt = row lengths in the new order
__global__ void k_perm_nodes(int64_t n, TrimScratch t, double* __restrict__ pos_s, int4* __restrict__ info_s,
                             int32_t* __restrict__ spec_s, uint8_t* __restrict__ owned_s, int32_t* __restrict__ perm,
                             int32_t* __restrict__ inv_perm, int32_t* __restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = t.newidx[i];
  pos_s[3 * (int64_t)k] = t.pos_o[3 * i];
  pos_s[3 * (int64_t)k + 1] = t.pos_o[3 * i + 1];
  pos_s[3 * (int64_t)k + 2] = t.pos_o[3 * i + 2];
  info_s[k] = t.info_o[i];
  spec_s[k] = t.spec_o[i];
  owned_s[k] = t.own_o[i];
  const int p = t.perm_o[i];
  perm[k] = p;
  inv_perm[p] = k;
  cnt[k] = t.rp_o[i + 1] - t.rp_o[i];
}

// (sender, shift, reverse edge) of every edge, staged before the scatter
__global__ void k_save_edges(const int32_t* __restrict__ rp_o, int64_t n, int64_t capacity,
                             const int32_t* __restrict__ e_src, const uint32_t* __restrict__ e_shift,
                             const int32_t* __restrict__ e_rev, int4* __restrict__ tmp) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if ((int64_t)rp_o[n] > capacity || e >= rp_o[n]) return;
  tmp[e] = make_int4(e_src[e], (int)e_shift[e], e_rev[e], 0);
}

__global__ void k_save_vec(const int32_t* __restrict__ rp_o, int64_t n, int64_t capacity,
                           const float4* __restrict__ e_vec, float4* __restrict__ tmp) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if ((int64_t)rp_o[n] > capacity || e >= rp_o[n]) return;
  tmp[e] = e_vec[e];
}

// new position of every edge (epos), 16 lanes per old row: inside its new
// row, the edges whose neighbour is a root come first, each group in the old
// order; root_end[new row] = end of the root group.  The whole wave takes
// part in every ballot (rows of one wave may differ in length).
__global__ __launch_bounds__(256) void k_edge_pos(int64_t n, int64_t capacity, TrimScratch t,
                                                  const int32_t* __restrict__ row_ptr, const int4* __restrict__ tmp,
                                                  int32_t* __restrict__ epos, int32_t* __restrict__ root_end) {
  const int64_t i = blockIdx.x * 16 + (threadIdx.x >> 4);
  const int l16 = threadIdx.x & 15, seg = (threadIdx.x & 63) >> 4;
  const bool ok = i < n && (int64_t)t.rp_o[n] <= capacity;
  const int r0 = ok ? t.rp_o[i] : 0, len = ok ? t.rp_o[i + 1] - r0 : 0;
  const int d0 = ok ? row_ptr[t.newidx[i]] : 0;
  int nr = 0;
  for (int k = l16; k < len; k += 16) nr += (t.hop[tmp[r0 + k].x] == 0) ? 1 : 0;
  for (int off = 8; off > 0; off >>= 1) nr += __shfl_xor(nr, off, 16);
  int top = len;
  top = max(top, __shfl_xor(top, 16));
  top = max(top, __shfl_xor(top, 32));
  const unsigned lt = (1u << l16) - 1u;
  int cr = 0, co = 0;
  for (int b = 0; b < top; b += 16) {
    const bool v = b + l16 < len;
    const bool root = v && t.hop[tmp[r0 + b + l16].x] == 0;
    const unsigned mr = (unsigned)(__ballot(root) >> (16 * seg)) & 0xffffu;
    const unsigned mv = (unsigned)(__ballot(v) >> (16 * seg)) & 0xffffu;
    if (v) epos[r0 + b + l16] = d0 + (root ? cr + __popc(mr & lt) : nr + co + __popc(mv & ~mr & lt));
    cr += __popc(mr);
    co += __popc(mv & ~mr);
  }
  if (ok && l16 == 0) root_end[t.newidx[i]] = d0 + nr;
}

// every edge to its new slot; senders renumbered, reverse edges through epos
__global__ void k_perm_edges(int64_t n, int64_t capacity, TrimScratch t, const int4* __restrict__ tmp,
                             const int32_t* __restrict__ epos, int32_t* __restrict__ e_src,
                             uint32_t* __restrict__ e_shift, int32_t* __restrict__ e_rev) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if ((int64_t)t.rp_o[n] > capacity || e >= t.rp_o[n]) return;
  const int4 v = tmp[e];
  const int ed = epos[e];
  e_src[ed] = t.newidx[v.x];
  e_shift[ed] = (uint32_t)v.y;
  e_rev[ed] = v.z >= 0 ? epos[v.z] : -1;
}

__global__ void k_perm_vec(int64_t n, int64_t capacity, TrimScratch t, const float4* __restrict__ tmp,
                           const int32_t* __restrict__ epos, float4* __restrict__ e_vec) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if ((int64_t)t.rp_o[n] > capacity || e >= t.rp_o[n]) return;
  e_vec[epos[e]] = tmp[e];
}

__global__ void k_zero_edges_from(float4* __restrict__ g, const int32_t* __restrict__ row_ptr, int64_t row0, int64_t n,
                                  int64_t capacity) {
  const int64_t e = row_ptr[row0] + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if ((int64_t)row_ptr[n] > capacity || e >= row_ptr[n]) return;
  g[e] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// g[e] = 0 for the edges past row_end[i] in rows i < n (16 lanes per row)
__global__ __launch_bounds__(256) void k_zero_row_tails(float4* __restrict__ g, const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ row_end, int64_t n, int64_t rows_all,
                                                        int64_t capacity) {
  const int64_t i = blockIdx.x * 16 + (threadIdx.x >> 4);
  if (i >= n || (int64_t)row_ptr[rows_all] > capacity) return;
  for (int e = row_end[i] + (threadIdx.x & 15); e < row_ptr[i + 1]; e += 16) g[e] = make_float4(0.f, 0.f, 0.f, 0.f);
}

}  // namespace

int trim_max_layers() { return kMaxClass - 1; }

void zero_row_tails(float4* g, const int32_t* row_ptr, const int32_t* row_end, int64_t n, int64_t rows_all,
                    int64_t capacity, hipStream_t s) {
  if (n > 0) k_zero_row_tails<<<(unsigned)((n + 15) / 16), 256, 0, s>>>(g, row_ptr, row_end, n, rows_all, capacity);
}

void hop_sweep_launch(const NbrBuffers& b, int64_t n, int h, int64_t capacity, int32_t* hop, hipStream_t s) {
  k_hop_sweep<<<(unsigned)((n + 15) / 16), 256, 0, s>>>(n, b.row_ptr, b.e_src, capacity, b.status, h, hop);
}

const int64_t* trim_classes(const NbrBuffers& b, int64_t n, int K, int64_t capacity, hipStream_t s) {
  const TrimScratch t = trim_scratch(b, n);
  const unsigned g1 = (unsigned)((n + 255) / 256), gw = (unsigned)((n + 15) / 16);
  k_hop_init<<<g1, 256, 0, s>>>(n, b.owned_s, K, t.hop);
  for (int h = 0; h + 1 < K; ++h)
    k_hop_sweep<<<gw, 256, 0, s>>>(n, b.row_ptr, b.e_src, capacity, b.status, h, t.hop);
  const int64_t nb = g1;
  int32_t* cnt = b.rank_count;
  int32_t* start = b.rank_start;
  int64_t* bounds = (int64_t*)(cnt + (((K + 1) * nb + 1) & ~(int64_t)1));
  k_class_count<<<g1, 256, 0, s>>>(n, t.hop, K, nb, cnt);
  exclusive_scan(cnt, (K + 1) * nb, start, b.scan_tmp, s);
  k_class_rank<<<g1, 256, 0, s>>>(n, t.hop, K, nb, start, t.newidx);
  k_class_bounds<<<1, 64, 0, s>>>(start, nb, K, n, b.row_ptr, capacity, b.status, bounds);
  return bounds;
}

void trim_permute(const NbrBuffers& b, int64_t n, int64_t capacity, float4* tmp, hipStream_t s) {
  const TrimScratch t = trim_scratch(b, n);
  const unsigned g1 = (unsigned)((n + 256) / 256), gw = (unsigned)((n + 15) / 16);
  const unsigned ge = (unsigned)((capacity + 255) / 256);
  k_save_nodes<<<g1, 256, 0, s>>>(n, b.pos_s, b.info_s, b.spec_s, b.owned_s, b.perm, b.row_ptr, t);
  k_perm_nodes<<<g1, 256, 0, s>>>(n, t, b.pos_s, b.info_s, b.spec_s, b.owned_s, b.perm, b.inv_perm, b.cnt);
  exclusive_scan(b.cnt, n, b.row_ptr, b.scan_tmp, s);
  if (ge == 0) return;
  // epos in e_dst (rebuilt later where needed), root-group ends in cnt (the
  // row lengths there are consumed by the scan above)
  k_save_edges<<<ge, 256, 0, s>>>(t.rp_o, n, capacity, b.e_src, b.e_shift, b.e_rev, (int4*)tmp);
  k_edge_pos<<<gw, 256, 0, s>>>(n, capacity, t, b.row_ptr, (const int4*)tmp, b.e_dst, b.cnt);
  k_perm_edges<<<ge, 256, 0, s>>>(n, capacity, t, (const int4*)tmp, b.e_dst, b.e_src, b.e_shift, b.e_rev);
  k_save_vec<<<ge, 256, 0, s>>>(t.rp_o, n, capacity, b.e_vec, tmp);
  k_perm_vec<<<ge, 256, 0, s>>>(n, capacity, t, tmp, b.e_dst, b.e_vec);
}

void zero_edges_from(float4* g, const int32_t* row_ptr, int64_t row0, int64_t n, int64_t capacity, hipStream_t s) {
  const unsigned ge = (unsigned)((capacity + 255) / 256);
  if (ge) k_zero_edges_from<<<ge, 256, 0, s>>>(g, row_ptr, row0, n, capacity);
}

}  // namespace mpip
