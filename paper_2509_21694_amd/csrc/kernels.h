// Internal interfaces between the host engine and the gfx950 kernels.
#pragma once
#include "common.h"

namespace mpip {

constexpr int kBoundsParts = 1024;
constexpr int kCandWords = 8;   // atoms with more than 64 kCandWords candidates test them again when filling
constexpr int kCandList = 64;   // rows of at most this many edges are filled from the counting pass's list

struct CellInfo {
  double cell[9];
  double L[3];       // diagonal of an orthorhombic cell
  int pbc[3];
  double rc;
  int n_species;
};

struct NbrBuffers {
  int64_t* status;       // [ST_WORDS]
  double* bounds;        // [kBoundsParts*6]
  GridParams* grid;      // [1]
  int max_bins;
  int32_t* bin_count;    // [max_bins+1]
  int32_t* bin_cursor;   // [max_bins+1]
  int32_t* bin_start;    // [max_bins+1] first sorted slot of each bin (bins laid out in curve order)
  int32_t* rank_count;   // [8*max_bins+1] bin counts in curve-rank order, then their exclusive scan
  int32_t* rank_start;   // [8*max_bins+1]
  int32_t* scan_tmp;     // [scan_tmp_elems(max(N, 8*max_bins))]
  int4* info;            // [N] image index (x,y,z) + bin (w), input order
  int32_t* perm;         // [N] sorted position -> input index
  int32_t* inv_perm;     // [N]
  double* pos_s;         // [N,3] raw positions, sorted order
  float4* ypos_s;        // [N] the positions minus their cell images, rounded to FP32 (prefilter)
  int4* info_s;          // [N]
  int32_t* spec_s;       // [N]
  uint8_t* owned_s;      // [N]
  int32_t* cnt;          // [N]
  int32_t* row_ptr;      // [N+1]
  int32_t* blk;          // [N][28] start of each of the 27 stencil-offset blocks within a row, and its end
  uint64_t* cmask;       // [N][kCandWords] candidate pass masks of the counting pass (64 candidates a word)
  uint32_t* cand;        // [N][kCandList] the counting pass's passing candidates in scan order,
                         // sender << 5 | stencil block (null when N >= 2^27)
  int32_t* e_src;        // [cap] sender (sorted index)
  uint32_t* e_shift;     // [cap] S packed as three int8
  float4* e_vec;         // [cap] r_e (FP32 of the FP64 difference), species of sender in .w bits
  int32_t* e_rev;        // [cap]
  int32_t* e_dst;        // [cap] scratch of the receptive-field trimming
};

// neighbour-list reuse within a skin: sorted positions refreshed from the
// input positions, and the working list (in b) compacted from a list built
// with a larger radius (row_ptr, e_src, e_shift, e_rev of `sup`) by the FP64
// predicate at ci.rc; map: [sup_cap] scratch
void refresh_sorted(const NbrBuffers& b, const double* pos, int64_t n, hipStream_t s);
void compact_list(const NbrBuffers& b, const NbrBuffers& sup, int64_t sup_cap, int32_t* map, const CellInfo& ci,
                  int64_t n, int64_t capacity, hipStream_t s);

// receptive-field trimming of a partition share (k_trim.hip): hop classes
// from the root atoms (owned_s) over the built list, K - 1 breadth-first
// levels (class K = K or more hops); returns a device array bounds[0..K+2]:
// first row of each class in the class-sorted order, n, and 1 if the list is
// unusable (then nothing may be permuted).  Needs n >= trim_min_atoms().
const int64_t* trim_classes(const NbrBuffers& b, int64_t n, int K, int64_t capacity, hipStream_t s);
// re-orders the rows (node arrays, CSR, senders, reverse edges) by class,
// and inside every row puts the edges whose neighbour is a root first; the
// end of that group per row is left in b.cnt.  tmp: [capacity] float4
// scratch (b.e_dst is used as scratch too)
void trim_permute(const NbrBuffers& b, int64_t n, int64_t capacity, float4* tmp, hipStream_t s);
// g[e] = 0 for the edges of rows row0 .. n-1
void zero_edges_from(float4* g, const int32_t* row_ptr, int64_t row0, int64_t n, int64_t capacity, hipStream_t s);
int trim_max_layers();
// g[e] = 0 for the edges of rows i < n past row_end[i] (rows_all: rows of the list)
void zero_row_tails(float4* g, const int32_t* row_ptr, const int32_t* row_end, int64_t n, int64_t rows_all,
                    int64_t capacity, hipStream_t s);
// one breadth-first level: neighbours of rows at hop h get min(hop, h + 1)
void hop_sweep_launch(const NbrBuffers& b, int64_t n, int h, int64_t capacity, int32_t* hop, hipStream_t s);
constexpr int64_t trim_min_atoms() { return 64; }

int64_t scan_tmp_elems(int64_t n);
void exclusive_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* tmp, hipStream_t s);
void build_neighbors(const NbrBuffers& b, const mpip_system& sys, const CellInfo& ci, int64_t capacity,
                     hipStream_t s);
void export_neighbors(const NbrBuffers& b, int64_t n, int64_t capacity, int32_t* oi, int32_t* oj, int32_t* os,
                      hipStream_t s);

// ------------------------------------------------------------------ layers

enum LayerKind { KIND_ONLY = 0, KIND_FIRST = 1, KIND_MID = 2, KIND_LAST = 3 };

// Device weights of one layer in the operand layouts used by the kernels.
// "A"/"B" refer to the MFMA operand the array feeds; bf16 arrays hold 8
// values per lane and k-chunk, f32 arrays one value.
struct LayerDev {
  // radial MLP, forward (transposed orientation: features x edges)
  const void* w1a;   // [4 mt][kc][64 lanes] x (8 bf16 | 1 f32)
  const void* w2a;   // [4 mt][kc][64][..]
  // radial MLP, backward
  const void* w2b;   // [4 mt][kc][64][..]
  const void* w1b;   // [kc][64][..]
  // BF16 form: the MLP's second hidden layer tabulated over [0, r_c]
  // (edge_common.h: rad_pos), [kRadTab][64] BF16 (value, increment) pairs
  const uint32_t* rtab;
  // W3 of the live paths, for t < K (index 0) and t == K (index 1)
  const void* w3f[2];   // forward B operand [p][nt][kc][64][..]
  const void* w3b[2];   // backward A operand [p][mt][kc][64][..]
  const float* cg[2];   // dense coupling tensors of the live paths, concatenated
  // node matrices as [Nout][K] (k contiguous): forward uses W^T, backward W
  const void* up_t[3];   // W_up[l]^T   [C][C]
  const void* up[3];     // W_up[l]     [C][C]
  const void* down_t[3]; // W_down[l]^T [C(1+L) or C][C]
  const void* down[3];   // W_down[l]   [C][C(1+L) or C]
  // specialised first / last layer kernels (k_fast.hip)
  const void* w2f;       // layer-2 B operand, edges x features orientation [nt 4][kc][64]
  const void* w3fp[2];   // layer-3 B operand, channel of (tile nt, col n) = (C/16) n + nt
  const void* w3t[2];    // layer-3 A operand, features x edges; channel of row rho in tile mt
                         //   = 32 (mt/2) + 8 (rho/4) + 4 (mt%2) + rho%4
  const void* w3bp[2];   // MLP-adjoint A operand; k-slot (g, j) of chunk kc = channel 32 kc + 8 g + j
  // first layer, species factorisation: V_l[(s,k)][c] = ht1[s][c] W3[k][(l,c)] / n_avg
  const void* vt[3];     // [C][S*64]  (A = Q V)
  const void* v[3];      // [S*64][C]  (P = dA V^T)
  // V_l folded with the down projection: z_l = Q_l (V_l W_down_l), P_l = zbar_l (V_l W_down_l)^T
  const void* vwt[3];    // [Nz_l][S*64]  (Nz_0 = C(1+L), Nz_l = C)
  const void* vw[3];     // [S*64][Nz_l]
  // fused node kernels between the first and a last second layer (BF16 form,
  // k_node1.hip), all as MFMA A operands [row tile][k chunk][64 lanes][8]:
  const void* n1_vwt[3];   // (V_l W_down_l)^T: rows z features, k = (s, k) in order
  const void* n1_upt[3];   // next layer's W_up_l^T: rows output channel (C/4)(r/4) + 4 mt + r%4, k permuted
  const void* n1_up[3];    // next layer's W_up_l: rows channel, k = channel in order
  const void* n1_vw[3];    // V_l W_down_l: rows (s, k) as (S*16)(r/4) + 4 mt + r%4, k = z feature permuted per C block
  const void* nk_dt;       // last layer, W_down's scalar block transposed: rows z feature, k = channel in order
  const void* nk_d;        // last layer, W_down's scalar block (/ n_avg): rows channel, k = z feature permuted
  // FP32 form, sender-side last layer (k_fast32.hip): row-major copies with odd row strides
  const float* w1r;        // W1 [n_basis 8][65]
  const float* w2r;        // W2 [64][65] (rows the layer input)
  const float* w3r;        // W3 of the last layer's live paths [64][P C + 1]
};

struct Node1Args {
  int64_t n;
  const void* Q;          // [N][nlm][64 S] bf16 (forward input; adjoint: recompute of z)
  void* P;                // [N][nlm][64 S] bf16 (adjoint output, may alias Q)
  float* h;               // [N][nlm][C]: forward writes h_0 (l = 0 rows) only
  void* ht;               // [N][nlm][C] bf16: next layer's h~ (forward output)
  const void* htbar;      // [N][nlm][C] bf16: next layer's h~bar (adjoint input)
  const int32_t* spec_s;
  const uint8_t* owned_s;
  const float* emb;       // [S][C]
  const float* w_read;    // [C]
  const void* vwt[3];
  const void* upt[3];
  const void* up[3];
  const void* vw[3];
};
void launch_node1(bool fwd, int C, int L, int S, const Node1Args& a, hipStream_t s);

// the last layer's node update, readout and their adjoint in one pass (BF16 form)
struct NodeKArgs {
  int64_t n;
  int nlm;
  float* A;               // [N][C]: the message sums in (unless msg), dE/dA out (same rows)
  // when set, the per-edge BF16 messages [E][C] in receiver-side CSR slots:
  // A_i = inv_n sum_{e in row i} msg[e] is formed here instead of read from A
  const unsigned short* msg;
  const int32_t* row_ptr;
  float inv_n;
  const float* h;         // [N][nlm][C]: the previous layer's h_0 rows
  const float* w_read;    // [C]
  const float* e0;        // [S]
  const int32_t* spec_s;
  const uint8_t* owned_s;
  double* atom_e;         // [N]
  const void* dt;         // LayerDev::nk_dt
  const void* d;          // LayerDev::nk_d
};
void launch_nodeK(int C, const NodeKArgs& a, hipStream_t s);

// molecular dynamics (k_md.hip): the two halves of a BAOAB / velocity-Verlet
// step around the force evaluation, and the per-step energy record
void md_first(int64_t n, double* x, double* v, const double* f, const int32_t* spec, const double* masses, double dt,
              double friction, double temperature, uint64_t seed, int64_t step, const double* xref, double thr2,
              int64_t* moved, hipStream_t s);
void md_reference(int64_t n, const double* x, double* xref, int64_t* moved, hipStream_t s);
void md_second(int64_t n, double* v, const double* f, const int32_t* spec, const double* masses, double dt,
               double* partials, hipStream_t s);
void md_record(const double* partials, int nblocks, const double* energy, const int64_t* status, double* epot,
               double* ekin, int64_t* sticky, hipStream_t s);
void md_flags(const int64_t* sticky, int64_t* status, hipStream_t s);

struct FastArgs {
  int64_t n;
  const int32_t* row_ptr;
  const int32_t* e_src;
  const int32_t* e_dst;  // receiver of each edge (edge-parallel adjoint a)
  const int32_t* e_rev;  // reverse edge (fused adjoint of the last layer)
  const float4* e_vec;
  int64_t capacity;
  const int64_t* status;
  float rc;
  int envelope_p;
  int n_species;
  float inv_n;
  const void* w1a;
  const void* w2a;
  const void* w2b;
  const void* w1b;
  const void* w2f;
  const void* w3f;       // permuted (w3fp)
  const void* w3t;
  const void* w3b;       // permuted (w3bp)
  const float* w1r;      // FP32 row-major copies (k_fast32.hip)
  const float* w2r;
  const float* w3r;
  const uint32_t* rtab;  // BF16 form: radial table of the layer (LayerDev::rtab)
  float rtab_scale;      // kRadTab / r_c
  const float* cg;
  float* Q;              // first layer forward: [N][nlm][S*64]
  const float* P;        // first layer adjoint: [N][nlm][S*64]
  const void* ht;        // last layer: [N][nlm][C], bf16 (BF16 form) or f32
  float* A;              // last layer forward: [N][C]
  const float* Abar;     // last layer adjoint input: [N][C]
  float* htbar;          // last layer adjoint output: [N][nlm][C]
  int htbar_bf16;        // 1: htbar stored as bf16 (same element offsets)
  float4* g;
  void* msg;             // last layer forward, BF16 form: messages [E][C] bf16 in CSR order
  // When set (two specialised layers, BF16 form): the fused last-layer adjoint
  // writes dE/dr of each edge's reverse into the edge's own slot of g2p, and
  // the first-layer adjoint, which runs after it, writes h_e = (its own
  // dE/dr_e) - g2p[e] to g (so g needs no clearing).  With
  // dE/dr_e = g1_e + g2p[rev(e)] and r_rev(e) = -r_e, the forces
  // sum_e (dE/dr_e - dE/dr_rev(e)) equal sum_e (h_e - h_rev(e)) and the virial
  // -sum_e r_e (x) dE/dr_e equals -sum_e r_e (x) h_e: the outputs read g as
  // when both layers accumulate into it.  Otherwise both accumulate into g.
  float4* g2p;
  // null, or per row the end of the edges whose receivers need the last
  // layer (a trimmed share's rows list them first): the sender-side last
  // layer (messages and fused adjoint) walks [row_ptr[i], row_end[i])
  const int32_t* row_end;
};

void launch_l1(int prec, int L, bool fwd, const FastArgs& a, hipStream_t s);
// which: 0 forward, 1 adjoint (dR, dY, MLP), 2 adjoint (sender-side pull),
// 3 both adjoints fused over the reverse edges, 4 forward as sender-side
// messages, 5 their segmented sum into A (3, 4 and 5: BF16 form only)
void launch_l2(int prec, int C, int L, int which, const FastArgs& a, hipStream_t s);
// last layer of the FP32 form, sender side (C = 64 or 128): which = 0 messages
// (FP32, into msg), 1 their sum into A, 2 the fused adjoint
void launch_l2_32(int C, int L, int which, const FastArgs& a, hipStream_t s);

struct EdgeArgs {
  int64_t n;               // atoms
  const int32_t* row_ptr;
  const int32_t* e_src;
  const float4* e_vec;
  const int32_t* spec_s;
  int64_t capacity;
  const int64_t* status;
  float rc;
  float inv_n;
  int envelope_p;
  // layer data
  const void* w1a;
  const void* w2a;
  const void* w2b;
  const void* w1b;
  const void* w3f;
  const void* w3b;
  const float* cg;
  const float* ht;         // FIRST/ONLY: species table [S][C]; else [N][nlm][C]
  float* A;                // forward output [N][nlm_out][C]
  const float* Abar;       // backward input [N][nlm_out][C] (scaled by inv_n in-kernel)
  float* htbar;            // backward output [N][nlm][C] (t >= 2)
  float4* g;               // backward: dE/dr_e accumulated over layers [cap]
  float* part;             // middle-layer adjoint: per-edge sums handed between launches [cap][kPartStride]
};
constexpr int kPartStride = 80;   // 64 MLP-adjoint inputs + up to 16 dE/dY

void launch_edge_fwd(int prec, int C, int L, int kind, const EdgeArgs& a, hipStream_t s);
void launch_edge_bwd(int prec, int C, int L, int kind, const EdgeArgs& a, hipStream_t s);

// Y[r, :] (=|+=) X[r, :] @ W for rows r < M; X row r at x + (r/rpa)*xs + (r%rpa)*xr,
// Y row r at y + (r/rpa)*ys + (r%rpa)*yr; W given as wt[Nout][ldw] (k contiguous).
struct GemmArgs {
  const float* x; int64_t xs; int64_t xr;
  float* y; int64_t ys; int64_t yr;
  int64_t M; int rpa;
  int K; int Nout; int ldw;
  const void* wt;
  int accumulate;
  int y_bf16;            // 1: y is bf16 (uint16) storage with the same strides
  int x_bf16;            // 1: x is bf16 (uint16) storage with the same strides (BF16 form only)
};
void launch_gemm(int prec, const GemmArgs& g, hipStream_t s);

struct NodeArgs {
  int64_t n;
  int C, L, nlm;
  const int32_t* spec_s;
  const uint8_t* owned_s;
  const float* emb;       // [S][C]
  const float* w_read;    // [C]
  const float* e0;        // [S]
  float* h;               // [N][nlm][C]
  float* z0;              // [N][C(1+L)]
  float* zl;              // [N][nlm-1][C]
  float* hbar;            // [N][nlm][C]
  double* atom_e;         // [N]
};
void launch_gate_fwd(const NodeArgs& a, int first, int last, hipStream_t s);
void launch_readout(const NodeArgs& a, hipStream_t s);
void launch_gate_bwd(const NodeArgs& a, int last, int init_hbar, hipStream_t s);

// rows per workgroup of the force / virial output pass
constexpr int kOutRowsPerBlock = 64;

struct OutArgs {
  int64_t n;
  const int32_t* row_ptr;
  const float4* e_vec;
  const float4* g;        // dE/dr_e, or h_e (see FastArgs::g2p): same forces and virial
  const int32_t* e_rev;
  const int32_t* perm;
  const uint8_t* owned_s;
  const double* atom_e;
  int64_t capacity;
  const int64_t* status;
  double* partials;       // [nblocks][10], nblocks = ceil(n / kOutRowsPerBlock)
  int nblocks;
  double* forces;         // out [N][3] input order
  double* atom_energy;    // out [N] or null
  double* energy;         // out [1]
  double* virial;         // out [9]
};
void launch_outputs(const OutArgs& a, hipStream_t s);

// ------------------------------------------------------------------ batches
struct BatchCell {
  double cell[9];
  double L[3];
  int pbc[3];
  int img[3];     // periodic images searched: -img..img per axis (0 if not periodic)
};
struct BatchBuffers {
  const int64_t* ptr;      // [B+1] atom offsets (device copy)
  const BatchCell* cells;  // [B]
  int32_t* sidx;           // [N] structure of each atom
};
// e_rev of a built list: -1, then for each edge pair (i, j, S) / (j, i, -S)
// the pair's owner searches row j (its stencil block of it when blocks) and
// writes both entries
void reverse_edges(const NbrBuffers& b, int64_t n, int64_t capacity, bool blocks, hipStream_t s);
void build_neighbors_batch(const NbrBuffers& b, const BatchBuffers& bb, int B, const double* pos,
                           const int32_t* spec, int64_t n, int n_species, double rc, int64_t capacity, hipStream_t s);
void launch_batch_outputs(int64_t n, int B, const NbrBuffers& nb, const float4* g,
                          const double* atom_e, const BatchBuffers& bb, int64_t capacity, double* forces,
                          double* energy, double* virial, hipStream_t s);

// ------------------------------------------------------------------ partitions
struct SlabArgs {
  int axis;
  int P;          // number of slabs
  int part;       // this slab
  int nimg;       // periodic images -nimg..nimg considered for the halo
  double L;       // cell length along the axis
  double halo;    // halo depth
  int64_t capacity;
  // graph halo: keep a halo image only if its atom is within max_hop hops of
  // a root (hop per input atom); null: every image in the geometric halo
  const int32_t* hop = nullptr;
  int max_hop = 0;
};
// hop distances for a graph halo over a built list (sorted rows): roots =
// atoms of slab sa.part; K breadth-first levels; result per input atom in
// hop_in (K + 1 = farther than K hops)
void bfs_hops_launch(const NbrBuffers& b, int64_t n, const SlabArgs& sa, int K, int64_t capacity, int32_t* hop_sorted,
                     int32_t* hop_in, hipStream_t s);
void slab_share_launch(const double* pos, const int32_t* spec, int64_t n, const SlabArgs& sa, int32_t* flags,
                       int32_t* offs, int32_t* scan_tmp, hipStream_t s);
void slab_write_launch(const double* pos, const int32_t* spec, int64_t n, const SlabArgs& sa, const int32_t* flags,
                       const int32_t* offs, const int64_t* base, double* out_pos, int32_t* out_spec,
                       int32_t* out_idx, hipStream_t s);
void accumulate_rows_launch(const double* src, const int32_t* index, int64_t n, int64_t n_dst, double* dst,
                            hipStream_t s);
void add_energy_virial_launch(const double* e, const double* w, double* E, double* W, hipStream_t s);
void scatter_scalars_launch(const double* src, const int32_t* index, int64_t n, int64_t n_dst, double* dst,
                            hipStream_t s);
void launch_zero(void* p, size_t bytes, hipStream_t s);
// p[0 .. n-1] *= f
void launch_scale(float* p, float f, int64_t n, hipStream_t s);
// fill `bytes` (a multiple of 4) with a 32-bit pattern
void launch_fill32(void* p, uint32_t value, size_t bytes, hipStream_t s);

}  // namespace mpip
