// Internal interfaces between the host engine and the gfx950 kernels.
#pragma once
#include "common.h"

namespace mpip {

constexpr int kBoundsParts = 1024;

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
  int32_t* bin_start;    // [max_bins+1]
  int32_t* scan_tmp;     // [scan_tmp_elems(max(N, max_bins))]
  int4* info;            // [N] image index (x,y,z) + bin (w), input order
  int32_t* perm;         // [N] sorted position -> input index
  int32_t* inv_perm;     // [N]
  double* pos_s;         // [N,3] raw positions, sorted order
  int4* info_s;          // [N]
  int32_t* spec_s;       // [N]
  uint8_t* owned_s;      // [N]
  int32_t* cnt;          // [N]
  int32_t* row_ptr;      // [N+1]
  int32_t* e_src;        // [cap] sender (sorted index)
  uint32_t* e_shift;     // [cap] S packed as three int8
  float4* e_vec;         // [cap] r_e (FP32 of the FP64 difference), species of sender in .w bits
  int32_t* e_rev;        // [cap]
};

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
  // W3 of the live paths, for t < K (index 0) and t == K (index 1)
  const void* w3f[2];   // forward B operand [p][nt][kc][64][..]
  const void* w3b[2];   // backward A operand [p][mt][kc][64][..]
  const float* cg[2];   // dense coupling tensors of the live paths, concatenated
  // node matrices as [Nout][K] (k contiguous): forward uses W^T, backward W
  const void* up_t[3];   // W_up[l]^T   [C][C]
  const void* up[3];     // W_up[l]     [C][C]
  const void* down_t[3]; // W_down[l]^T [C(1+L) or C][C]
  const void* down[3];   // W_down[l]   [C][C(1+L) or C]
};

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
};

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

struct OutArgs {
  int64_t n;
  const int32_t* row_ptr;
  const float4* e_vec;
  const float4* g;
  const int32_t* e_rev;
  const int32_t* perm;
  const uint8_t* owned_s;
  const double* atom_e;
  int64_t capacity;
  const int64_t* status;
  double* partials;       // [nblocks][10]
  int nblocks;
  double* forces;         // out [N][3] input order
  double* atom_energy;    // out [N] or null
  double* energy;         // out [1]
  double* virial;         // out [9]
};
void launch_outputs(const OutArgs& a, hipStream_t s);
void launch_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace mpip
