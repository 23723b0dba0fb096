// Shared device/host definitions of libmpip (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpip.h"

namespace mpip {

constexpr int kWave = 64;
constexpr int kTileE = 16;      // edges per MFMA tile (16x16 MFMA shapes)
constexpr int kHidden = 64;     // radial MLP hidden width (fixed in this library)
constexpr int kNB = 8;          // radial basis size (fixed in this library)
constexpr int kRadTab = MPIP_RADIAL_TABLE_INTERVALS;   // intervals of the BF16 form's radial table over [0, r_c]
constexpr int kMaxNlm = 9;      // (l_max+1)^2 for l_max <= 2

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// Status word layout in the workspace (int64 each).
enum { ST_CODE = 0, ST_NEDGES = 1, ST_FLAGS = 2, ST_WORDS = 8 };
// Data-dependent error flags (bit mask in ST_FLAGS).
enum { FL_CAPACITY = 1, FL_SPECIES = 2, FL_NONFINITE = 4, FL_COINCIDENT = 8, FL_BINS = 16 };

// Geometry of the cell list, computed on the device.
struct GridParams {
  double lo[3];        // origin of bin 0 per dimension (periodic: 0)
  double len[3];       // periodic: cell length; non-periodic: covered extent
  double inv_bin[3];   // 1 / bin width
  int nb[3];           // bins per dimension
  int img[3];          // periodic dims with fewer than 3 bins: images -img..img
  int stencil[3];      // 1: use -1..1 neighbour bins, 0: single bin + image loop
  int nbins;
  int mbits[3];        // bits per dimension of the bins' space-filling-curve rank
  int nrank;           // size of the rank space, 2^(mbits[0]+mbits[1]+mbits[2])
  float pf_rc2;        // r_c^2 in FP32, and the half-width of the band around it (and above 0) in
  float pf_margin;     // which the FP32 prefilter defers to the FP64 predicate; < 0: prefilter off
};

// ---- MFMA wrappers (16x16 output tile, 64 lanes) --------------------------
// Operand lane layout (verified on gfx950): A[row = lane%16][k-slot],
// B[k-slot][col = lane%16], where the k-slot of register j in lane group
// g = lane/16 is the same for A and B; D[row = 4*g + r][col = lane%16].
__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// NT tiles of 64 x 16 bytes, contiguous at src, copied into LDS at dst by
// the whole workgroup with direct global -> LDS loads (each wave copies whole
// tiles: lane k of a load lands at byte 16 k of the tile).  No data passes
// through registers and every load of the copy is in flight at once; call
// lds_dma_sync() before the tiles are read.
template <int NT, typename T>
__device__ __forceinline__ void lds_dma_tiles(T* dst, const T* src) {
  static_assert(sizeof(T) == 16, "16-byte elements");
  const int lane = threadIdx.x & 63, nw = (int)(blockDim.x >> 6);
  for (int t = (int)(threadIdx.x >> 6); t < NT; t += nw)
    __builtin_amdgcn_global_load_lds((const void*)(src + (size_t)t * 64 + lane),
                                     (__attribute__((address_space(3))) void*)(dst + t * 64), 16, 0, 0);
}
// this wave's direct loads landed, then a workgroup barrier
__device__ __forceinline__ void lds_dma_sync() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// LDS written by some lanes of a wave and read by others of the same wave
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// logistic function with the hardware reciprocal (1 ulp) instead of an IEEE division
__device__ __forceinline__ float sigm(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }
__device__ __forceinline__ float silu(float x) { return x * sigm(x); }
__device__ __forceinline__ float dsilu(float x) {
  float s = sigm(x);
  return s * (1.0f + x * (1.0f - s));
}

}  // namespace mpip
