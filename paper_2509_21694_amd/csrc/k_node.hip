// Node-side kernels: channel-mixing GEMMs on MFMA, gated non-linearity with
// residual, readout, their adjoints, and the final force / virial / energy
// reductions (fixed-order, FP64).
#include "kernels.h"

namespace mpip {

// ------------------------------------------------------------ GEMM
// One wave computes 16 rows x 64 output columns; a block of 4 waves covers
// 64 rows.  A operand: lane (g, r) holds row r, k-slots 8g..8g+7 (bf16) or
// 4q+g (f32); B operand from wt[n][k] with the same k-slots.

template <int PREC>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs a) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, rr = lane & 15;
  const int64_t r = ((int64_t)blockIdx.x * 4 + w) * 16 + rr;
  const int n0 = blockIdx.y * 64;
  const bool rv = r < a.M;
  const float* xrow = nullptr;
  const __bf16* xbrow = nullptr;
  if (rv) {
    xrow = a.x + (r / a.rpa) * a.xs + (r % a.rpa) * a.xr;
    xbrow = (const __bf16*)a.x + (r / a.rpa) * a.xs + (r % a.rpa) * a.xr;
  }
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
  const int ntl = (a.Nout - n0) >= 64 ? 4 : (a.Nout - n0) / 16;
  if constexpr (PREC == 1) {
    const __bf16* W = (const __bf16*)a.wt;
    for (int k0 = 0; k0 < a.K; k0 += 32) {
      bf16x8 av;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        av[j] = rv ? (a.x_bf16 ? xbrow[k0 + 8 * g + j] : (__bf16)xrow[k0 + 8 * g + j]) : (__bf16)0.f;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < ntl) {
          const int n = n0 + 16 * t + rr;
          bf16x8 bv = *(const bf16x8*)(W + (int64_t)n * a.ldw + k0 + 8 * g);
          acc[t] = mfma_bf16(av, bv, acc[t]);
        }
      }
    }
  } else {
    const float* W = (const float*)a.wt;
    for (int k0 = 0; k0 < a.K; k0 += 4) {
      const float av = rv ? xrow[k0 + g] : 0.f;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < ntl) {
          const int n = n0 + 16 * t + rr;
          acc[t] = mfma_f32(av, W[(int64_t)n * a.ldw + k0 + g], acc[t]);
        }
      }
    }
  }
  // D: lane (g, col rr) holds rows 4g + q of the wave's 16-row tile
  const int64_t rbase = ((int64_t)blockIdx.x * 4 + w) * 16;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t ro = rbase + 4 * g + q;
    if (ro >= a.M) continue;
    const int64_t yo = (ro / a.rpa) * a.ys + (ro % a.rpa) * a.yr;
    float* yrow = a.y + yo;
    __bf16* ybrow = (__bf16*)a.y + yo;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < ntl) {
        const int n = n0 + 16 * t + rr;
        if (a.y_bf16) ybrow[n] = (__bf16)acc[t][q];
        else if (a.accumulate) yrow[n] += acc[t][q];
        else yrow[n] = acc[t][q];
      }
    }
  }
}

// Weight-stationary GEMM: the block stages its NT x 16 columns of W in LDS
// once (as MFMA B operands), then its 4 waves stream 16-row tiles of X
// (grid-stride over row tiles), so W is read from L2 once per block.
template <int PREC, int NT>
__global__ __launch_bounds__(256) void k_gemm_lds(GemmArgs a, int64_t row_tiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, rr = lane & 15;
  const int KCH = (PREC == 1) ? a.K / 32 : a.K / 4;
  const int n0 = blockIdx.y * NT * 16;
  if constexpr (PREC == 1) {
    bf16x8* sb = (bf16x8*)smem;
    const __bf16* W = (const __bf16*)a.wt;
    for (int idx = threadIdx.x; idx < NT * KCH * 64; idx += 256) {
      const int l = idx & 63, kc = (idx >> 6) % KCH, nt = (idx >> 6) / KCH;
      const int n = n0 + 16 * nt + (l & 15);
      sb[idx] = *(const bf16x8*)(W + (int64_t)n * a.ldw + 32 * kc + 8 * (l >> 4));
    }
  } else {
    // FP32: k-slot g of chunk kc is k = 16 (kc / 4) + 4 g + kc % 4, so one
    // float4 of X per lane feeds four consecutive chunks
    float* sb = (float*)smem;
    const float* W = (const float*)a.wt;
    for (int idx = threadIdx.x; idx < NT * KCH * 64; idx += 256) {
      const int l = idx & 63, kc = (idx >> 6) % KCH, nt = (idx >> 6) / KCH;
      const int n = n0 + 16 * nt + (l & 15);
      sb[idx] = W[(int64_t)n * a.ldw + 16 * (kc / 4) + 4 * (l >> 4) + (kc % 4)];
    }
  }
  __syncthreads();
  for (int64_t tile = (int64_t)blockIdx.x * 4 + w; tile < row_tiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t r = tile * 16 + rr;
    const bool rv = r < a.M;
    const int64_t xo = rv ? (r / a.rpa) * a.xs + (r % a.rpa) * a.xr : 0;
    const float* xrow = a.x + xo;
    const __bf16* xbrow = (const __bf16*)a.x + xo;
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
    if constexpr (PREC == 1) {
      const bf16x8* sb = (const bf16x8*)smem;
      for (int kc = 0; kc < KCH; ++kc) {
        bf16x8 av;
        if (rv && a.x_bf16) {
          av = *(const bf16x8*)(xbrow + 32 * kc + 8 * g);
        } else if (rv) {
          const float4 u0 = *(const float4*)(xrow + 32 * kc + 8 * g);
          const float4 u1 = *(const float4*)(xrow + 32 * kc + 8 * g + 4);
          av[0] = (__bf16)u0.x; av[1] = (__bf16)u0.y; av[2] = (__bf16)u0.z; av[3] = (__bf16)u0.w;
          av[4] = (__bf16)u1.x; av[5] = (__bf16)u1.y; av[6] = (__bf16)u1.z; av[7] = (__bf16)u1.w;
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) av[j] = (__bf16)0.f;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma_bf16(av, sb[(t * KCH + kc) * 64 + lane], acc[t]);
      }
    } else {
      const float* sb = (const float*)smem;
      const int KQ = KCH / 4;   // K / 16
      const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
      float4 xv = rv ? *(const float4*)(xrow + 4 * g) : zero;
      for (int q = 0; q < KQ; ++q) {
        const float4 cur = xv;
        if (q + 1 < KQ) xv = rv ? *(const float4*)(xrow + 16 * (q + 1) + 4 * g) : zero;
        const float c4[4] = {cur.x, cur.y, cur.z, cur.w};
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int t = 0; t < NT; ++t) acc[t] = mfma_f32(c4[j], sb[(t * KCH + 4 * q + j) * 64 + lane], acc[t]);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t ro = tile * 16 + 4 * g + q;
      if (ro >= a.M) continue;
      const int64_t yo = (ro / a.rpa) * a.ys + (ro % a.rpa) * a.yr;
      float* yrow = a.y + yo;
      __bf16* ybrow = (__bf16*)a.y + yo;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int n = n0 + 16 * t + rr;
        if (a.y_bf16) ybrow[n] = (__bf16)acc[t][q];
        else if (a.accumulate) yrow[n] += acc[t][q];
        else yrow[n] = acc[t][q];
      }
    }
  }
}

template <int PREC>
static bool gemm_lds_try(int nt, const GemmArgs& g, hipStream_t s) {
  if (PREC == 0 && g.K % 16 != 0) return false;   // the FP32 loads take K in 16s
  const int KCH = (PREC == 1) ? g.K / 32 : g.K / 4;
  const size_t per = (size_t)KCH * 64 * (PREC == 1 ? 16 : 4);
  if ((g.Nout / 16) % nt != 0 || per * nt > 64 * 1024) return false;
  const int64_t row_tiles = (g.M + 15) / 16;
  int64_t gx = (row_tiles + 3) / 4;
  if (gx > 1024) gx = 1024;
  dim3 grid((unsigned)gx, (unsigned)(g.Nout / (16 * nt)));
  const size_t lds = per * nt;
  switch (nt) {
    case 12: k_gemm_lds<PREC, 12><<<grid, 256, lds, s>>>(g, row_tiles); break;
    case 8: k_gemm_lds<PREC, 8><<<grid, 256, lds, s>>>(g, row_tiles); break;
    case 4: k_gemm_lds<PREC, 4><<<grid, 256, lds, s>>>(g, row_tiles); break;
    default: k_gemm_lds<PREC, 2><<<grid, 256, lds, s>>>(g, row_tiles); break;
  }
  return true;
}

void launch_gemm(int prec, const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0) return;
  const int vec = g.x_bf16 ? 8 : 4;   // elements per 16-byte load
  const bool aligned = (g.xs % vec == 0) && (g.xr % vec == 0) && ((uintptr_t)g.x % 16 == 0);
  if (aligned && g.M >= 4096) {
    for (int nt : {12, 8, 4, 2}) {
      if (prec == MPIP_BF16_MIXED ? gemm_lds_try<1>(nt, g, s) : gemm_lds_try<0>(nt, g, s)) return;
    }
  }
  dim3 grid((unsigned)((g.M + 63) / 64), (unsigned)((g.Nout + 63) / 64));
  if (prec == MPIP_BF16_MIXED) k_gemm<1><<<grid, 256, 0, s>>>(g);
  else k_gemm<0><<<grid, 256, 0, s>>>(g);
}

// ------------------------------------------------------------ gates

// h <- h + update; at the first layer h starts from the embedding (scalars)
// and zero for l >= 1.  `last`: only the scalar output exists.
__global__ void k_gate_fwd(NodeArgs a, int first, int last) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= a.n * a.C) return;
  const int64_t i = idx / a.C;
  const int c = (int)(idx % a.C);
  const int C = a.C, nlm = a.nlm, nz = C * (1 + a.L);
  float* h = a.h + i * nlm * C;
  const float* z0 = a.z0 + i * nz;
  const float h0 = first ? a.emb[(int64_t)a.spec_s[i] * C + c] : h[c];
  h[c] = h0 + silu(z0[c]);
  if (last) return;
  for (int l = 1; l <= a.L; ++l) {
    const float gt = sigm(z0[l * C + c]);
    for (int m = 0; m < 2 * l + 1; ++m) {
      const int lm = l * l + m;
      const float zv = a.zl[(i * (nlm - 1) + lm - 1) * C + c];
      h[lm * C + c] = (first ? 0.f : h[lm * C + c]) + gt * zv;
    }
  }
}

void launch_gate_fwd(const NodeArgs& a, int first, int last, hipStream_t s) {
  const int64_t tot = a.n * a.C;
  k_gate_fwd<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(a, first, last);
}

// E_i = e0[z_i] + h[i,0,:] . w_read  (one wave per atom)
__global__ void k_readout(NodeArgs a) {
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= a.n) return;
  double s = 0.0;
  for (int c = lane; c < a.C; c += 64) s += (double)a.h[i * a.nlm * a.C + c] * (double)a.w_read[c];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) a.atom_e[i] = (double)a.e0[a.spec_s[i]] + s;
}

void launch_readout(const NodeArgs& a, hipStream_t s) {
  k_readout<<<(unsigned)((a.n + 3) / 4), 256, 0, s>>>(a);
}

// Adjoint of the gates.  z buffers are overwritten by their adjoints.
// last: hbar of the scalars is w_read on root atoms (seed of the backward).
// init_hbar: also write the residual part of hbar for the layer below
// (w_read on root scalars, zero elsewhere).
__global__ void k_gate_bwd(NodeArgs a, int last, int init_hbar) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= a.n * a.C) return;
  const int64_t i = idx / a.C;
  const int c = (int)(idx % a.C);
  const int C = a.C, nlm = a.nlm, nz = C * (1 + a.L);
  float* z0 = a.z0 + i * nz;
  float* hb = a.hbar + i * nlm * C;
  if (last) {
    const float seed = a.owned_s[i] ? a.w_read[c] : 0.f;
    z0[c] = seed * dsilu(z0[c]);
    if (init_hbar) {
      hb[c] = seed;
      for (int lm = 1; lm < nlm; ++lm) hb[lm * C + c] = 0.f;
    }
    return;
  }
  z0[c] = hb[c] * dsilu(z0[c]);
  for (int l = 1; l <= a.L; ++l) {
    const float gi = z0[l * C + c];
    const float s = sigm(gi);
    float dg = 0.f;
    for (int m = 0; m < 2 * l + 1; ++m) {
      const int lm = l * l + m;
      float* zp = a.zl + (i * (nlm - 1) + lm - 1) * C + c;
      const float hv = hb[lm * C + c];
      dg += hv * (*zp);
      *zp = hv * s;
    }
    z0[l * C + c] = dg * s * (1.f - s);
  }
}

void launch_gate_bwd(const NodeArgs& a, int last, int init_hbar, hipStream_t s) {
  const int64_t tot = a.n * a.C;
  k_gate_bwd<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(a, last, init_hbar);
}

// ------------------------------------------------------------ outputs

// Per atom: F_i = sum_{e in row i} G_e - G_rev(e) (FP64), written in input
// order, with G_e = g[e] (dE/dr_e, or the h_e of FastArgs::g2p, which gives
// the same sums); per block: sum of root energies and of r_e (x) G_e, fixed
// order.
// A wave takes 16 rows, 4 at a time with 16 lanes over each row's edges
// (three edges per lane in flight, so a row of up to 48 edges costs one
// round of dependent loads) and a 16-lane butterfly per row; each lane keeps
// its virial partial sums, reduced over the wave by shuffles and over the
// block's 4 waves in LDS, always in the same order.
__global__ __launch_bounds__(256) void k_forces(OutArgs a) {
  __shared__ double sh[4][10];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q = lane >> 4, el = lane & 15;
  double loc[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) loc[k] = 0.0;
  const bool run = (a.status[ST_FLAGS] == 0) && ((int64_t)a.row_ptr[a.n] <= a.capacity);
  if (run) {
    const int64_t r0 = (int64_t)blockIdx.x * kOutRowsPerBlock + w * 16;
#pragma unroll 1
    for (int64_t ib = r0; ib < r0 + 16; ib += 4) {
      const int64_t i = ib + q;
      double F[3] = {0.0, 0.0, 0.0};
      if (i < a.n) {
        const int e1 = a.row_ptr[i + 1];
        for (int e = a.row_ptr[i] + el; e < e1; e += 48) {
          int rv[3];
          float4 ge[3], gr[3], r[3];
#pragma unroll
          for (int u = 0; u < 3; ++u) {
            const int eu = e + 16 * u;
            const bool ok = eu < e1;
            rv[u] = ok ? a.e_rev[eu] : -1;
            ge[u] = ok ? a.g[eu] : make_float4(0.f, 0.f, 0.f, 0.f);
            r[u] = ok ? a.e_vec[eu] : make_float4(0.f, 0.f, 0.f, 0.f);
          }
#pragma unroll
          for (int u = 0; u < 3; ++u) gr[u] = rv[u] >= 0 ? a.g[rv[u]] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
          for (int u = 0; u < 3; ++u) {
            F[0] += (double)ge[u].x - (double)gr[u].x;
            F[1] += (double)ge[u].y - (double)gr[u].y;
            F[2] += (double)ge[u].z - (double)gr[u].z;
            const double rr[3] = {r[u].x, r[u].y, r[u].z}, gg[3] = {ge[u].x, ge[u].y, ge[u].z};
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
              for (int c = 0; c < 3; ++c) loc[1 + 3 * p + c] += rr[p] * gg[c];
          }
        }
      }
#pragma unroll
      for (int off = 8; off > 0; off >>= 1)
#pragma unroll
        for (int d = 0; d < 3; ++d) F[d] += __shfl_xor(F[d], off);
      if (el == 0 && i < a.n) {
        const int o = a.perm[i];
        a.forces[3 * (int64_t)o + 0] = F[0];
        a.forces[3 * (int64_t)o + 1] = F[1];
        a.forces[3 * (int64_t)o + 2] = F[2];
        if (a.atom_energy) a.atom_energy[o] = a.atom_e[i];
        if (a.owned_s[i]) loc[0] += a.atom_e[i];
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
  if (threadIdx.x < 10)
    a.partials[(int64_t)blockIdx.x * 10 + threadIdx.x] =
        ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) + sh[3][threadIdx.x];
}

__global__ void k_final(OutArgs a) {
  __shared__ double sh[10][256];
  double loc[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) loc[k] = 0.0;
  for (int b = threadIdx.x; b < a.nblocks; b += 256)
#pragma unroll
    for (int k = 0; k < 10; ++k) loc[k] += a.partials[(int64_t)b * 10 + k];
#pragma unroll
  for (int k = 0; k < 10; ++k) sh[k][threadIdx.x] = loc[k];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
#pragma unroll
      for (int k = 0; k < 10; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
    __syncthreads();
  }
  // a data-dependent error (the passes skipped their work) leaves NaN in the
  // energy and virial, visible to callers that cannot read the status word
  const bool ok = (a.status[ST_FLAGS] == 0) && ((int64_t)a.row_ptr[a.n] <= a.capacity);
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  if (threadIdx.x == 0) a.energy[0] = ok ? sh[0][0] : nan;
  if (threadIdx.x < 9) a.virial[threadIdx.x] = ok ? -sh[1 + threadIdx.x][0] : nan;
}

void launch_outputs(const OutArgs& a, hipStream_t s) {
  k_forces<<<a.nblocks, 256, 0, s>>>(a);
  k_final<<<1, 256, 0, s>>>(a);
}

__global__ void k_fill(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// a kernel rather than hipMemsetAsync, so that a captured graph holds only kernel nodes
void launch_fill32(void* p, uint32_t value, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_fill<<<(unsigned)blocks, 256, 0, s>>>((uint32_t*)p, n, value);
}

void launch_zero(void* p, size_t bytes, hipStream_t s) { launch_fill32(p, 0u, bytes, s); }

__global__ void k_scale(float* p, int64_t n, float f) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] *= f;
}

void launch_scale(float* p, float f, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_scale<<<(unsigned)blocks, 256, 0, s>>>(p, n, f);
}

}  // namespace mpip
