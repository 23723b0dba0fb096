// Host engine and C ABI of libmpip: parameter validation, weight upload in
// the kernels' operand layouts, workspace planning and the launch sequence
// of one evaluation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "cg.h"
#include "kernels.h"

using namespace mpip;

namespace {

thread_local std::string g_err;

mpip_status fail(mpip_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t _e = (x);                                                                   \
    if (_e != hipSuccess) return fail(MPIP_EDEVICE, std::string(#x ": ") + hipGetErrorString(_e)); \
  } while (0)

uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  uint32_t r = ((u >> 16) & 1u) + 0x7fffu;
  return (uint16_t)((u + r) >> 16);
}

int n_paths_stored(int t, int L) { return (int)layer_paths(t, L).size(); }

// The BF16 form's radial table of one layer, in the layout rad_pos and
// rad_tiles read (edge_common.h): the MLP's second hidden layer
// a(d) = silu(W2^T silu(W1^T b(d))) at the kRadTab + 1 knots
// d_k = k r_c / kRadTab, in FP64 from the FP32 weights, with the Bessel
// basis times the polynomial envelope, b_n(d) = sqrt(2/r_c) sin(n pi d / r_c) / d f(d / r_c)
// (at d = 0 its limit sqrt(2/r_c) n pi / r_c), f(x) = 1 - a x^p + b x^(p+1) - c x^(p+2)
// below x = 1 and 0 from there.  Word (k, h) packs BF16 a_h(d_k) (low
// half) and BF16 of a_h(d_k+1) - a_h(d_k) (high half).
std::vector<uint32_t> radial_table(const float* W1, const float* W2, int nb, int H, double rc, int p) {
  const int N = kRadTab;
  const double pi = 3.14159265358979323846;
  const double ea = 0.5 * (p + 1) * (p + 2), eb = (double)p * (p + 2), ec = 0.5 * p * (p + 1);
  std::vector<double> a((size_t)(N + 1) * H), b(nb), h1(H);
  for (int k = 0; k <= N; ++k) {
    const double d = rc * k / N, x = (double)k / N;
    const double env = x < 1.0 ? 1.0 - ea * std::pow(x, p) + eb * std::pow(x, p + 1) - ec * std::pow(x, p + 2) : 0.0;
    for (int n_ = 0; n_ < nb; ++n_) {
      const double w = (n_ + 1) * pi / rc;
      b[n_] = std::sqrt(2.0 / rc) * (k == 0 ? w : std::sin(w * d) / d) * env;
    }
    for (int h = 0; h < H; ++h) {
      double z = 0.0;
      for (int n_ = 0; n_ < nb; ++n_) z += (double)W1[(size_t)n_ * H + h] * b[n_];
      h1[h] = z / (1.0 + std::exp(-z));
    }
    for (int h = 0; h < H; ++h) {
      double z = 0.0;
      for (int i = 0; i < H; ++i) z += (double)W2[(size_t)i * H + h] * h1[i];
      a[(size_t)k * H + h] = z / (1.0 + std::exp(-z));
    }
  }
  std::vector<uint32_t> t((size_t)N * H);
  for (int k = 0; k < N; ++k)
    for (int h = 0; h < H; ++h) {
      const double v = a[(size_t)k * H + h], dv = a[(size_t)(k + 1) * H + h] - v;
      t[(size_t)k * H + h] = (uint32_t)f2bf((float)v) | ((uint32_t)f2bf((float)dv) << 16);
    }
  return t;
}

bool valid_hp(const mpip_hparams* hp, std::string* why) {
  if (!hp) { *why = "null hparams"; return false; }
  if (hp->n_species < 1 || hp->n_species > 64) { *why = "n_species must be in 1..64"; return false; }
  if (hp->n_layers < 1 || hp->n_layers > 16) { *why = "n_layers must be in 1..16"; return false; }
  if (hp->l_max < 1 || hp->l_max > 2) { *why = "l_max must be 1 or 2"; return false; }
  if (hp->channels != 32 && hp->channels != 64 && hp->channels != 128) { *why = "channels must be 32, 64 or 128"; return false; }
  if (hp->n_basis != kNB) { *why = "n_basis must be 8"; return false; }
  if (hp->radial_hidden != kHidden) { *why = "radial_hidden must be 64"; return false; }
  if (hp->envelope_p < 2 || hp->envelope_p > 16) { *why = "envelope_p must be in 2..16"; return false; }
  if (!(hp->r_cut > 0.0) || !std::isfinite(hp->r_cut)) { *why = "r_cut must be positive"; return false; }
  if (!std::isfinite(hp->inv_avg_neighbors)) { *why = "inv_avg_neighbors must be finite"; return false; }
  return true;
}

size_t count_weights(const mpip_hparams& hp) {
  const size_t C = hp.channels, H = hp.radial_hidden, nb = hp.n_basis, L = hp.l_max, S = hp.n_species;
  size_t n = S * C;
  for (int t = 1; t <= hp.n_layers; ++t) {
    const size_t nin = (t == 1) ? 1 : (L + 1);
    n += nin * C * C + nb * H + H * H + H * n_paths_stored(t, (int)L) * C + C * C * (1 + L) + L * C * C;
  }
  return n + C + S;
}

// Device buffer list owned by a model.
struct DevArena {
  std::vector<void*> ptrs;
  ~DevArena() {
    for (void* p : ptrs) hipFree(p);
  }
};

}  // namespace

// Workspace of mpip_evaluate_noalloc: one fixed-size array in every device's
// copy of this code object, held until the process ends.  In host code its
// name is only a stand-in; the device address is resolved once per device
// (with that device current) and kept in scratch_ptr.
constexpr size_t kNoAllocScratchBytes = (size_t)MPIP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on device `dev`, which must be current
mpip_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(MPIP_EUNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(MPIP_EDEVICE, "hipGetSymbolAddress returned a null address for the static scratch");
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return MPIP_OK;
}

}  // namespace

// Events created when timing is enabled: two per phase, about 12 phases per
// evaluation, so 170 timed evaluations between two reads need no new event.
constexpr size_t kTimingEvents = 4096;

// Event-pair timer of evaluation phases (enabled on request only).
struct PhaseTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<std::string, size_t>> pending;  // name, index of start event
  std::vector<std::string> names;
  std::vector<double> ms;
  std::vector<int64_t> calls;
  // events are created when timing is switched on (reserve), so a timed
  // evaluation only records them; the pool grows here only past that reserve
  void reserve(size_t n) {
    while (pool.size() < n) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) break;
      pool.push_back(e);
    }
  }
  // a phase takes its start and end events in begin(); if none can be
  // created, timing switches itself off
  void begin(const std::string& name, hipStream_t s) {
    if (!on) return;
    if (used + 2 > pool.size()) reserve(used + 64);
    if (used + 2 > pool.size()) {
      on = false;
      return;
    }
    pending.push_back({name, used});
    hipEventRecord(pool[used++], s);
  }
  void end(hipStream_t s) {
    if (!on) return;
    hipEventRecord(pool[used++], s);
  }
  ~PhaseTimer() {
    for (hipEvent_t e : pool) hipEventDestroy(e);
  }
};

struct mpip_model {
  mpip_hparams hp;
  int device;
  bool force_generic = false;  // MPIP_FORCE_GENERIC=1 at creation: generic edge kernels only
  PhaseTimer timer;
  DevArena arena;
  // per precision (0 = f32, 1 = bf16), per layer
  std::vector<LayerDev> layers[2];
  float* emb = nullptr;
  float* w_read = nullptr;
  float* e0 = nullptr;
};

namespace {

template <typename T>
mpip_status upload(mpip_model* m, const std::vector<T>& v, const void** out) {
  void* p = nullptr;
  size_t bytes = v.size() * sizeof(T);
  if (bytes == 0) bytes = 16;
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(MPIP_ENOMEM, "hipMalloc failed for weights");
  m->arena.ptrs.push_back(p);
  if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = p;
  return MPIP_OK;
}

// Pack a matrix generator f(lane, slot) into operand arrays.
// bf16: 8 values per lane per chunk; f32: 1 value per lane per chunk.
struct Packer {
  std::vector<uint16_t> b;
  std::vector<float> f;
};

inline int phi_bf(int kc, int g, int j) { return 16 * (2 * kc + j / 4) + 4 * g + (j % 4); }
inline int phi_f(int q, int g) { return 16 * (q / 4) + 4 * g + (q % 4); }

}  // namespace

extern "C" {

size_t mpip_weights_count(const mpip_hparams* hp) {
  std::string why;
  if (!valid_hp(hp, &why)) return 0;
  return count_weights(*hp);
}

const char* mpip_last_error(void) { return g_err.c_str(); }

mpip_status mpip_coupling_tensor(int32_t l1, int32_t l2, int32_t l3, double* out) {
  if (!out) return fail(MPIP_EINVAL, "null output");
  if (!coupling_tensor(l1, l2, l3, out)) return fail(MPIP_EINVAL, "not a natural-parity path with l <= 2");
  return MPIP_OK;
}

mpip_status mpip_radial_table(const mpip_hparams* hp, const float* w, size_t n, int32_t layer, uint32_t* out) {
  std::string why;
  if (!valid_hp(hp, &why)) return fail(MPIP_EINVAL, why);
  if (!w || !out) return fail(MPIP_EINVAL, "null weights or output");
  if (n != count_weights(*hp)) return fail(MPIP_EINVAL, "weight count does not match the hyper-parameters");
  if (layer < 1 || layer > hp->n_layers) return fail(MPIP_EINVAL, "no such layer");
  // the layer's W1 and W2 in the weight blob (the order mpip_model_create reads)
  const size_t C = hp->channels, H = hp->radial_hidden, nb = hp->n_basis, L = hp->l_max, S = hp->n_species;
  size_t off = S * C;
  for (int t = 1; t < layer; ++t)
    off += ((t == 1) ? 1 : (L + 1)) * C * C + nb * H + H * H + H * n_paths_stored(t, (int)L) * C +
           C * C * (1 + L) + L * C * C;
  off += ((layer == 1) ? 1 : (L + 1)) * C * C;
  const std::vector<uint32_t> t = radial_table(w + off, w + off + nb * H, (int)nb, (int)H, hp->r_cut, hp->envelope_p);
  std::memcpy(out, t.data(), t.size() * sizeof(uint32_t));
  return MPIP_OK;
}

mpip_status mpip_model_destroy(mpip_model* m) {
  if (!m) return MPIP_OK;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(m->device);
  delete m;
  hipSetDevice(cur);
  return MPIP_OK;
}

mpip_status mpip_model_create(const mpip_hparams* hp, const float* w, size_t n, int32_t device, mpip_model** out) {
  std::string why;
  if (!out) return fail(MPIP_EINVAL, "null output handle");
  *out = nullptr;
  if (!valid_hp(hp, &why)) return fail(MPIP_EINVAL, why);
  if (!w) return fail(MPIP_EINVAL, "null weights");
  if (n != count_weights(*hp)) return fail(MPIP_EINVAL, "weight count does not match the hyper-parameters");
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(MPIP_EINVAL, "no such device");
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  HIPCHK(hipSetDevice(device));
  mpip_model* m = new mpip_model();
  m->hp = *hp;
  {
    const char* fg = std::getenv("MPIP_FORCE_GENERIC");
    m->force_generic = fg && fg[0] == '1';
  }
  m->device = device;
  const int C = hp->channels, H = hp->radial_hidden, nb = hp->n_basis, L = hp->l_max, S = hp->n_species;
  const int T = hp->n_layers;
  size_t off = 0;
  auto take = [&](size_t k) { const float* p = w + off; off += k; return p; };
  mpip_status st = MPIP_OK;
  const float* emb = take((size_t)S * C);
  struct LayerHost {
    std::vector<const float*> up;
    const float *W1, *W2, *W3;
    std::vector<const float*> down;
    int P;
  };
  std::vector<LayerHost> lh(T);
  for (int t = 1; t <= T; ++t) {
    LayerHost& x = lh[t - 1];
    const int nin = (t == 1) ? 1 : (L + 1);
    for (int l = 0; l < nin; ++l) x.up.push_back(take((size_t)C * C));
    x.W1 = take((size_t)nb * H);
    x.W2 = take((size_t)H * H);
    x.P = n_paths_stored(t, L);
    x.W3 = take((size_t)H * x.P * C);
    x.down.push_back(take((size_t)C * C * (1 + L)));
    for (int l = 1; l <= L; ++l) x.down.push_back(take((size_t)C * C));
  }
  const float* w_read = take(C);
  const float* e0 = take(S);
  (void)off;
  {
    const void* p;
    std::vector<float> v(emb, emb + (size_t)S * C);
    if ((st = upload(m, v, &p)) != MPIP_OK) goto done;
    m->emb = (float*)p;
    std::vector<float> r(w_read, w_read + C);
    if ((st = upload(m, r, &p)) != MPIP_OK) goto done;
    m->w_read = (float*)p;
    std::vector<float> e(e0, e0 + S);
    if ((st = upload(m, e, &p)) != MPIP_OK) goto done;
    m->e0 = (float*)p;
  }
  for (int prec = 0; prec < 2; ++prec) m->layers[prec].resize(T);
  for (int t = 1; t <= T; ++t) {
    const LayerHost& x = lh[t - 1];
    const std::vector<Path> stored = layer_paths(t, L);
    const int PC = x.P * C;
    auto W1 = [&](int n_, int h) { return x.W1[n_ * H + h]; };
    auto W2 = [&](int a, int b) { return x.W2[a * H + b]; };
    auto W3 = [&](int h, int col) { return x.W3[(size_t)h * PC + col]; };
    // live path lists: role 0 (t < K): all stored; role 1 (t == K): l3 == 0
    std::vector<int> live[2];
    for (int k = 0; k < (int)stored.size(); ++k) {
      live[0].push_back(k);
      if (stored[k].l3 == 0) live[1].push_back(k);
    }
    for (int prec = 0; prec < 2; ++prec) {
      LayerDev& d = m->layers[prec][t - 1];
      const bool bf = prec == 1;
      // generic packers
      auto pack = [&](int nchunk_outer, int nchunk_k, auto val, const void** dst) -> mpip_status {
        // layout [outer][k][lane][8|1]
        if (bf) {
          std::vector<uint16_t> v((size_t)nchunk_outer * nchunk_k * 64 * 8);
          for (int o = 0; o < nchunk_outer; ++o)
            for (int k = 0; k < nchunk_k; ++k)
              for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j)
                  v[(((size_t)o * nchunk_k + k) * 64 + lane) * 8 + j] = f2bf(val(o, k, lane, j));
          return upload(m, v, dst);
        } else {
          std::vector<float> v((size_t)nchunk_outer * nchunk_k * 64);
          for (int o = 0; o < nchunk_outer; ++o)
            for (int k = 0; k < nchunk_k; ++k)
              for (int lane = 0; lane < 64; ++lane)
                v[((size_t)o * nchunk_k + k) * 64 + lane] = val(o, k, lane, 0);
          return upload(m, v, dst);
        }
      };
      const int KC64 = bf ? 2 : 16;
      d.rtab = nullptr;
      if (bf) {
        const void* tp;
        if ((st = upload(m, radial_table(x.W1, x.W2, nb, H, hp->r_cut, hp->envelope_p), &tp)) != MPIP_OK) goto done;
        d.rtab = (const uint32_t*)tp;
      }
      // w1a: [mt 4][k][lane]: row h = 16mt + lane%16; bf16 k-slot (g,j) -> basis 8g+j; f32 chunk q -> basis 4q+g
      if ((st = pack(4, bf ? 1 : 2, [&](int mt, int k, int lane, int j) {
             const int h = 16 * mt + (lane & 15), g = lane >> 4;
             const int n_ = bf ? (8 * g + j) : (4 * k + g);
             return n_ < nb ? W1(n_, h) : 0.f;
           }, &d.w1a)) != MPIP_OK) goto done;
      if ((st = pack(4, KC64, [&](int mt, int k, int lane, int j) {
             const int h2 = 16 * mt + (lane & 15), g = lane >> 4;
             const int h1 = bf ? phi_bf(k, g, j) : phi_f(k, g);
             return W2(h1, h2);
           }, &d.w2a)) != MPIP_OK) goto done;
      if ((st = pack(4, KC64, [&](int mt, int k, int lane, int j) {
             const int h1 = 16 * mt + (lane & 15), g = lane >> 4;
             const int h2 = bf ? phi_bf(k, g, j) : phi_f(k, g);
             return W2(h1, h2);
           }, &d.w2b)) != MPIP_OK) goto done;
      if ((st = pack(1, KC64, [&](int, int k, int lane, int j) {
             const int n_ = lane & 15, g = lane >> 4;
             const int h1 = bf ? phi_bf(k, g, j) : phi_f(k, g);
             return n_ < nb ? W1(n_, h1) : 0.f;
           }, &d.w1b)) != MPIP_OK) goto done;
      for (int role = 0; role < 2; ++role) {
        const std::vector<int>& lv = live[role];
        const int NPl = (int)lv.size();
        // w3f: [pi][nt][kc][lane]: col c = 16nt + lane%16, k-slot -> hidden
        if ((st = pack(NPl * (C / 16), KC64, [&](int o, int k, int lane, int j) {
               const int pi = o / (C / 16), nt = o % (C / 16), g = lane >> 4;
               const int c = 16 * nt + (lane & 15);
               const int h = bf ? phi_bf(k, g, j) : phi_f(k, g);
               return W3(h, lv[pi] * C + c);
             }, &d.w3f[role])) != MPIP_OK) goto done;
        const int KCC = bf ? C / 32 : C / 4;
        // w3b: [pi][mt][kc][lane]: row h = 16mt + lane%16, k-slot -> channel
        if ((st = pack(NPl * 4, KCC, [&](int o, int k, int lane, int j) {
               const int pi = o / 4, mt = o % 4, g = lane >> 4;
               const int h = 16 * mt + (lane & 15);
               const int c = bf ? (32 * k + 8 * g + j) : (4 * k + g);
               return W3(h, lv[pi] * C + c);
             }, &d.w3b[role])) != MPIP_OK) goto done;
        std::vector<float> cgv;
        for (int pi = 0; pi < NPl; ++pi) {
          const Path& pp = stored[lv[pi]];
          const int nn = (2 * pp.l1 + 1) * (2 * pp.l2 + 1) * (2 * pp.l3 + 1);
          std::vector<double> tmp(nn);
          if (!coupling_tensor(pp.l1, pp.l2, pp.l3, tmp.data())) { st = fail(MPIP_EINVAL, "coupling"); goto done; }
          if (pp.l3 == 0 || pp.l1 == 0) {
            // the specialised first- and last-layer kernels use only the
            // diagonal of a (0, l, l) or (l, l, 0) coupling
            const int n1 = 2 * std::max(pp.l1, pp.l3) + 1;
            for (int a = 0; a < n1; ++a)
              for (int b2 = 0; b2 < n1; ++b2)
                if (a != b2 && tmp[a * n1 + b2] != 0.0) { st = fail(MPIP_EINVAL, "scalar coupling not diagonal"); goto done; }
          }
          for (double v : tmp) cgv.push_back((float)v);
        }
        const void* cgp;
        if ((st = upload(m, cgv, &cgp)) != MPIP_OK) goto done;
        d.cg[role] = (const float*)cgp;
      }
      // node matrices, [Nout][K] with k contiguous
      auto node = [&](const float* Wm, int rows, int cols, bool transpose, const void** dst) -> mpip_status {
        // Wm is [rows][cols]; transpose: out[c][r] = Wm[r][c]
        const int NO = transpose ? cols : rows, KK = transpose ? rows : cols;
        if (bf) {
          std::vector<uint16_t> v((size_t)NO * KK);
          for (int a = 0; a < NO; ++a)
            for (int b = 0; b < KK; ++b) v[(size_t)a * KK + b] = f2bf(transpose ? Wm[(size_t)b * cols + a] : Wm[(size_t)a * cols + b]);
          return upload(m, v, dst);
        } else {
          std::vector<float> v((size_t)NO * KK);
          for (int a = 0; a < NO; ++a)
            for (int b = 0; b < KK; ++b) v[(size_t)a * KK + b] = transpose ? Wm[(size_t)b * cols + a] : Wm[(size_t)a * cols + b];
          return upload(m, v, dst);
        }
      };
      for (int l = 0; l < 3; ++l) { d.up_t[l] = d.up[l] = d.down_t[l] = d.down[l] = nullptr; }
      for (int l = 0; l < (int)x.up.size(); ++l) {
        if ((st = node(x.up[l], C, C, true, &d.up_t[l])) != MPIP_OK) goto done;
        if ((st = node(x.up[l], C, C, false, &d.up[l])) != MPIP_OK) goto done;
      }
      if ((st = node(x.down[0], C, C * (1 + L), true, &d.down_t[0])) != MPIP_OK) goto done;
      if ((st = node(x.down[0], C, C * (1 + L), false, &d.down[0])) != MPIP_OK) goto done;
      for (int l = 1; l <= L; ++l) {
        if ((st = node(x.down[l], C, C, true, &d.down_t[l])) != MPIP_OK) goto done;
        if ((st = node(x.down[l], C, C, false, &d.down[l])) != MPIP_OK) goto done;
      }
      // the fused last-layer node kernel (BF16 form; any layer t >= 2 can be the last)
      d.nk_dt = d.nk_d = nullptr;
      if (bf && t >= 2 && (C == 64 || C == 128)) {
        const float* Wd = x.down[0];   // [C][C (1 + L)]; the scalar block is columns 0..C-1
        const int nzd = C * (1 + L);
        if ((st = pack(C / 16, C / 32, [&](int mt, int kc, int lane, int j) {
               return Wd[(size_t)(32 * kc + 8 * (lane >> 4) + j) * nzd + 16 * mt + (lane & 15)];
             }, &d.nk_dt)) != MPIP_OK) goto done;
        // dE/dA = W_down zbar with the message normalisation 1/n_avg folded in:
        // the fused last-layer adjoint reads dA / n_avg
        const double inv_n = hp->inv_avg_neighbors;
        if ((st = pack(C / 16, C / 32, [&](int mt, int kc, int lane, int j) {
               return (float)(Wd[(size_t)(16 * mt + (lane & 15)) * nzd + phi_bf(kc, lane >> 4, j)] * inv_n);
             }, &d.nk_d)) != MPIP_OK) goto done;
      }
      // FP32 form, specialised first and sender-side last layer: row-major
      // copies with odd row strides
      d.w1r = d.w2r = d.w3r = nullptr;
      if (!bf && (C == 64 || C == 128)) {
        std::vector<float> v1((size_t)8 * 65, 0.f), v2((size_t)64 * 65, 0.f);
        for (int n_ = 0; n_ < nb; ++n_)
          for (int h = 0; h < H; ++h) v1[(size_t)n_ * 65 + h] = W1(n_, h);
        for (int a = 0; a < H; ++a)
          for (int b2 = 0; b2 < H; ++b2) v2[(size_t)a * 65 + b2] = W2(a, b2);
        const void* p1;
        if ((st = upload(m, v1, &p1)) != MPIP_OK) goto done;
        d.w1r = (const float*)p1;
        if ((st = upload(m, v2, &p1)) != MPIP_OK) goto done;
        d.w2r = (const float*)p1;
        if (t >= 2) {   // W3 of the live paths when the layer is the last one
          const std::vector<int>& lv = live[1];
          const int ws = (int)lv.size() * C + 1;
          std::vector<float> v3((size_t)H * ws, 0.f);
          for (int h = 0; h < H; ++h)
            for (int pi = 0; pi < (int)lv.size(); ++pi)
              for (int c = 0; c < C; ++c) v3[(size_t)h * ws + pi * C + c] = W3(h, lv[pi] * C + c);
          if ((st = upload(m, v3, &p1)) != MPIP_OK) goto done;
          d.w3r = (const float*)p1;
        }
      }
      // ---- operand layouts of the specialised first / last layer kernels
      // layer-2 B operand, edges x features: col h2 = 16 nt + lane%16, k-slot -> h1
      if ((st = pack(4, KC64, [&](int nt, int k, int lane, int j) {
             const int h2 = 16 * nt + (lane & 15), g = lane >> 4;
             const int h1 = bf ? phi_bf(k, g, j) : phi_f(k, g);
             return W2(h1, h2);
           }, &d.w2f)) != MPIP_OK) goto done;
      for (int role = 0; role < 2; ++role) {
        const std::vector<int>& lv = live[role];
        const int NPl = (int)lv.size();
        const int CN = C / 16, CB = C / 4;
        if ((st = pack(NPl * CN, KC64, [&](int o, int k, int lane, int j) {
               const int pi = o / CN, nt = o % CN, g = lane >> 4;
               const int c = CN * (lane & 15) + nt;
               const int h = bf ? phi_bf(k, g, j) : phi_f(k, g);
               return W3(h, lv[pi] * C + c);
             }, &d.w3fp[role])) != MPIP_OK) goto done;
        if ((st = pack(NPl * CN, KC64, [&](int o, int k, int lane, int j) {
               const int pi = o / CN, mt = o % CN, g = lane >> 4, rho = lane & 15;
               // chunk k = mt/2 of lane group rho/4: channels 32k + 8(rho/4) + 4(mt%2) + rho%4
               const int c = 32 * (mt / 2) + 8 * (rho / 4) + 4 * (mt % 2) + (rho % 4);
               const int h = bf ? phi_bf(k, g, j) : phi_f(k, g);
               return W3(h, lv[pi] * C + c);
             }, &d.w3t[role])) != MPIP_OK) goto done;
        const int KCC = bf ? C / 32 : C / 4;
        if ((st = pack(NPl * 4, KCC, [&](int o, int k, int lane, int j) {
               const int pi = o / 4, mt = o % 4, g = lane >> 4;
               const int h = 16 * mt + (lane & 15);
               const int c = bf ? (32 * k + 8 * g + j) : (32 * (k / 8) + 8 * g + k % 8);
               return W3(h, lv[pi] * C + c);
             }, &d.w3bp[role])) != MPIP_OK) goto done;
      }
      for (int l = 0; l < 3; ++l)
        d.vt[l] = d.v[l] = d.vwt[l] = d.vw[l] = d.n1_vwt[l] = d.n1_upt[l] = d.n1_up[l] = d.n1_vw[l] = nullptr;
      if (t == 1) {
        // species table ht1 = W_emb W_up[0] (FP64), then V_l = ht1 (x) W3_l / n_avg
        std::vector<double> ht1((size_t)S * C, 0.0);
        for (int sp = 0; sp < S; ++sp)
          for (int c = 0; c < C; ++c) {
            double acc = 0.0;
            for (int cc = 0; cc < C; ++cc) acc += (double)emb[sp * C + cc] * (double)x.up[0][(size_t)cc * C + c];
            ht1[(size_t)sp * C + c] = acc;
          }
        const int KQ = 64 * S;
        for (int l = 0; l <= L; ++l) {
          std::vector<float> V((size_t)KQ * C);   // [(s,k)][c]
          for (int sp = 0; sp < S; ++sp)
            for (int k = 0; k < H; ++k)
              for (int c = 0; c < C; ++c)
                V[((size_t)sp * 64 + k) * C + c] =
                    (float)(ht1[(size_t)sp * C + c] * (double)W3(k, l * C + c) * hp->inv_avg_neighbors);
          if ((st = node(V.data(), KQ, C, true, &d.vt[l])) != MPIP_OK) goto done;
          if ((st = node(V.data(), KQ, C, false, &d.v[l])) != MPIP_OK) goto done;
          // VW_l = V_l W_down_l (FP64): the messages A_l only feed the down projection
          const int nz_l = l == 0 ? C * (1 + L) : C;
          const float* Wd = x.down[l];   // [C][nz_l]
          std::vector<float> VW((size_t)KQ * nz_l);
          for (int sp = 0; sp < S; ++sp)
            for (int k = 0; k < H; ++k)
              for (int o = 0; o < nz_l; ++o) {
                double acc = 0.0;
                for (int c = 0; c < C; ++c)
                  acc += ht1[(size_t)sp * C + c] * (double)W3(k, l * C + c) * (double)Wd[(size_t)c * nz_l + o];
                VW[((size_t)sp * 64 + k) * nz_l + o] = (float)(acc * hp->inv_avg_neighbors);
              }
          if ((st = node(VW.data(), KQ, nz_l, true, &d.vwt[l])) != MPIP_OK) goto done;
          if ((st = node(VW.data(), KQ, nz_l, false, &d.vw[l])) != MPIP_OK) goto done;
          // operands of the fused node kernels between layer 1 and a last layer 2 (BF16 form)
          d.n1_vwt[l] = d.n1_upt[l] = d.n1_up[l] = d.n1_vw[l] = nullptr;
          if (bf && T >= 2 && (C == 64 || C == 128) && S <= 4) {
            const float* Wu = lh[1].up[l];   // layer 2's W_up_l, [C_in][C_out]
            auto VWq = [&](int q, int f) { return VW[(size_t)q * nz_l + f]; };
            if ((st = pack(nz_l / 16, KQ / 32, [&](int mt, int kc, int lane, int j) {
                   return VWq(32 * kc + 8 * (lane >> 4) + j, 16 * mt + (lane & 15));
                 }, &d.n1_vwt[l])) != MPIP_OK) goto done;
            if ((st = pack(C / 16, C / 32, [&](int mt, int kc, int lane, int j) {
                   const int rho = lane & 15;
                   const int cin = phi_bf(kc, lane >> 4, j), cout = (C / 4) * (rho / 4) + 4 * mt + rho % 4;
                   return Wu[(size_t)cin * C + cout];
                 }, &d.n1_upt[l])) != MPIP_OK) goto done;
            if ((st = pack(C / 16, C / 32, [&](int mt, int kc, int lane, int j) {
                   const int cin = 16 * mt + (lane & 15), cout = 32 * kc + 8 * (lane >> 4) + j;
                   return Wu[(size_t)cin * C + cout];
                 }, &d.n1_up[l])) != MPIP_OK) goto done;
            if ((st = pack(KQ / 16, nz_l / 32, [&](int mt, int kcg, int lane, int j) {
                   const int rho = lane & 15, b = kcg / (C / 32), kc = kcg % (C / 32);
                   const int q = (KQ / 4) * (rho / 4) + 4 * mt + rho % 4;
                   return VWq(q, b * C + phi_bf(kc, lane >> 4, j));
                 }, &d.n1_vw[l])) != MPIP_OK) goto done;
          }
        }
      }
    }
  }
  {
    // the static scratch of mpip_evaluate_noalloc, resolved once per device while it is current
    void* sp = nullptr;
    if ((st = scratch_address(device, &sp)) != MPIP_OK) goto done;
  }
  HIPCHK(hipDeviceSynchronize());
done:
  hipSetDevice(cur);
  if (st != MPIP_OK) {
    delete m;
    return st;
  }
  *out = m;
  return MPIP_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ workspace

namespace {

// per-layer workspace offsets; K <= 16 (the model limit)
struct LayerOffsets {
  size_t v[16] = {};
  int n = 0;
  void push_back(size_t x) { v[n++] = x; }
  size_t operator[](int i) const { return v[i]; }
};

struct Plan {
  size_t total = 0;
  size_t o_status, o_bounds, o_grid, o_bcount, o_bcursor, o_bstart, o_rcount, o_rstart, o_scan, o_info, o_perm, o_iperm, o_pos,
      o_info_s, o_spec, o_owned, o_cnt, o_row, o_blk, o_cmask, o_esrc, o_eshift, o_evec, o_erev, o_edst, o_g,
      o_ypos, o_cand;
  size_t o_ht1, o_h, o_A, o_hbar, o_htbar, o_atom_e, o_partials;
  size_t o_qp = 0;  // first-layer species factorisation: Q (forward) / P (adjoint) [N][nlm][64 S]
  size_t o_msg = 0; // last-layer messages of the BF16 form, [max_edges][C] bf16
  size_t o_part = 0; // middle-layer adjoint: per-edge sums between its launches, [max_edges][kPartStride]
  LayerOffsets o_ht, o_z0, o_zl;  // per layer 1..K (index t-1)
  int max_bins;
  int nblocks_out;
  int64_t N = 0;
};

size_t take(size_t& cur, size_t bytes) {
  size_t o = (cur + 255) & ~(size_t)255;
  cur = o + bytes;
  return o;
}

// prec: the message buffer of the sender-side last layer holds BF16 or FP32
// values (the default sizes it for FP32, the larger)
Plan make_plan(int64_t N, int64_t cap, const mpip_hparams* hp, int K, int prec = MPIP_FP32) {
  Plan p;
  size_t cur = 0;
  p.N = N;
  p.max_bins = (int)std::min<int64_t>(std::max<int64_t>(4096, 2 * N), 1 << 26);
  p.o_status = take(cur, sizeof(int64_t) * ST_WORDS);
  p.o_bounds = take(cur, sizeof(double) * kBoundsParts * 6);
  p.o_grid = take(cur, sizeof(GridParams));
  p.o_bcount = take(cur, sizeof(int32_t) * (p.max_bins + 1));
  p.o_bcursor = take(cur, sizeof(int32_t) * (p.max_bins + 1));
  p.o_bstart = take(cur, sizeof(int32_t) * (p.max_bins + 1));
  p.o_rcount = take(cur, sizeof(int32_t) * (8 * (int64_t)p.max_bins + 1));
  p.o_rstart = take(cur, sizeof(int32_t) * (8 * (int64_t)p.max_bins + 1));
  p.o_scan = take(cur, sizeof(int32_t) * scan_tmp_elems(std::max<int64_t>(N, 8 * (int64_t)p.max_bins) + 1));
  p.o_info = take(cur, sizeof(int4) * N);
  p.o_perm = take(cur, sizeof(int32_t) * N);
  p.o_iperm = take(cur, sizeof(int32_t) * N);
  p.o_pos = take(cur, sizeof(double) * 3 * N);
  p.o_info_s = take(cur, sizeof(int4) * N);
  p.o_ypos = take(cur, sizeof(float4) * N);
  p.o_spec = take(cur, sizeof(int32_t) * N);
  p.o_owned = take(cur, N);
  p.o_cnt = take(cur, sizeof(int32_t) * N);
  p.o_row = take(cur, sizeof(int32_t) * (N + 1));
  p.o_blk = take(cur, sizeof(int32_t) * 28 * N);
  p.o_cmask = take(cur, sizeof(uint64_t) * kCandWords * N);
  p.o_cand = take(cur, sizeof(uint32_t) * kCandList * N);
  p.o_esrc = take(cur, sizeof(int32_t) * cap);
  p.o_eshift = take(cur, sizeof(uint32_t) * cap);
  p.o_evec = take(cur, sizeof(float4) * cap);
  p.o_erev = take(cur, sizeof(int32_t) * cap);
  p.o_edst = take(cur, sizeof(int32_t) * cap);
  if (hp) {
    const int64_t C = hp->channels, L = hp->l_max, nlm = (L + 1) * (L + 1), S = hp->n_species;
    p.o_g = take(cur, sizeof(float4) * cap);
    p.o_ht1 = take(cur, sizeof(float) * S * C);
    p.o_h = take(cur, sizeof(float) * N * nlm * C);
    p.o_A = take(cur, sizeof(float) * N * nlm * C);
    p.o_hbar = take(cur, sizeof(float) * N * nlm * C);
    p.o_htbar = take(cur, sizeof(float) * N * nlm * C);
    for (int t = 1; t <= K; ++t) {
      p.o_ht.push_back(t >= 2 ? take(cur, sizeof(float) * N * nlm * C) : 0);
      p.o_z0.push_back(take(cur, sizeof(float) * N * C * (1 + L)));
      p.o_zl.push_back(t < K ? take(cur, sizeof(float) * N * (nlm - 1) * C) : 0);
    }
    if ((C == 64 || C == 128) && S * nlm <= 64 && K >= 2)
      p.o_qp = take(cur, sizeof(float) * N * nlm * 64 * S);
    if ((C == 64 || C == 128) && K >= 2)
      p.o_msg = take(cur, (prec == MPIP_BF16_MIXED ? sizeof(uint16_t) : sizeof(float)) * cap * C);
    if (K >= 3) p.o_part = take(cur, sizeof(float) * kPartStride * cap);
    p.o_atom_e = take(cur, sizeof(double) * N);
    p.nblocks_out = (int)((N + kOutRowsPerBlock - 1) / kOutRowsPerBlock);
    p.o_partials = take(cur, sizeof(double) * 10 * p.nblocks_out);
  }
  p.total = cur + 256;
  return p;
}

mpip_status check_system(const mpip_system* sys, CellInfo* ci, double rc, int n_species) {
  if (!sys) return fail(MPIP_EINVAL, "null system");
  if (sys->n_atoms < 1 || sys->n_atoms > (int64_t)1 << 30) return fail(MPIP_EINVAL, "n_atoms out of range");
  if (sys->n_owned < 0 || sys->n_owned > sys->n_atoms) return fail(MPIP_EINVAL, "n_owned out of range");
  if (!sys->positions || !sys->species) return fail(MPIP_EINVAL, "null positions or species");
  for (int k = 0; k < 9; ++k) {
    if (!std::isfinite(sys->cell[k])) return fail(MPIP_ECELL, "non-finite cell");
    ci->cell[k] = sys->cell[k];
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      if (r != c && sys->cell[3 * r + c] != 0.0)
        return fail(MPIP_EUNSUPPORTED, "only orthorhombic cells are supported");
  for (int d = 0; d < 3; ++d) {
    ci->pbc[d] = sys->pbc[d] ? 1 : 0;
    ci->L[d] = sys->cell[4 * d];
    if (ci->pbc[d] && !(ci->L[d] > 0.0)) return fail(MPIP_ECELL, "periodic cell length must be positive");
  }
  ci->rc = rc;
  ci->n_species = n_species;
  return MPIP_OK;
}

NbrBuffers nbr_buffers(char* ws, const Plan& p) {
  NbrBuffers b;
  b.status = (int64_t*)(ws + p.o_status);
  b.bounds = (double*)(ws + p.o_bounds);
  b.grid = (GridParams*)(ws + p.o_grid);
  b.max_bins = p.max_bins;
  b.bin_count = (int32_t*)(ws + p.o_bcount);
  b.bin_cursor = (int32_t*)(ws + p.o_bcursor);
  b.bin_start = (int32_t*)(ws + p.o_bstart);
  b.rank_count = (int32_t*)(ws + p.o_rcount);
  b.rank_start = (int32_t*)(ws + p.o_rstart);
  b.scan_tmp = (int32_t*)(ws + p.o_scan);
  b.info = (int4*)(ws + p.o_info);
  b.perm = (int32_t*)(ws + p.o_perm);
  b.inv_perm = (int32_t*)(ws + p.o_iperm);
  b.pos_s = (double*)(ws + p.o_pos);
  b.info_s = (int4*)(ws + p.o_info_s);
  b.ypos_s = (float4*)(ws + p.o_ypos);
  b.spec_s = (int32_t*)(ws + p.o_spec);
  b.owned_s = (uint8_t*)(ws + p.o_owned);
  b.cnt = (int32_t*)(ws + p.o_cnt);
  b.row_ptr = (int32_t*)(ws + p.o_row);
  b.blk = (int32_t*)(ws + p.o_blk);
  b.cmask = (uint64_t*)(ws + p.o_cmask);
  b.cand = p.N < ((int64_t)1 << 27) ? (uint32_t*)(ws + p.o_cand) : nullptr;
  b.e_src = (int32_t*)(ws + p.o_esrc);
  b.e_shift = (uint32_t*)(ws + p.o_eshift);
  b.e_vec = (float4*)(ws + p.o_evec);
  b.e_rev = (int32_t*)(ws + p.o_erev);
  b.e_dst = (int32_t*)(ws + p.o_edst);
  return b;
}

}  // namespace

extern "C" {

mpip_status mpip_workspace_size(const mpip_model* m, const mpip_system* sys, mpip_precision prec, int32_t K,
                                int64_t max_edges, size_t* bytes) {
  if (!m || !sys || !bytes) return fail(MPIP_EINVAL, "null argument");
  if (prec != MPIP_FP32 && prec != MPIP_BF16_MIXED) return fail(MPIP_EINVAL, "bad precision");
  if (K < 1 || K > m->hp.n_layers) return fail(MPIP_EINVAL, "K must be in 1..n_layers");
  if (max_edges < 0 || max_edges > ((int64_t)1 << 31) - 1) return fail(MPIP_EINVAL, "max_edges out of range");
  if (sys->n_atoms < 1) return fail(MPIP_EINVAL, "n_atoms must be >= 1");
  *bytes = make_plan(sys->n_atoms, max_edges, &m->hp, K, prec).total;
  return MPIP_OK;
}

size_t mpip_neighbor_workspace_size(int64_t n_atoms, int64_t capacity) {
  if (n_atoms < 1 || capacity < 0) return 0;
  return make_plan(n_atoms, capacity, nullptr, 0).total;
}

mpip_status mpip_workspace_status(const void* ws, void* stream, int64_t* n_edges) {
  if (!ws) return fail(MPIP_EINVAL, "null workspace");
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  int64_t st[ST_WORDS];
  HIPCHK(hipMemcpy(st, ws, sizeof(st), hipMemcpyDeviceToHost));
  if (n_edges) *n_edges = st[ST_NEDGES];
  const int64_t fl = st[ST_FLAGS];
  if (fl & FL_CAPACITY) return fail(MPIP_ECAPACITY, "edge capacity exceeded");
  if (fl & FL_SPECIES) return fail(MPIP_EINVAL, "species out of range");
  if (fl & FL_NONFINITE) return fail(MPIP_EINVAL, "non-finite position");
  if (fl & FL_COINCIDENT) return fail(MPIP_EINVAL, "coincident atoms");
  if (fl) return fail(MPIP_EINVAL, "data error");
  return MPIP_OK;
}

mpip_status mpip_neighbor_list(const mpip_system* sys, double r_cut, void* stream, void* ws, size_t ws_bytes,
                               int64_t capacity, int32_t* oi, int32_t* oj, int32_t* os, int64_t* n_edges) {
  CellInfo ci;
  mpip_status st = check_system(sys, &ci, r_cut, 1 << 30);
  if (st != MPIP_OK) return st;
  if (!(r_cut > 0.0)) return fail(MPIP_EINVAL, "r_cut must be positive");
  if (!ws || !n_edges || capacity < 0) return fail(MPIP_EINVAL, "bad workspace or outputs");
  if (capacity > 0 && (!oi || !oj || !os)) return fail(MPIP_EINVAL, "null edge outputs");
  Plan p = make_plan(sys->n_atoms, capacity, nullptr, 0);
  if (ws_bytes < p.total) return fail(MPIP_ECAPACITY, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  NbrBuffers b = nbr_buffers((char*)ws, p);
  launch_zero(b.status, sizeof(int64_t) * ST_WORDS, s);
  build_neighbors(b, *sys, ci, capacity, s);
  HIPCHK(hipGetLastError());
  int64_t ne = 0;
  st = mpip_workspace_status(ws, stream, &ne);
  *n_edges = ne;
  if (st != MPIP_OK) return st;
  export_neighbors(b, sys->n_atoms, capacity, oi, oj, os, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return MPIP_OK;
}

}  // extern "C"

// Layers forward, readout and the adjoint of all layers on a built CSR:
// leaves dE/dr_e, or the equivalent h_e of FastArgs::g2p, in the workspace
// (g) and per-atom energies (atom_e).
// rows: null, or rows[t] (t = 0..K) = the row prefix that layer t updates on
// a share whose rows are sorted by hop class (receptive-field trimming):
// layer t's receivers are rows < rows[t], and the passes that act on senders
// (features into layer t, the adjoint's pull) cover rows < rows[t - 1].
static void run_model(mpip_model* m, const Plan& p, char* w, const NbrBuffers& b, int64_t N,
                               mpip_precision prec, int32_t K, int64_t max_edges, hipStream_t s,
                               const int64_t* rows = nullptr) {
  const mpip_hparams& hp = m->hp;
  const int C = hp.channels, L = hp.l_max, nlm = (L + 1) * (L + 1), S = hp.n_species;
  const int pi = prec == MPIP_BF16_MIXED ? 1 : 0;
  const std::vector<LayerDev>& LD = m->layers[pi];
  float* ht1 = (float*)(w + p.o_ht1);
  float* h = (float*)(w + p.o_h);
  float* A = (float*)(w + p.o_A);
  float* hbar = (float*)(w + p.o_hbar);
  float* htbar = (float*)(w + p.o_htbar);
  float4* g = (float4*)(w + p.o_g);
  double* atom_e = (double*)(w + p.o_atom_e);
  PhaseTimer& T = m->timer;
  // rows layer t updates (R(0) = N: layer-1 senders are all atoms)
  auto R = [&](int t) -> int64_t { return rows ? rows[t] : N; };
  // zero rows [r0, N) of an array with `width` floats per row
  auto zero_rows = [&](float* base, int64_t r0, int64_t width) {
    if (r0 < N) launch_zero(base + r0 * width, sizeof(float) * (size_t)((N - r0) * width), s);
  };
  EdgeArgs ea;
  ea.n = N;
  ea.row_ptr = b.row_ptr;
  ea.e_src = b.e_src;
  ea.e_vec = b.e_vec;
  ea.spec_s = b.spec_s;
  ea.capacity = max_edges;
  ea.status = b.status;
  ea.rc = (float)hp.r_cut;
  ea.inv_n = (float)hp.inv_avg_neighbors;
  ea.envelope_p = hp.envelope_p;
  ea.g = g;
  ea.htbar = htbar;
  ea.part = p.o_part ? (float*)(w + p.o_part) : nullptr;

  NodeArgs na;
  na.n = N; na.C = C; na.L = L; na.nlm = nlm;
  na.spec_s = b.spec_s; na.owned_s = b.owned_s;
  na.emb = m->emb; na.w_read = m->w_read; na.e0 = m->e0;
  na.h = h; na.hbar = hbar; na.atom_e = atom_e;

  auto gemm = [&](const float* x, int64_t xs, int64_t xr, float* y, int64_t ys, int64_t yr, int64_t M, int rpa,
                  int Kd, int Nout, int ldw, const void* wt, int accumulate, int y_bf16 = 0, int x_bf16 = 0) {
    GemmArgs ga{x, xs, xr, y, ys, yr, M, rpa, Kd, Nout, ldw, wt, accumulate, y_bf16, x_bf16};
    T.begin("node_gemm", s);
    launch_gemm(prec, ga, s);
    T.end(s);
  };
  // layer-1 input features depend on species only: ht1 = W_emb @ W_up[1][0]
  gemm(m->emb, C, 0, ht1, C, 0, S, 1, C, C, C, LD[0].up_t[0], 0);

  auto kind_of = [&](int t) {
    if (t == 1) return K == 1 ? KIND_ONLY : KIND_FIRST;
    return t == K ? KIND_LAST : KIND_MID;
  };
  // specialised kernels: first layer (species factorisation) and last layer
  const bool fast_cl = !m->force_generic && (C == 64 || C == 128);
  auto fast_layer = [&](int t) {
    const int kind = kind_of(t);
    if (!fast_cl) return false;
    if (kind == KIND_FIRST) return S <= 4;   // species-factorised kernels: S <= 4
    return kind == KIND_LAST;
  };
  const int KQ = 64 * S;
  float* qp = p.o_qp ? (float*)(w + p.o_qp) : nullptr;
  FastArgs fa;
  fa.n = N; fa.row_ptr = b.row_ptr; fa.e_src = b.e_src; fa.e_dst = b.e_dst; fa.e_rev = b.e_rev; fa.e_vec = b.e_vec; fa.capacity = max_edges;
  fa.status = b.status; fa.rc = (float)hp.r_cut; fa.envelope_p = hp.envelope_p; fa.n_species = S;
  fa.inv_n = (float)hp.inv_avg_neighbors; fa.Q = qp; fa.P = qp; fa.g = g; fa.htbar = htbar;
  fa.msg = p.o_msg ? (void*)(w + p.o_msg) : nullptr;
  fa.g2p = nullptr;
  fa.row_end = nullptr;
  // trimmed share: rows list the edges to root atoms first (ends in b.cnt)
  const int32_t* root_end = rows ? b.cnt : nullptr;
  auto set_fast = [&](const LayerDev& d, int role) {
    fa.w1a = d.w1a; fa.w2a = d.w2a; fa.w2b = d.w2b; fa.w1b = d.w1b; fa.w2f = d.w2f;
    fa.w3f = d.w3fp[role]; fa.w3t = d.w3t[role]; fa.w3b = d.w3bp[role]; fa.cg = d.cg[role];
    fa.w1r = d.w1r; fa.w2r = d.w2r; fa.w3r = d.w3r;
    fa.rtab = d.rtab; fa.rtab_scale = (float)(kRadTab / hp.r_cut);
  };
  const int ht_bf16 = prec == MPIP_BF16_MIXED ? 1 : 0;
  // two-layer evaluation with specialised first and last layers (BF16 form):
  // the node work between them runs in the fused kernels of k_node1.hip
  const bool node1 = ht_bf16 && K == 2 && fast_layer(1) && fast_layer(2) && LD[0].n1_vwt[0] != nullptr;
  fa.htbar_bf16 = node1 ? 1 : 0;
  // the last layer's node update fused with its adjoint (needs the messages of the BF16 form in A)
  const bool nodeK = node1 && fa.msg && LD[K - 1].nk_dt != nullptr;
  // FP32 form: the last layer runs sender side (messages, their sum, one fused adjoint)
  // (the message buffer and W3 copy exist whenever the last layer is specialised)
  const bool send32 = !ht_bf16 && fa.msg && fast_layer(K) && kind_of(K) == KIND_LAST && LD[K - 1].w3r != nullptr;
  // two specialised layers in the sender-side form: the last layer's edge
  // gradients go to the (then dead) message buffer and the first layer's
  // adjoint combines them
  if ((node1 && fa.msg) || (send32 && K == 2 && fast_layer(1))) fa.g2p = (float4*)fa.msg;
  NodeKArgs nk;
  nk.n = N; nk.nlm = nlm; nk.A = A; nk.h = h; nk.w_read = m->w_read; nk.e0 = m->e0;
  nk.spec_s = b.spec_s; nk.owned_s = b.owned_s; nk.atom_e = atom_e;
  nk.dt = LD[K - 1].nk_dt; nk.d = LD[K - 1].nk_d;
  nk.msg = nodeK && ht_bf16 ? (const unsigned short*)fa.msg : nullptr;
  nk.row_ptr = b.row_ptr;
  nk.inv_n = fa.inv_n;
  Node1Args n1;
  n1.n = N; n1.Q = qp; n1.P = qp; n1.h = h; n1.ht = node1 ? (void*)(w + p.o_ht[1]) : nullptr; n1.htbar = htbar;
  n1.spec_s = b.spec_s; n1.owned_s = b.owned_s; n1.emb = m->emb; n1.w_read = m->w_read;
  for (int l = 0; l < 3; ++l) {
    n1.vwt[l] = LD[0].n1_vwt[l]; n1.upt[l] = LD[0].n1_upt[l]; n1.up[l] = LD[0].n1_up[l]; n1.vw[l] = LD[0].n1_vw[l];
  }
  // element offset into an array stored in FP32, or in BF16 when bf is set
  auto at = [](float* base, int64_t elems, int bf) -> float* {
    return bf ? (float*)((uint16_t*)base + elems) : base + elems;
  };

  const int nz = C * (1 + L);
  for (int t = 1; t <= K; ++t) {
    const LayerDev& d = LD[t - 1];
    const int kind = kind_of(t), role = (t == K) ? 1 : 0;
    const int nout = (kind == KIND_ONLY || kind == KIND_LAST) ? 1 : nlm;
    const bool fast = fast_layer(t);
    float* ht = (t == 1) ? ht1 : (float*)(w + p.o_ht[t - 1]);
    if (t >= 2 && !node1)
      for (int l = 0; l <= L; ++l)
        gemm(h + l * l * C, (int64_t)nlm * C, C, at(ht, l * l * C, fast ? ht_bf16 : 0), (int64_t)nlm * C, C,
             R(t - 1) * (2 * l + 1), 2 * l + 1, C, C, C, d.up_t[l], 0, fast ? ht_bf16 : 0);
    // trimmed: the generic adjoint of layer t walks rows up to R(t - 1) and
    // reads the features of their neighbours (times a zero dA where the
    // receiver is outside layer t); rows it was not given must be finite
    if (rows && t >= 2 && !node1 && !fast) zero_rows(ht, R(t - 1), (int64_t)nlm * C);
    T.begin("edge_fwd_t" + std::to_string(t), s);
    if (fast) {
      set_fast(d, role);
      if (kind == KIND_FIRST) {
        fa.n = R(1);
        launch_l1(prec, L, true, fa, s);
      } else {
        fa.ht = ht; fa.A = A;
        if (ht_bf16 && fa.msg) {
          fa.n = R(K - 1);   // sender-side: rows whose features feed the roots
          fa.row_end = root_end;
          launch_l2(prec, C, L, 4, fa, s);
          fa.row_end = nullptr;
          if (!nodeK) {   // else the last-layer node pass sums the messages itself
            T.end(s);
            T.begin("edge_sum_t" + std::to_string(t), s);
            fa.n = R(K);
            launch_l2(prec, C, L, 5, fa, s);
          }
        } else {   // FP32 form (send32)
          fa.n = R(K - 1);
          fa.row_end = root_end;
          launch_l2_32(C, L, 0, fa, s);
          fa.row_end = nullptr;
          T.end(s);
          T.begin("edge_sum_t" + std::to_string(t), s);
          fa.n = R(K);
          launch_l2_32(C, L, 1, fa, s);
        }
      }
    } else {
      ea.w1a = d.w1a; ea.w2a = d.w2a; ea.w2b = d.w2b; ea.w1b = d.w1b;
      ea.w3f = d.w3f[role]; ea.w3b = d.w3b[role]; ea.cg = d.cg[role];
      ea.ht = ht; ea.A = A;
      ea.n = R(t);
      launch_edge_fwd(prec, C, L, kind, ea, s);
    }
    T.end(s);
    float* z0 = (float*)(w + p.o_z0[t - 1]);
    float* zl = t < K ? (float*)(w + p.o_zl[t - 1]) : nullptr;
    if (node1 && t == 1) {
      T.begin("node_fused", s);
      n1.n = R(1);
      launch_node1(true, C, L, S, n1, s);
      T.end(s);
      continue;
    }
    if (nodeK && t == K) {
      // node update, readout and their adjoint: atom energies, and dE/dA over A
      T.begin("node_last", s);
      nk.n = R(K);
      launch_nodeK(C, nk, s);
      T.end(s);
      continue;
    }
    const int64_t Mt = R(t);
    if (fast && kind == KIND_FIRST) {
      // z_l = Q_l (V_l W_down_l) (Q in BF16 in the BF16 form); the messages are never stored
      gemm(at(qp, 0, ht_bf16), (int64_t)nlm * KQ, 0, z0, nz, 0, Mt, 1, KQ, nz, KQ, d.vwt[0], 0, 0, ht_bf16);
      for (int l = 1; l <= L; ++l)
        gemm(at(qp, l * l * KQ, ht_bf16), (int64_t)nlm * KQ, KQ, zl + (l * l - 1) * C, (int64_t)(nlm - 1) * C, C,
             Mt * (2 * l + 1), 2 * l + 1, KQ, C, KQ, d.vwt[l], 0, 0, ht_bf16);
    } else {
      gemm(A, (int64_t)nout * C, 0, z0, nz, 0, Mt, 1, C, (t == K) ? C : nz, C, d.down_t[0], 0);
      if (t < K)
        for (int l = 1; l <= L; ++l)
          gemm(A + l * l * C, (int64_t)nlm * C, C, zl + (l * l - 1) * C, (int64_t)(nlm - 1) * C, C, Mt * (2 * l + 1),
               2 * l + 1, C, C, C, d.down_t[l], 0);
    }
    na.z0 = z0; na.zl = zl;
    na.n = Mt;
    T.begin("gates", s);
    launch_gate_fwd(na, t == 1, t == K, s);
    T.end(s);
  }
  if (!nodeK) {
    T.begin("gates", s);
    na.n = R(K);
    launch_readout(na, s);
    T.end(s);
  }
  // atoms beyond the roots' receptive field get no energy
  if (rows && R(K) < N) launch_zero(atom_e + R(K), sizeof(double) * (size_t)(N - R(K)), s);

  // ---------------- adjoint ----------------
  T.begin("outputs", s);
  if (!fa.g2p) launch_zero(g, sizeof(float4) * (size_t)max_edges, s);
  // trimmed: the adjoint's pull adds into hbar rows up to R(K - 1), the
  // layer-K seed (gate adjoint) writes rows < R(K) only
  if (rows && !node1 && K >= 2) zero_rows(hbar, R(K), (int64_t)nlm * C);
  T.end(s);
  for (int t = K; t >= 1; --t) {
    const LayerDev& d = LD[t - 1];
    const int kind = kind_of(t), role = (t == K) ? 1 : 0;
    const int nout = (kind == KIND_ONLY || kind == KIND_LAST) ? 1 : nlm;
    const bool fast = fast_layer(t);
    float* ht = (t == 1) ? ht1 : (float*)(w + p.o_ht[t - 1]);
    float* z0 = (float*)(w + p.o_z0[t - 1]);
    float* zl = t < K ? (float*)(w + p.o_zl[t - 1]) : nullptr;
    na.z0 = z0; na.zl = zl;
    if (node1 && t == 1) {
      T.begin("node_fused", s);
      n1.n = R(1);
      launch_node1(false, C, L, S, n1, s);
      T.end(s);
      T.begin("edge_bwd_t1", s);
      set_fast(d, role);
      fa.n = R(1);
      launch_l1(prec, L, false, fa, s);
      T.end(s);
      continue;
    }
    if (nodeK && t == K) {
      // dE/dA is already in A on the roots; the pull reads it on every receiver
      if (rows) zero_rows(A, R(K), (int64_t)nout * C);
      goto edge_adjoint;
    }
    na.n = R(t);
    T.begin("gates", s);
    launch_gate_bwd(na, t == K, (t == K && K >= 2 && !node1) ? 1 : 0, s);
    T.end(s);
    if (fast && kind == KIND_FIRST) {
      // P_l = zbar_l (V_l W_down_l)^T (P in BF16 in the BF16 form)
      gemm(z0, nz, 0, at(qp, 0, ht_bf16), (int64_t)nlm * KQ, 0, R(1), 1, nz, KQ, nz, d.vw[0], 0, ht_bf16);
      for (int l = 1; l <= L; ++l)
        gemm(zl + (l * l - 1) * C, (int64_t)(nlm - 1) * C, C, at(qp, l * l * KQ, ht_bf16), (int64_t)nlm * KQ, KQ,
             R(1) * (2 * l + 1), 2 * l + 1, C, KQ, C, d.vw[l], 0, ht_bf16);
    } else {
      // Abar (in A) = zbar @ W_down^T; zero beyond layer t's receivers
      gemm(z0, nz, 0, A, (int64_t)nout * C, 0, R(t), 1, (t == K) ? C : nz, C, nz, d.down[0], 0);
      if (t < K)
        for (int l = 1; l <= L; ++l)
          gemm(zl + (l * l - 1) * C, (int64_t)(nlm - 1) * C, C, A + l * l * C, (int64_t)nlm * C, C, R(t) * (2 * l + 1),
               2 * l + 1, C, C, C, d.down[l], 0);
      if (rows) zero_rows(A, R(t), (int64_t)nout * C);
    }
  edge_adjoint:
    T.begin("edge_bwd_t" + std::to_string(t), s);
    if (fast) {
      set_fast(d, role);
      if (kind == KIND_FIRST) {
        fa.n = R(1);
        launch_l1(prec, L, false, fa, s);
      } else {
        fa.ht = ht; fa.Abar = A;
        // the BF16 adjoint reads dA / n_avg, which the fused last-layer node
        // kernel writes; after the generic node adjoint, scale here
        if (ht_bf16 && !nodeK) launch_scale(A, (float)hp.inv_avg_neighbors, R(K) * (int64_t)C, s);
        fa.n = R(K - 1);   // sender-side
        fa.row_end = root_end;
        // the walked prefix gets its gradient slots written; the rest of
        // those rows (receivers with dA = 0) must read as zero
        if (root_end && fa.g2p) zero_row_tails(fa.g2p, b.row_ptr, root_end, R(K - 1), N, max_edges, s);
        if (ht_bf16) launch_l2(prec, C, L, 3, fa, s);
        else launch_l2_32(C, L, 2, fa, s);
        fa.row_end = nullptr;
      }
    } else {
      ea.w1a = d.w1a; ea.w2a = d.w2a; ea.w2b = d.w2b; ea.w1b = d.w1b;
      ea.w3f = d.w3f[role]; ea.w3b = d.w3b[role]; ea.cg = d.cg[role];
      ea.ht = ht; ea.Abar = A;
      // every row with a receiver of layer t among its neighbours
      ea.n = R(t - 1);
      launch_edge_bwd(prec, C, L, kind, ea, s);
    }
    T.end(s);
    if (t >= 2 && !node1)
      for (int l = 0; l <= L; ++l)
        gemm(htbar + l * l * C, (int64_t)nlm * C, C, hbar + l * l * C, (int64_t)nlm * C, C, R(t - 1) * (2 * l + 1),
             2 * l + 1, C, C, C, d.up[l], 1);
  }
  if (rows && fa.g2p) {
    // g is written, not accumulated, on the rows the first layer's adjoint
    // walked (it reads g2p there only, where the last layer's adjoint wrote
    // it); the rest must read as zero
    zero_edges_from(g, b.row_ptr, R(1), N, max_edges, s);
  }
}


// the model, its adjoint and the outputs on the neighbour list already in b
static void eval_on_list(mpip_model* m, const Plan& p, char* w, const NbrBuffers& b, int64_t N, mpip_precision prec,
                         int32_t K, int64_t max_edges, hipStream_t s, const mpip_outputs* out,
                         const int64_t* rows = nullptr) {
  PhaseTimer& T = m->timer;
  run_model(m, p, w, b, N, prec, K, max_edges, s, rows);
  OutArgs oa;
  oa.n = N; oa.row_ptr = b.row_ptr; oa.e_vec = b.e_vec; oa.g = (float4*)(w + p.o_g); oa.e_rev = b.e_rev;
  oa.perm = b.perm; oa.owned_s = b.owned_s; oa.atom_e = (double*)(w + p.o_atom_e); oa.capacity = max_edges;
  oa.status = b.status; oa.partials = (double*)(w + p.o_partials); oa.nblocks = p.nblocks_out;
  oa.forces = out->forces; oa.atom_energy = out->atom_energy; oa.energy = out->energy; oa.virial = out->virial;
  T.begin("outputs", s);
  launch_outputs(oa, s);
  T.end(s);
}

static mpip_status evaluate_impl(mpip_model* m, const mpip_system* sys, mpip_precision prec, int32_t K,
                                 void* stream, void* ws, size_t ws_bytes, int64_t max_edges,
                                 const mpip_outputs* out) {
  if (!m) return fail(MPIP_EINVAL, "null model");
  const mpip_hparams& hp = m->hp;
  CellInfo ci;
  mpip_status st = check_system(sys, &ci, hp.r_cut, hp.n_species);
  if (st != MPIP_OK) return st;
  if (prec != MPIP_FP32 && prec != MPIP_BF16_MIXED) return fail(MPIP_EINVAL, "bad precision");
  if (K < 1 || K > hp.n_layers) return fail(MPIP_EINVAL, "K must be in 1..n_layers");
  if (!out || !out->energy || !out->forces || !out->virial) return fail(MPIP_EINVAL, "null output buffer");
  if (!ws) return fail(MPIP_EINVAL, "null workspace");
  if (max_edges < 0 || max_edges > ((int64_t)1 << 31) - 1) return fail(MPIP_EINVAL, "max_edges out of range");
  const int64_t N = sys->n_atoms;
  Plan p = make_plan(N, max_edges, &hp, K, prec);
  if (ws_bytes < p.total) return fail(MPIP_ECAPACITY, "workspace too small");
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  if (cur != m->device) HIPCHK(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  NbrBuffers b = nbr_buffers(w, p);
  float4* g = (float4*)(w + p.o_g);
  double* atom_e = (double*)(w + p.o_atom_e);

  PhaseTimer& T = m->timer;
  launch_zero(b.status, sizeof(int64_t) * ST_WORDS, s);
  T.begin("neighbors", s);
  build_neighbors(b, *sys, ci, max_edges, s);
  T.end(s);
  (void)atom_e;
  int64_t rows[16 + 1];
  bool trimmed = false;
  if (sys->n_owned > 0 && sys->n_owned < N && N >= trim_min_atoms() && K <= trim_max_layers()) {
    // receptive-field trimming of a partition share: hop classes from the
    // roots, read back once, then the rows are re-ordered by class
    T.begin("trim", s);
    const int64_t* d = trim_classes(b, N, K, max_edges, s);
    T.end(s);
    int64_t hb[16 + 3];
    HIPCHK(hipMemcpyAsync(hb, d, sizeof(int64_t) * (K + 3), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hb[K + 2] == 0) {   // else the list is unusable and every pass skips on the status word
      T.begin("trim", s);
      trim_permute(b, N, max_edges, g, s);
      T.end(s);
      trimmed = true;
      for (int t = 0; t <= K; ++t) rows[t] = hb[K - t + 1];
    }
  }
  eval_on_list(m, p, w, b, N, prec, K, max_edges, s, out, trimmed ? rows : nullptr);
  hipError_t e = hipGetLastError();
  if (cur != m->device) hipSetDevice(cur);
  if (e != hipSuccess) return fail(MPIP_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return MPIP_OK;
}

extern "C" {

mpip_status mpip_evaluate(mpip_model* m, const mpip_system* sys, mpip_precision prec, int32_t K, void* stream,
                          void* ws, size_t ws_bytes, int64_t max_edges, const mpip_outputs* out) {
  return evaluate_impl(m, sys, prec, K, stream, ws, ws_bytes, max_edges, out);
}

mpip_status mpip_evaluate_noalloc(mpip_model* m, const mpip_system* sys, mpip_precision prec, int32_t K,
                                  void* stream, int64_t max_edges, const mpip_outputs* out) {
  if (!m) return fail(MPIP_EINVAL, "null model");
  if (!sys || sys->n_atoms < 1) return fail(MPIP_EINVAL, "null system or n_atoms < 1");
  if (K < 1 || K > m->hp.n_layers) return fail(MPIP_EINVAL, "K must be in 1..n_layers");
  if (max_edges < 0 || max_edges > ((int64_t)1 << 31) - 1) return fail(MPIP_EINVAL, "max_edges out of range");
  const size_t need = make_plan(sys->n_atoms, max_edges, &m->hp, K, prec).total;
  if (need > kNoAllocScratchBytes)
    return fail(MPIP_ECAPACITY, "mpip_evaluate_noalloc: this system needs " + std::to_string(need) +
                                    " bytes of workspace; the static scratch holds " +
                                    std::to_string(kNoAllocScratchBytes));
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  if (cur != m->device) HIPCHK(hipSetDevice(m->device));
  void* ws = nullptr;
  const mpip_status st = scratch_address(m->device, &ws);
  if (cur != m->device) hipSetDevice(cur);
  if (st != MPIP_OK) return st;
  return evaluate_impl(m, sys, prec, K, stream, ws, kNoAllocScratchBytes, max_edges, out);
}

mpip_status mpip_timing_enable(mpip_model* m, int32_t on) {
  if (!m) return fail(MPIP_EINVAL, "null model");
  PhaseTimer& T = m->timer;
  T.on = on != 0;
  if (T.on) T.reserve(kTimingEvents);
  T.used = 0;
  T.pending.clear();
  T.names.clear();
  T.ms.clear();
  T.calls.clear();
  return MPIP_OK;
}

mpip_status mpip_timing_read(mpip_model* m, mpip_timing* out) {
  if (!m || !out) return fail(MPIP_EINVAL, "null argument");
  PhaseTimer& T = m->timer;
  for (const auto& pr : T.pending) {
    hipEvent_t a = T.pool[pr.second], b = T.pool[pr.second + 1];
    HIPCHK(hipEventSynchronize(b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    size_t k = 0;
    while (k < T.names.size() && T.names[k] != pr.first) ++k;
    if (k == T.names.size()) {
      T.names.push_back(pr.first);
      T.ms.push_back(0.0);
      T.calls.push_back(0);
    }
    T.ms[k] += ms;
    T.calls[k] += 1;
  }
  T.pending.clear();
  T.used = 0;
  std::memset(out, 0, sizeof(*out));
  out->n = (int32_t)std::min<size_t>(T.names.size(), MPIP_MAX_PHASES);
  for (int k = 0; k < out->n; ++k) {
    std::strncpy(out->name[k], T.names[k].c_str(), sizeof(out->name[k]) - 1);
    out->ms[k] = T.ms[k];
    out->calls[k] = T.calls[k];
  }
  return MPIP_OK;
}

static int slab_nimg(double L, double halo) { return (int)std::ceil(halo / L) + 1; }

size_t mpip_slab_workspace_size(int64_t n, double L, double halo) {
  if (n < 1 || !(L > 0.0) || !(halo >= 0.0)) return 0;
  const int ncat = 2 * slab_nimg(L, halo) + 2;
  size_t cur = 0;
  take(cur, sizeof(int32_t) * ncat * n);
  take(cur, sizeof(int32_t) * ncat * (n + 1));
  take(cur, sizeof(int32_t) * scan_tmp_elems(n + 1));
  take(cur, sizeof(int64_t) * (ncat + 1));
  return cur + 256;
}

// the share of slab `part`; hop (input order, device) != null keeps only the
// halo images of atoms within max_hop hops of a root
static mpip_status slab_share_impl(const double* pos, const int32_t* spec, int64_t n, const double* cell, int32_t axis,
                                   int32_t n_parts, int32_t part, double halo, void* stream, void* ws,
                                   size_t ws_bytes, int64_t capacity, double* out_pos, int32_t* out_spec,
                                   int32_t* out_idx, int64_t* n_local, int64_t* n_owned, const int32_t* hop,
                                   int max_hop) {
  if (!pos || !spec || !cell || !ws || !n_local || !n_owned) return fail(MPIP_EINVAL, "null argument");
  if (n < 1 || axis < 0 || axis > 2 || n_parts < 1 || part < 0 || part >= n_parts || !(halo >= 0.0))
    return fail(MPIP_EINVAL, "bad partition arguments");
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      if (r != c && cell[3 * r + c] != 0.0) return fail(MPIP_EUNSUPPORTED, "only orthorhombic cells are supported");
  const double L = cell[4 * axis];
  if (!(L > 0.0)) return fail(MPIP_ECELL, "cell length along the axis must be positive");
  if (capacity > 0 && (!out_pos || !out_spec || !out_idx)) return fail(MPIP_EINVAL, "null outputs");
  if (ws_bytes < mpip_slab_workspace_size(n, L, halo)) return fail(MPIP_ECAPACITY, "workspace too small");
  SlabArgs sa;
  sa.axis = axis; sa.P = n_parts; sa.part = part; sa.nimg = slab_nimg(L, halo); sa.L = L; sa.halo = halo;
  sa.capacity = capacity;
  sa.hop = hop;
  sa.max_hop = max_hop;
  const int ncat = 2 * sa.nimg + 2;
  size_t cur = 0;
  char* w = (char*)ws;
  int32_t* flags = (int32_t*)(w + take(cur, sizeof(int32_t) * ncat * n));
  int32_t* offs = (int32_t*)(w + take(cur, sizeof(int32_t) * ncat * (n + 1)));
  int32_t* tmp = (int32_t*)(w + take(cur, sizeof(int32_t) * scan_tmp_elems(n + 1)));
  int64_t* base = (int64_t*)(w + take(cur, sizeof(int64_t) * (ncat + 1)));
  hipStream_t s = (hipStream_t)stream;
  slab_share_launch(pos, spec, n, sa, flags, offs, tmp, s);
  HIPCHK(hipGetLastError());
  std::vector<int64_t> hb(ncat + 1, 0);
  for (int c = 0; c < ncat; ++c) {
    int32_t tot = 0;
    HIPCHK(hipMemcpyAsync(&tot, offs + (int64_t)c * (n + 1) + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    hb[c + 1] = hb[c] + tot;
  }
  *n_local = hb[ncat];
  *n_owned = hb[1];
  if (hb[ncat] > capacity) return fail(MPIP_ECAPACITY, "share larger than capacity");
  HIPCHK(hipMemcpyAsync(base, hb.data(), sizeof(int64_t) * (ncat + 1), hipMemcpyHostToDevice, s));
  slab_write_launch(pos, spec, n, sa, flags, offs, base, out_pos, out_spec, out_idx, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return MPIP_OK;
}

mpip_status mpip_slab_share(const double* pos, const int32_t* spec, int64_t n, const double* cell, int32_t axis,
                            int32_t n_parts, int32_t part, double halo, void* stream, void* ws, size_t ws_bytes,
                            int64_t capacity, double* out_pos, int32_t* out_spec, int32_t* out_idx,
                            int64_t* n_local, int64_t* n_owned) {
  return slab_share_impl(pos, spec, n, cell, axis, n_parts, part, halo, stream, ws, ws_bytes, capacity, out_pos,
                         out_spec, out_idx, n_local, n_owned, nullptr, 0);
}

// graph (K-hop) halo: the full structure's list at r_cut, K breadth-first
// levels from the slab's atoms, then the geometric share of depth K r_cut
// restricted to atoms within K hops
namespace {
struct BfsLayout {
  Plan nbr;
  size_t o_nbr, o_slab, o_hop, o_hin, total, slab_bytes;
};
BfsLayout bfs_layout(int64_t n, double L, int K, double r_cut, int64_t max_edges) {
  BfsLayout q;
  size_t cur = 0;
  q.nbr = make_plan(n, max_edges, nullptr, 0);
  q.o_nbr = take(cur, q.nbr.total);
  q.slab_bytes = mpip_slab_workspace_size(n, L, K * r_cut);
  q.o_slab = take(cur, q.slab_bytes);
  q.o_hop = take(cur, sizeof(int32_t) * n);
  q.o_hin = take(cur, sizeof(int32_t) * n);
  q.total = cur + 256;
  return q;
}
}  // namespace

size_t mpip_bfs_share_workspace_size(int64_t n_atoms, double axis_length, int32_t K, double r_cut,
                                     int64_t max_edges) {
  if (n_atoms < 1 || !(axis_length > 0.0) || K < 1 || !(r_cut > 0.0) || max_edges < 0) return 0;
  return bfs_layout(n_atoms, axis_length, K, r_cut, max_edges).total;
}

namespace {
mpip_status check_bfs(const mpip_system* sys, CellInfo* ci, double r_cut, int32_t axis, int32_t n_parts, int32_t K,
                      int64_t max_edges) {
  mpip_status st = check_system(sys, ci, r_cut, 1 << 30);
  if (st != MPIP_OK) return st;
  if (axis < 0 || axis > 2 || n_parts < 1 || K < 1 || !(r_cut > 0.0)) return fail(MPIP_EINVAL, "bad partition arguments");
  if (max_edges < 0 || max_edges > ((int64_t)1 << 31) - 1) return fail(MPIP_EINVAL, "max_edges out of range");
  if (!sys->pbc[axis]) return fail(MPIP_EUNSUPPORTED, "the split axis must be periodic");
  const double L = sys->cell[4 * axis];
  // one image per atom: the slab and both halo layers must fit in the box
  if (L / n_parts + 2.0 * K * r_cut > L) return fail(MPIP_EUNSUPPORTED, "slab plus halo wider than the cell");
  return MPIP_OK;
}

// the whole structure's list at r_cut (once for every part); *n_edges = its size
mpip_status bfs_build(const mpip_system* sys, const CellInfo& ci, const BfsLayout& q, char* w, int64_t max_edges,
                      hipStream_t s, int64_t* n_edges) {
  NbrBuffers b = nbr_buffers(w + q.o_nbr, q.nbr);
  launch_zero(b.status, sizeof(int64_t) * ST_WORDS, s);
  build_neighbors(b, *sys, ci, max_edges, s);
  HIPCHK(hipGetLastError());
  int64_t ne = 0;
  mpip_status st = mpip_workspace_status(w + q.o_nbr, s, &ne);
  if (n_edges) *n_edges = ne;
  return st;
}

// hops from the roots of slab `part` over the built list, then the share
mpip_status bfs_part(const mpip_system* sys, double r_cut, const BfsLayout& q, char* w, int32_t axis, int32_t n_parts,
                     int32_t part, int32_t K, int64_t max_edges, hipStream_t s, int64_t capacity, double* out_pos,
                     int32_t* out_spec, int32_t* out_idx, int64_t* n_local, int64_t* n_owned) {
  NbrBuffers b = nbr_buffers(w + q.o_nbr, q.nbr);
  SlabArgs sa;
  sa.axis = axis; sa.P = n_parts; sa.part = part; sa.L = sys->cell[4 * axis]; sa.nimg = 0; sa.halo = 0.0;
  sa.capacity = 0;
  int32_t* hop_in = (int32_t*)(w + q.o_hin);
  bfs_hops_launch(b, sys->n_atoms, sa, K, max_edges, (int32_t*)(w + q.o_hop), hop_in, s);
  HIPCHK(hipGetLastError());
  return slab_share_impl(sys->positions, sys->species, sys->n_atoms, sys->cell, axis, n_parts, part, K * r_cut, s,
                         w + q.o_slab, q.slab_bytes, capacity, out_pos, out_spec, out_idx, n_local, n_owned, hop_in, K);
}
}  // namespace

mpip_status mpip_bfs_share(const mpip_system* sys, double r_cut, int32_t axis, int32_t n_parts, int32_t part,
                           int32_t K, void* stream, void* ws, size_t ws_bytes, int64_t max_edges, int64_t capacity,
                           double* out_pos, int32_t* out_spec, int32_t* out_idx, int64_t* n_local,
                           int64_t* n_owned, int64_t* n_edges) {
  CellInfo ci;
  mpip_status st = check_bfs(sys, &ci, r_cut, axis, n_parts, K, max_edges);
  if (st != MPIP_OK) return st;
  if (!ws || !n_local || !n_owned) return fail(MPIP_EINVAL, "null argument");
  if (part < 0 || part >= n_parts) return fail(MPIP_EINVAL, "bad partition arguments");
  const BfsLayout q = bfs_layout(sys->n_atoms, sys->cell[4 * axis], K, r_cut, max_edges);
  if (ws_bytes < q.total) return fail(MPIP_ECAPACITY, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  st = bfs_build(sys, ci, q, (char*)ws, max_edges, s, n_edges);
  if (st != MPIP_OK) return st;
  return bfs_part(sys, r_cut, q, (char*)ws, axis, n_parts, part, K, max_edges, s, capacity, out_pos, out_spec,
                  out_idx, n_local, n_owned);
}

mpip_status mpip_accumulate_rows(const double* src, const int32_t* index, int64_t n_rows, int64_t n_dst,
                                 double* dst, void* stream) {
  if (n_rows < 0 || n_dst < 0) return fail(MPIP_EINVAL, "negative size");
  if (n_rows > 0 && (!src || !index || !dst)) return fail(MPIP_EINVAL, "null argument");
  accumulate_rows_launch(src, index, n_rows, n_dst, dst, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return MPIP_OK;
}

// ------------------------------------------------------- partitioned driver

namespace {
struct PartLayout {
  size_t o_slab, o_pos, o_spec, o_idx, o_e, o_w, o_f, o_ae, o_eval, total;
  size_t slab_bytes, eval_bytes;
  BfsLayout bfs;   // graph halo: the whole structure's list and hops (in the o_slab region)
};

PartLayout part_layout(const mpip_model* m, int64_t N, double L, double halo, int64_t max_local, int64_t max_edges,
                       int K, int64_t full_edges) {
  PartLayout q;
  size_t cur = 0;
  if (full_edges >= 0) {
    q.bfs = bfs_layout(N, L, K, m->hp.r_cut, full_edges);
    q.slab_bytes = q.bfs.total;
  } else {
    q.slab_bytes = mpip_slab_workspace_size(N, L, halo);
  }
  q.o_slab = take(cur, q.slab_bytes);
  q.o_pos = take(cur, sizeof(double) * 3 * max_local);
  q.o_spec = take(cur, sizeof(int32_t) * max_local);
  q.o_idx = take(cur, sizeof(int32_t) * max_local);
  q.o_e = take(cur, sizeof(double));
  q.o_w = take(cur, sizeof(double) * 9);
  q.o_f = take(cur, sizeof(double) * 3 * max_local);
  q.o_ae = take(cur, sizeof(double) * max_local);
  q.eval_bytes = make_plan(max_local, max_edges, &m->hp, K).total;   // sized for either precision
  q.o_eval = take(cur, q.eval_bytes);
  q.total = cur + 256;
  return q;
}

mpip_status check_partitioned(const mpip_model* m, const mpip_system* sys, int32_t K, int32_t n_parts, int32_t axis,
                              double halo, int64_t max_local, int64_t max_edges) {
  if (!m || !sys) return fail(MPIP_EINVAL, "null argument");
  if (K < 1 || K > m->hp.n_layers) return fail(MPIP_EINVAL, "K must be in 1..n_layers");
  if (n_parts < 1 || axis < 0 || axis > 2 || !(halo >= 0.0) || !std::isfinite(halo))
    return fail(MPIP_EINVAL, "bad partition arguments");
  if (sys->n_atoms < 1 || sys->n_owned != sys->n_atoms) return fail(MPIP_EINVAL, "every atom must be owned");
  if (!sys->pbc[axis]) return fail(MPIP_EUNSUPPORTED, "the split axis must be periodic");
  if (!(sys->cell[4 * axis] > 0.0)) return fail(MPIP_ECELL, "cell length along the axis must be positive");
  if (max_local < 1 || max_local > (int64_t)1 << 30) return fail(MPIP_EINVAL, "max_local out of range");
  if (max_edges < 0 || max_edges > ((int64_t)1 << 31) - 1) return fail(MPIP_EINVAL, "max_edges out of range");
  return MPIP_OK;
}
}  // namespace

mpip_status mpip_partitioned_workspace_size(const mpip_model* m, const mpip_system* sys, mpip_precision prec,
                                            int32_t K, int32_t n_parts, int32_t axis, double halo,
                                            int64_t graph_edges, int64_t max_local, int64_t max_edges,
                                            size_t* bytes) {
  (void)prec;
  mpip_status st = check_partitioned(m, sys, K, n_parts, axis, halo, max_local, max_edges);
  if (st != MPIP_OK) return st;
  if (!bytes) return fail(MPIP_EINVAL, "null argument");
  *bytes = part_layout(m, sys->n_atoms, sys->cell[4 * axis], halo, max_local, max_edges, K, graph_edges).total;
  return MPIP_OK;
}

mpip_status mpip_evaluate_partitioned(mpip_model* m, const mpip_system* sys, mpip_precision prec, int32_t K,
                                      int32_t n_parts, int32_t axis, double halo, int64_t graph_edges, void* stream,
                                      void* ws, size_t ws_bytes, int64_t max_local, int64_t max_edges,
                                      const mpip_outputs* out, int64_t* part_sizes) {
  mpip_status st = check_partitioned(m, sys, K, n_parts, axis, halo, max_local, max_edges);
  if (st != MPIP_OK) return st;
  if (!out || !out->energy || !out->forces || !out->virial) return fail(MPIP_EINVAL, "null output buffer");
  if (!ws) return fail(MPIP_EINVAL, "null workspace");
  const int64_t N = sys->n_atoms;
  const bool graph = graph_edges >= 0;
  CellInfo cib;
  if (graph) {
    st = check_bfs(sys, &cib, m->hp.r_cut, axis, n_parts, K, graph_edges);
    if (st != MPIP_OK) return st;
  }
  const PartLayout q = part_layout(m, N, sys->cell[4 * axis], halo, max_local, max_edges, K, graph_edges);
  if (ws_bytes < q.total) return fail(MPIP_ECAPACITY, "workspace too small");
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  if (cur != m->device) HIPCHK(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  double* lpos = (double*)(w + q.o_pos);
  int32_t* lspec = (int32_t*)(w + q.o_spec);
  int32_t* lidx = (int32_t*)(w + q.o_idx);
  double* le = (double*)(w + q.o_e);
  double* lw = (double*)(w + q.o_w);
  double* lf = (double*)(w + q.o_f);
  double* lae = (double*)(w + q.o_ae);
  launch_zero(out->energy, sizeof(double), s);
  launch_zero(out->virial, sizeof(double) * 9, s);
  launch_zero(out->forces, sizeof(double) * 3 * (size_t)N, s);
  if (out->atom_energy) launch_zero(out->atom_energy, sizeof(double) * (size_t)N, s);
  auto done = [&](mpip_status r) {
    if (cur != m->device) hipSetDevice(cur);
    return r;
  };
  if (graph) {
    // graph halo: the whole structure's list once, hops per part
    int64_t ne = 0;
    st = bfs_build(sys, cib, q.bfs, w + q.o_slab, graph_edges, s, &ne);
    if (st != MPIP_OK) {
      if (part_sizes) part_sizes[2] = ne;
      return done(st);
    }
  }
  for (int part = 0; part < n_parts; ++part) {
    int64_t nl = 0, no = 0;
    if (graph)
      st = bfs_part(sys, m->hp.r_cut, q.bfs, w + q.o_slab, axis, n_parts, part, K, graph_edges, s, max_local, lpos,
                    lspec, lidx, &nl, &no);
    else
      st = mpip_slab_share(sys->positions, sys->species, N, sys->cell, axis, n_parts, part, halo, s, w + q.o_slab,
                           q.slab_bytes, max_local, lpos, lspec, lidx, &nl, &no);
    if (part_sizes) { part_sizes[3 * part] = nl; part_sizes[3 * part + 1] = no; part_sizes[3 * part + 2] = 0; }
    if (st != MPIP_OK) return done(st);
    if (nl == 0) continue;
    mpip_system ss;
    ss.n_atoms = nl;
    ss.n_owned = no;
    ss.positions = lpos;
    ss.species = lspec;
    for (int k = 0; k < 9; ++k) ss.cell[k] = sys->cell[k];
    for (int d = 0; d < 3; ++d) ss.pbc[d] = d == axis ? 0 : sys->pbc[d];
    mpip_outputs so;
    so.energy = le; so.forces = lf; so.virial = lw; so.atom_energy = out->atom_energy ? lae : nullptr;
    st = mpip_evaluate(m, &ss, prec, K, s, w + q.o_eval, q.eval_bytes, max_edges, &so);
    if (st != MPIP_OK) return done(st);
    int64_t ne = 0;
    st = mpip_workspace_status(w + q.o_eval, s, &ne);
    if (part_sizes) part_sizes[3 * part + 2] = ne;
    if (st != MPIP_OK) return done(st);
    // output integration: partial forces of roots and halo images onto the
    // atoms they copy, root energy and virial summed, root atom energies
    accumulate_rows_launch(lf, lidx, nl, N, out->forces, s);
    add_energy_virial_launch(le, lw, out->energy, out->virial, s);
    if (out->atom_energy) scatter_scalars_launch(lae, lidx, no, N, out->atom_energy, s);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return done(fail(MPIP_EDEVICE, std::string("partitioned evaluation: ") + hipGetErrorString(e)));
  return done(MPIP_OK);
}

// ------------------------------------------------------------------ batches

static size_t batch_extra_offset(const Plan& p) { return (p.total + 255) & ~(size_t)255; }

static size_t batch_bytes(const Plan& p, int64_t N, int B) {
  size_t cur = batch_extra_offset(p);
  take(cur, sizeof(int32_t) * N);
  take(cur, sizeof(int64_t) * (B + 1));
  take(cur, sizeof(BatchCell) * B);
  return cur + 256;
}

mpip_status mpip_batch_workspace_size(const mpip_model* m, int64_t n_atoms, int32_t B, mpip_precision prec,
                                      int32_t K, int64_t max_edges, size_t* bytes) {
  if (!m || !bytes) return fail(MPIP_EINVAL, "null argument");
  if (n_atoms < 1 || B < 1 || K < 1 || K > m->hp.n_layers || max_edges < 0) return fail(MPIP_EINVAL, "bad sizes");
  if (prec != MPIP_FP32 && prec != MPIP_BF16_MIXED) return fail(MPIP_EINVAL, "bad precision");
  *bytes = batch_bytes(make_plan(n_atoms, max_edges, &m->hp, K, prec), n_atoms, B);
  return MPIP_OK;
}

mpip_status mpip_evaluate_batch(mpip_model* m, int32_t B, const int64_t* atom_ptr, const double* positions,
                                const int32_t* species, const double* cells, const uint8_t* pbc,
                                mpip_precision prec, int32_t K, void* stream, void* ws, size_t ws_bytes,
                                int64_t max_edges, double* energy, double* forces, double* virial) {
  if (!m || !atom_ptr || !positions || !species || !cells || !pbc || !ws || !energy || !forces || !virial)
    return fail(MPIP_EINVAL, "null argument");
  const mpip_hparams& hp = m->hp;
  if (B < 1) return fail(MPIP_EINVAL, "B must be >= 1");
  if (prec != MPIP_FP32 && prec != MPIP_BF16_MIXED) return fail(MPIP_EINVAL, "bad precision");
  if (K < 1 || K > hp.n_layers) return fail(MPIP_EINVAL, "K must be in 1..n_layers");
  if (max_edges < 0 || max_edges > ((int64_t)1 << 31) - 1) return fail(MPIP_EINVAL, "max_edges out of range");
  if (atom_ptr[0] != 0) return fail(MPIP_EINVAL, "atom_ptr[0] must be 0");
  std::vector<BatchCell> hc(B);
  for (int b = 0; b < B; ++b) {
    if (atom_ptr[b + 1] <= atom_ptr[b]) return fail(MPIP_EINVAL, "every structure needs at least one atom");
    BatchCell& c = hc[b];
    for (int k = 0; k < 9; ++k) {
      if (!std::isfinite(cells[9 * b + k])) return fail(MPIP_ECELL, "non-finite cell");
      c.cell[k] = cells[9 * b + k];
    }
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q)
        if (r != q && c.cell[3 * r + q] != 0.0) return fail(MPIP_EUNSUPPORTED, "only orthorhombic cells are supported");
    for (int d = 0; d < 3; ++d) {
      c.pbc[d] = pbc[3 * b + d] ? 1 : 0;
      c.L[d] = c.cell[4 * d];
      if (c.pbc[d] && !(c.L[d] > 0.0)) return fail(MPIP_ECELL, "periodic cell length must be positive");
      // positions are taken to their image in [0, L) before the search, so a
      // pair within r_cut has |S_d| < r_cut / L + 1; the slack covers the
      // rounding of the wrap
      c.img[d] = c.pbc[d] ? (int)std::ceil(hp.r_cut / c.L[d] + 1e-6) : 0;
      if (c.img[d] > 60) return fail(MPIP_ECELL, "cell too thin for the cutoff");
    }
  }
  const int64_t N = atom_ptr[B];
  if (N > ((int64_t)1 << 30)) return fail(MPIP_EINVAL, "too many atoms");
  Plan p = make_plan(N, max_edges, &hp, K, prec);
  if (ws_bytes < batch_bytes(p, N, B)) return fail(MPIP_ECAPACITY, "workspace too small");
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  if (cur != m->device) HIPCHK(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  NbrBuffers b = nbr_buffers(w, p);
  size_t off = batch_extra_offset(p);
  BatchBuffers bb;
  bb.sidx = (int32_t*)(w + take(off, sizeof(int32_t) * N));
  int64_t* dptr = (int64_t*)(w + take(off, sizeof(int64_t) * (B + 1)));
  BatchCell* dcells = (BatchCell*)(w + take(off, sizeof(BatchCell) * B));
  bb.ptr = dptr;
  bb.cells = dcells;
  PhaseTimer& T = m->timer;
  HIPCHK(hipMemcpyAsync(dptr, atom_ptr, sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dcells, hc.data(), sizeof(BatchCell) * B, hipMemcpyHostToDevice, s));
  launch_zero(b.status, sizeof(int64_t) * ST_WORDS, s);
  T.begin("neighbors", s);
  build_neighbors_batch(b, bb, B, positions, species, N, hp.n_species, hp.r_cut, max_edges, s);
  T.end(s);
  run_model(m, p, w, b, N, prec, K, max_edges, s);
  T.begin("outputs", s);
  launch_batch_outputs(N, B, b, (const float4*)(w + p.o_g), (const double*)(w + p.o_atom_e), bb, max_edges,
                       forces, energy, virial, s);
  T.end(s);
  hipError_t e = hipGetLastError();
  if (cur != m->device) hipSetDevice(cur);
  if (e != hipSuccess) return fail(MPIP_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return MPIP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- molecular dynamics

namespace {
struct MdScratch {
  size_t base, total;   // evaluation workspace bytes; plus the integrator's scratch
  size_t o_sticky, o_energy, o_virial, o_partials, o_flag;
  // neighbour list of radius r_c + skin and what its reuse needs (skin > 0)
  size_t o_srow = 0, o_ssrc = 0, o_sshift = 0, o_svec = 0, o_srev = 0, o_map = 0, o_xref = 0;
  int64_t sup_cap = 0;
  int nblocks;
};
int64_t skin_capacity(int64_t max_edges, double r_cut, double skin) {
  const double q = (r_cut + skin) / r_cut;
  // 1.5: a lattice shell just outside r_cut can make the ratio well above the volume ratio
  const double c = (double)max_edges * q * q * q * 1.5 + 1024.0;
  return c > 2147483000.0 ? 2147483000 : (int64_t)c;
}
MdScratch md_scratch(int64_t N, int64_t max_edges, const mpip_hparams* hp, int K, double skin) {
  MdScratch s;
  s.base = make_plan(N, max_edges, hp, K).total;
  size_t cur = s.base;
  s.nblocks = (int)((N + 255) / 256);
  s.o_sticky = take(cur, sizeof(int64_t));
  s.o_flag = take(cur, sizeof(int64_t));
  s.o_energy = take(cur, sizeof(double));
  s.o_virial = take(cur, 9 * sizeof(double));
  s.o_partials = take(cur, sizeof(double) * (size_t)s.nblocks);
  if (skin > 0.0) {
    s.sup_cap = skin_capacity(max_edges, hp->r_cut, skin);
    s.o_srow = take(cur, sizeof(int32_t) * (size_t)(N + 1));
    s.o_ssrc = take(cur, sizeof(int32_t) * (size_t)s.sup_cap);
    s.o_sshift = take(cur, sizeof(uint32_t) * (size_t)s.sup_cap);
    s.o_svec = take(cur, sizeof(float4) * (size_t)s.sup_cap);
    s.o_srev = take(cur, sizeof(int32_t) * (size_t)s.sup_cap);
    s.o_map = take(cur, sizeof(int32_t) * (size_t)s.sup_cap);
    s.o_xref = take(cur, sizeof(double) * 3 * (size_t)N);
  }
  s.total = cur + 256;
  return s;
}
}  // namespace

extern "C" {

mpip_status mpip_md_workspace_size(const mpip_model* m, const mpip_system* sys, const mpip_md_params* prm,
                                   mpip_precision prec, int32_t K, int64_t max_edges, size_t* bytes) {
  if (!prm) return fail(MPIP_EINVAL, "null params");
  size_t b = 0;
  const mpip_status st = mpip_workspace_size(m, sys, prec, K, max_edges, &b);
  if (st != MPIP_OK) return st;
  *bytes = md_scratch(sys->n_atoms, max_edges, &m->hp, K, prm->skin > 0.0 ? prm->skin : 0.0).total;
  return MPIP_OK;
}

mpip_status mpip_md_run(mpip_model* m, const mpip_system* sys, double* positions, double* velocities, double* forces,
                        const double* masses, const mpip_md_params* prm, mpip_precision prec, int32_t K,
                        void* stream, void* ws, size_t ws_bytes, int64_t max_edges, double* epot, double* ekin) {
  if (!m || !sys || !prm) return fail(MPIP_EINVAL, "null argument");
  if (!positions || !velocities || !forces || !masses) return fail(MPIP_EINVAL, "null positions, velocities, forces or masses");
  if (!(prm->dt > 0.0) || !std::isfinite(prm->dt)) return fail(MPIP_EINVAL, "dt must be positive");
  if (prm->n_steps < 0) return fail(MPIP_EINVAL, "n_steps must be >= 0");
  if (!(prm->friction >= 0.0) || !(prm->temperature >= 0.0)) return fail(MPIP_EINVAL, "friction and temperature must be >= 0");
  if (!(prm->skin >= 0.0) || !std::isfinite(prm->skin)) return fail(MPIP_EINVAL, "skin must be >= 0");
  if (prec != MPIP_FP32 && prec != MPIP_BF16_MIXED) return fail(MPIP_EINVAL, "bad precision");
  if (K < 1 || K > m->hp.n_layers) return fail(MPIP_EINVAL, "K must be in 1..n_layers");
  if (!ws) return fail(MPIP_EINVAL, "null workspace");
  if (max_edges < 0 || max_edges > ((int64_t)1 << 31) - 1) return fail(MPIP_EINVAL, "max_edges out of range");
  mpip_system s2 = *sys;
  s2.positions = positions;
  CellInfo ci;
  mpip_status st0 = check_system(&s2, &ci, m->hp.r_cut, m->hp.n_species);
  if (st0 != MPIP_OK) return st0;
  const int64_t N = sys->n_atoms;
  const bool skin = prm->skin > 0.0;
  const MdScratch sc = md_scratch(N, max_edges, &m->hp, K, skin ? prm->skin : 0.0);
  if (ws_bytes < sc.total) return fail(MPIP_ECAPACITY, "workspace too small");
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  if (cur != m->device) HIPCHK(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const Plan p = make_plan(N, max_edges, &m->hp, K);
  const NbrBuffers b = nbr_buffers(w, p);
  // the list of radius r_c + skin shares the atom order and scratch of b
  NbrBuffers sup = b;
  CellInfo ci_list = ci;
  if (skin) {
    sup.row_ptr = (int32_t*)(w + sc.o_srow);
    sup.e_src = (int32_t*)(w + sc.o_ssrc);
    sup.e_shift = (uint32_t*)(w + sc.o_sshift);
    sup.e_vec = (float4*)(w + sc.o_svec);
    sup.e_rev = (int32_t*)(w + sc.o_srev);
    ci_list.rc = m->hp.r_cut + prm->skin;
  }
  int32_t* map = skin ? (int32_t*)(w + sc.o_map) : nullptr;
  double* xref = skin ? (double*)(w + sc.o_xref) : nullptr;
  int64_t* moved = (int64_t*)(w + sc.o_flag);
  int64_t* sticky = (int64_t*)(w + sc.o_sticky);
  double* energy = (double*)(w + sc.o_energy);
  double* partials = (double*)(w + sc.o_partials);
  mpip_outputs out;
  out.energy = energy;
  out.forces = forces;
  out.virial = (double*)(w + sc.o_virial);
  out.atom_energy = nullptr;
  PhaseTimer& T = m->timer;
  launch_zero(sticky, sizeof(int64_t), s);
  // the list of the starting positions is built once and its status read
  // before anything moves: a capacity (or input) error returns here with the
  // positions, velocities and forces untouched
  if (prm->n_steps > 0) {
    launch_zero(b.status, sizeof(int64_t) * ST_WORDS, s);
    if (!skin) build_neighbors(b, s2, ci, max_edges, s);
    else build_neighbors(sup, s2, ci_list, sc.sup_cap, s);
    int64_t st[ST_WORDS];
    HIPCHK(hipMemcpyAsync(st, b.status, sizeof(st), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st[ST_FLAGS] != 0) {
      if (cur != m->device) hipSetDevice(cur);
      if (st[ST_FLAGS] & FL_CAPACITY)
        return fail(MPIP_ECAPACITY, "edge capacity exceeded by the starting positions (" +
                                        std::to_string(st[ST_NEDGES]) + " edges needed); nothing was moved");
      return fail(MPIP_EINVAL, "invalid starting positions or species; nothing was moved");
    }
  }
  bool rebuild = true;
  for (int64_t step = 0; step < prm->n_steps; ++step) {
    md_first(N, positions, velocities, forces, sys->species, masses, prm->dt, prm->friction, prm->temperature,
             prm->seed, step, xref, 0.25 * prm->skin * prm->skin, moved, s);
    if (skin && step > 0) {
      // the rebuild decision needs the displacement flag on the host; the
      // errors of the steps so far are read with it, and the run stops after
      // the first step whose list overflowed (positions and velocities are
      // then those after that step)
      int64_t f[2] = {0, 0};
      HIPCHK(hipMemcpyAsync(&f[0], moved, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(&f[1], sticky, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (f[1] != 0) break;
      rebuild = f[0] != 0;
    }
    launch_zero(b.status, sizeof(int64_t) * ST_WORDS, s);
    T.begin("neighbors", s);
    if (!skin) {
      build_neighbors(b, s2, ci, max_edges, s);
    } else {
      if (rebuild) {
        build_neighbors(sup, s2, ci_list, sc.sup_cap, s);
        md_reference(N, positions, xref, moved, s);
      } else {
        refresh_sorted(b, positions, N, s);
      }
      compact_list(b, sup, sc.sup_cap, map, ci, N, max_edges, s);
    }
    T.end(s);
    eval_on_list(m, p, w, b, N, prec, K, max_edges, s, &out);
    md_second(N, velocities, forces, sys->species, masses, prm->dt, partials, s);
    md_record(partials, sc.nblocks, energy, (const int64_t*)w, epot ? epot + step : nullptr,
              ekin ? ekin + step : nullptr, sticky, s);
  }
  md_flags(sticky, (int64_t*)w, s);
  hipError_t e = hipGetLastError();
  if (cur != m->device) hipSetDevice(cur);
  if (e != hipSuccess) return fail(MPIP_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return MPIP_OK;
}

}  // extern "C"
