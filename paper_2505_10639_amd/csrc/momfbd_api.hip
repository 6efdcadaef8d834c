// C-ABI layer of libmomfbd: argument checks, plan tables, workspace, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "bf16split.h"
#include "internal.h"
#include "momfbd.h"

using namespace mfbd;

enum KernelKind { KK_PHASE, KK_FORWARD, KK_OBJECT, KK_ADJOINT, KK_GRAD, KK_PREPARE, KK_OBJIMG,
                  KK_FILTER, KK_MOSAIC, KK_FWDOBJ, KK_COUNT };
static const char* kKernelNames[KK_COUNT] = {"phase", "forward", "object", "adjoint", "grad",
                                             "prepare", "objimg", "filter", "mosaic",
                                             "forward_object"};

// Optional kernel timing: an event pair around every launch, on its stream;
// or, with a repeat kind set, only around the launches of that kind, each
// issued `reps` times in a row inside its pair.
struct Profiler {
  bool on = false;
  int used = 0;
  int rep_kind = -1, reps = 1;
  std::vector<hipEvent_t> ev0, ev1;
  std::vector<int> kind, count;
};

struct momfbd_plan_s {
  Dims d;
  Profiler prof;
  ChanTab ct;
  int device = -1;
  int shift_y[kMaxC];      // translation applied to each channel's pupil
  int shift_x[kMaxC];
  float* Ab = nullptr;     // [C][N/2][N/2]    aperture on the band
  // the band modes in turns, split into three bf16 parts (bf16split.h),
  // eight values per uint4: Zs [C][Mp][(N/2)^2/8][3] (pixel index fastest,
  // rows M..Mp-1 zero) for the gradient, ZsT [C][(N/2)^2][Mq/8][3] (mode
  // index fastest, modes M..Mq-1 zero) for the phase
  uint4* Zs = nullptr;
  uint4* ZsT = nullptr;
  int Mp = 0;              // M rounded up to a multiple of 16
  int Mq = 0;              // M rounded up to a multiple of 32
  float* thetat = nullptr; // [C][N/2][N/2]    diversity in turns
  int* hflag = nullptr;    // pinned host word for the solver's "still searching" count
  int* supp = nullptr;     // [K][N/2+1] spectral support of each object (see LossArgs)
};

// Scratch of the allocation-free loss/gradient entry point: one fixed
// buffer per device, held from library load until the process ends.  In
// host code `scratch` names a host-side stand-in, not device memory; its
// device address is taken once per device (momfbd_plan_create, with that
// device current) and only that address is handed to kernels.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch, looked up on first use.
int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return MOMFBD_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return MOMFBD_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return MOMFBD_EDEVICE;
  }
  g_scratch_ptr[device] = ptr;
  return MOMFBD_OK;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

constexpr double kTwoPi = 6.283185307179586476925286766559;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool valid_dims(const momfbd_desc* d) {
  return d && d->P >= 1 && d->C >= 1 && d->K >= 1 && d->J >= 1 && d->M >= 1 && d->N >= 1 &&
         d->channel_object != nullptr;
}

// Bounding interval [lo, lo+len) of the rows (or columns) in use, allowing
// wrap-around: the shortest cyclic interval covering every used index.
bool cyclic_extent(const std::vector<char>& used, int N, int* start, int* len) {
  int count = 0;
  for (int i = 0; i < N; ++i) count += used[i] ? 1 : 0;
  if (count == 0) return false;
  // largest run of unused indices (cyclic) defines the complement
  int best_gap = 0, best_end = 0;
  for (int i = 0; i < N; ++i) {
    if (used[i]) continue;
    int g = 0;
    while (g < N && !used[(i + g) % N]) ++g;
    if (g > best_gap) {
      best_gap = g;
      best_end = (i + g) % N;
    }
  }
  *start = best_end;
  *len = N - best_gap;
  return true;
}

// Records a start event before and an end event after one launch when the
// plan's profiler is on (no effect otherwise).
// Issue one launch (the callable returns its hipError_t) under the plan's
// profiler.  Every kernel overwrites its outputs, so a repeated launch
// leaves the results unchanged.
template <class F>
hipError_t prof_launch(momfbd_plan plan, int kind, hipStream_t s, F&& launch) {
  Profiler& pr = plan->prof;
  const bool rep = pr.on && pr.rep_kind == kind;
  int slot = -1;
  if (pr.on && (pr.rep_kind < 0 || rep) && pr.used < (int)pr.ev0.size()) {
    slot = pr.used++;
    pr.kind[slot] = kind;
    pr.count[slot] = rep ? pr.reps : 1;
    (void)hipEventRecord(pr.ev0[slot], s);
  }
  hipError_t e = launch();
  for (int i = 1; rep && i < pr.reps && e == hipSuccess; ++i) e = launch();
  if (slot >= 0) (void)hipEventRecord(pr.ev1[slot], s);
  return e;
}

// A plan, and a workspace that is present, 256-byte aligned and at least
// momfbd_workspace_size bytes long; checked before anything is enqueued.
int check_call(momfbd_plan plan, const void* ws, size_t ws_bytes) {
  if (!plan) return MOMFBD_EINVAL;
  if (!ws) return MOMFBD_EWORKSPACE;
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return MOMFBD_EWORKSPACE;
  if (ws_bytes < workspace_bytes(plan->d)) return MOMFBD_EWORKSPACE;
  return MOMFBD_OK;
}

// The solver state: present, 256-byte aligned and large enough.
int check_state(const void* state, size_t state_bytes, size_t need) {
  if (!state) return MOMFBD_EINVAL;
  if (reinterpret_cast<uintptr_t>(state) % 256 != 0) return MOMFBD_EINVAL;
  if (state_bytes < need) return MOMFBD_EWORKSPACE;
  return MOMFBD_OK;
}

int to_status(hipError_t e) { return e == hipSuccess ? MOMFBD_OK : MOMFBD_EDEVICE; }

// Any error left by earlier asynchronous work is reported before new work.
int pending_error() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MOMFBD_OK : MOMFBD_EDEVICE;
}

}  // namespace

namespace mfbd {

size_t workspace_bytes(const Dims& d) {
  const size_t units = (size_t)d.P * d.C * d.J;
  const size_t hs = (size_t)d.N * (d.N / 2 + 1);
  size_t b = 0;
  const size_t bp = d.bandpix();
  b += align256(units * bp * sizeof(float));                 // phi
  b += align256(units * hs * sizeof(float2));                // S
  b += align256((size_t)d.P * d.K * hs * sizeof(float2));    // O
  b += align256(units * bp * sizeof(float));                 // gphi
  b += align256((size_t)d.P * d.K * object_blocks(d.N) * sizeof(double));  // loss_pk
  b += align256((size_t)kMaxGradSplits * d.P * d.J * d.M * sizeof(float));    // gpart
  return b;
}

Workspace carve_workspace(const Dims& d, void* base) {
  const size_t units = (size_t)d.P * d.C * d.J;
  const size_t hs = (size_t)d.N * (d.N / 2 + 1);
  const size_t bp = d.bandpix();
  char* p = static_cast<char*>(base);
  Workspace w;
  w.phi = reinterpret_cast<float*>(p);
  p += align256(units * bp * sizeof(float));
  w.S = reinterpret_cast<float2*>(p);
  p += align256(units * hs * sizeof(float2));
  w.O = reinterpret_cast<float2*>(p);
  p += align256((size_t)d.P * d.K * hs * sizeof(float2));
  w.gphi = reinterpret_cast<float*>(p);
  p += align256(units * bp * sizeof(float));
  w.loss_pk = reinterpret_cast<double*>(p);
  p += align256((size_t)d.P * d.K * object_blocks(d.N) * sizeof(double));
  w.gpart = reinterpret_cast<float*>(p);
  return w;
}

}  // namespace mfbd

static void profile_free(Profiler& pr);

extern "C" {

const char* momfbd_status_string(int status) {
  switch (status) {
    case MOMFBD_OK: return "ok";
    case MOMFBD_EINVAL: return "invalid argument";
    case MOMFBD_EUNSUPPORTED: return "unsupported configuration";
    case MOMFBD_EWORKSPACE: return "workspace missing, misaligned or too small";
    case MOMFBD_EDEVICE: return "HIP device error";
    case MOMFBD_ESCRATCH:
      return "problem needs more scratch than the allocation-free entry point's fixed buffer";
    default: return "unknown status";
  }
}

int momfbd_plan_create(const momfbd_desc* desc, const float* pupil, const float* basis,
                       const float* diversity, momfbd_plan* out) {
  if (!out) return MOMFBD_EINVAL;
  if (!valid_dims(desc) || !pupil || !basis) return MOMFBD_EINVAL;
  const int N = desc->N, C = desc->C, K = desc->K, M = desc->M, J = desc->J;
  if (C > kMaxC || K > kMaxK) return MOMFBD_EUNSUPPORTED;
  for (int c = 0; c < C; ++c)
    if (desc->channel_object[c] < 0 || desc->channel_object[c] >= K) return MOMFBD_EINVAL;
  for (int k = 0; k < K; ++k) {
    bool any = false;
    for (int c = 0; c < C; ++c) any |= desc->channel_object[c] == k;
    if (!any) return MOMFBD_EINVAL;
  }
  if (N != 64 && N != 96 && N != 128) return MOMFBD_EUNSUPPORTED;
  if (M > kMaxM || (long)J * M > 8192) return MOMFBD_EUNSUPPORTED;

  momfbd_plan_s* pl = new (std::nothrow) momfbd_plan_s();
  if (!pl) return MOMFBD_EDEVICE;
  pl->d = Dims{N, desc->P, C, K, J, M};
  std::memset(&pl->ct, 0, sizeof(pl->ct));
  int nfill = 0;
  for (int k = 0; k < K; ++k) {
    pl->ct.obj_first[k] = nfill;
    for (int c = 0; c < C; ++c)
      if (desc->channel_object[c] == k) pl->ct.obj_chans[nfill++] = c;
  }
  pl->ct.obj_first[K] = nfill;
  // the forward/object launch takes a (patch, object) per workgroup, one
  // wave per unit
  pl->d.fuse_ok = N == 64;
  for (int k = 0; k < K; ++k)
    if ((pl->ct.obj_first[k + 1] - pl->ct.obj_first[k]) * J > kFusedWaves) pl->d.fuse_ok = false;

  const int B = N / 2, B0 = N / 4;
  const size_t BP = (size_t)B * B;
  std::vector<float> hA((size_t)C * BP, 0.f), hT((size_t)C * BP, 0.f);
  std::vector<float> hZ((size_t)C * M * BP, 0.f);
  for (int c = 0; c < C; ++c) {
    pl->ct.chan_obj[c] = desc->channel_object[c];
    const float* A = pupil + (size_t)c * N * N;
    std::vector<char> rows(N, 0), cols(N, 0);
    double sumA2 = 0.0;
    for (int y = 0; y < N; ++y)
      for (int x = 0; x < N; ++x) {
        const float a = A[y * N + x];
        if (!(a >= 0.f) || !std::isfinite(a)) { delete pl; return MOMFBD_EINVAL; }
        if (a != 0.f) {
          rows[y] = cols[x] = 1;
          sumA2 += (double)a * a;
        }
      }
    int y0, ly, x0, lx;
    if (!cyclic_extent(rows, N, &y0, &ly) || !cyclic_extent(cols, N, &x0, &lx) || sumA2 <= 0.0) {
      delete pl;
      return MOMFBD_EINVAL;
    }
    if (ly > B || lx > B) { delete pl; return MOMFBD_EUNSUPPORTED; }
    // place the support at the start of the band, centred within it
    const int oy = (B - ly) / 2, ox = (B - lx) / 2;
    pl->shift_y[c] = B0 + oy - y0;
    pl->shift_x[c] = B0 + ox - x0;
    pl->ct.kappa[c] = (float)(1.0 / ((double)N * N * sumA2));
    for (int n = 0; n < B; ++n)
      for (int qx = 0; qx < B; ++qx) {
        const int y = ((y0 - oy + n) % N + N) % N, x = ((x0 - ox + qx) % N + N) % N;
        const size_t src = (size_t)y * N + x, dst = (size_t)n * B + qx;
        hA[(size_t)c * BP + dst] = A[src];
        const double th = diversity ? diversity[(size_t)c * N * N + src] : 0.0;
        hT[(size_t)c * BP + dst] = (float)(th / kTwoPi);
        for (int m = 0; m < M; ++m)
          hZ[((size_t)c * M + m) * BP + dst] =
              (float)((double)basis[((size_t)c * M + m) * N * N + src] / kTwoPi);
      }
  }
  // Spectral support of each object: a channel's OTF is nonzero only at
  // differences of two pupil pixels (its autocorrelation).  Each pair of
  // band rows contributes the differences between their column spans (the
  // span of a row with gaps covers more than its pixels, so the result may
  // exceed the support, never miss part of it); column kx keeps the largest
  // |row difference| that reaches it, the two signs of a difference giving
  // the same |kx| and |ky|.
  std::vector<int> hS((size_t)K * (B + 1), -1);
  for (int c = 0; c < C; ++c) {
    std::vector<int> lo(B, B), hi(B, -1);
    for (int n = 0; n < B; ++n)
      for (int qx = 0; qx < B; ++qx)
        if (hA[(size_t)c * BP + (size_t)n * B + qx] != 0.f) {
          lo[n] = std::min(lo[n], qx);
          hi[n] = std::max(hi[n], qx);
        }
    int* Fk = hS.data() + (size_t)desc->channel_object[c] * (B + 1);
    for (int y1 = 0; y1 < B; ++y1) {
      if (hi[y1] < 0) continue;
      for (int y2 = 0; y2 < B; ++y2) {
        if (hi[y2] < 0) continue;
        const int ady = std::abs(y2 - y1);
        for (int dx = lo[y2] - hi[y1]; dx <= hi[y2] - lo[y1]; ++dx)
          Fk[std::abs(dx)] = std::max(Fk[std::abs(dx)], ady);
      }
    }
  }
  // one basis for all channels when their band-sampled bases agree bit for bit
  bool shared = true;
  for (int c = 1; c < C && shared; ++c)
    shared = std::memcmp(hZ.data() + (size_t)c * M * BP, hZ.data(),
                         (size_t)M * BP * sizeof(float)) == 0;
  pl->d.zc = shared ? 1 : C;
  pl->Mp = (M + 15) / 16 * 16;
  pl->Mq = (M + 31) / 32 * 32;
  const int Mp = pl->Mp, Mq = pl->Mq;
  auto zval = [&](int c, int m, size_t px) {
    return m < M ? hZ[((size_t)c * M + m) * BP + px] : 0.f;
  };
  auto put = [](uint4* dst, const Split8& sp) {
    dst[0] = make_uint4(sp.h[0], sp.h[1], sp.h[2], sp.h[3]);
    dst[1] = make_uint4(sp.m[0], sp.m[1], sp.m[2], sp.m[3]);
    dst[2] = make_uint4(sp.l[0], sp.l[1], sp.l[2], sp.l[3]);
  };
  std::vector<uint4> hZs((size_t)C * Mp * (BP / 8) * 3), hZsT((size_t)C * BP * (Mq / 8) * 3);
  for (int c = 0; c < C; ++c) {
    for (int m = 0; m < Mp; ++m)
      for (size_t p8 = 0; p8 < BP / 8; ++p8) {
        float v[8];
        for (int e = 0; e < 8; ++e) v[e] = zval(c, m, 8 * p8 + e);
        put(&hZs[(((size_t)c * Mp + m) * (BP / 8) + p8) * 3], split8(v));
      }
    for (size_t px = 0; px < BP; ++px)
      for (int m8 = 0; m8 < Mq / 8; ++m8) {
        float v[8];
        for (int e = 0; e < 8; ++e) v[e] = zval(c, 8 * m8 + e, px);
        put(&hZsT[(((size_t)c * BP + px) * (Mq / 8) + m8) * 3], split8(v));
      }
  }
  if (hipGetDevice(&pl->device) != hipSuccess) { delete pl; return MOMFBD_EDEVICE; }
  // the scratch of momfbd_loss_grad_noalloc on this device (a failure here
  // only disables that entry point, which then reports EDEVICE)
  (void)scratch_setup(pl->device);
  if (hipHostMalloc(&pl->hflag, sizeof(int)) != hipSuccess) { delete pl; return MOMFBD_EDEVICE; }
  bool ok = hipMalloc(&pl->Ab, hA.size() * sizeof(float)) == hipSuccess &&
            hipMalloc(&pl->Zs, hZs.size() * sizeof(uint4)) == hipSuccess &&
            hipMalloc(&pl->thetat, hT.size() * sizeof(float)) == hipSuccess &&
            hipMalloc(&pl->ZsT, hZsT.size() * sizeof(uint4)) == hipSuccess &&
            hipMalloc(&pl->supp, hS.size() * sizeof(int)) == hipSuccess &&
            hipMemcpy(pl->supp, hS.data(), hS.size() * sizeof(int), hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMemcpy(pl->ZsT, hZsT.data(), hZsT.size() * sizeof(uint4), hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMemcpy(pl->Ab, hA.data(), hA.size() * sizeof(float), hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMemcpy(pl->Zs, hZs.data(), hZs.size() * sizeof(uint4), hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMemcpy(pl->thetat, hT.data(), hT.size() * sizeof(float), hipMemcpyHostToDevice) ==
                hipSuccess;
  if (!ok) {
    momfbd_plan_destroy(pl);
    return MOMFBD_EDEVICE;
  }
  *out = pl;
  return MOMFBD_OK;
}

int momfbd_plan_destroy(momfbd_plan plan) {
  if (!plan) return MOMFBD_OK;
  profile_free(plan->prof);
  if (plan->Ab) (void)hipFree(plan->Ab);
  if (plan->Zs) (void)hipFree(plan->Zs);
  if (plan->thetat) (void)hipFree(plan->thetat);
  if (plan->ZsT) (void)hipFree(plan->ZsT);
  if (plan->supp) (void)hipFree(plan->supp);
  if (plan->hflag) (void)hipHostFree(plan->hflag);
  delete plan;
  return MOMFBD_OK;
}

static bool tuning_ok(const momfbd_tuning* t) {
  return t && (t->xcd_forward == 0 || t->xcd_forward == 1) &&
         (t->xcd_adjoint == 0 || t->xcd_adjoint == 1) &&
         (t->object_pairs_per_thread == 1 || t->object_pairs_per_thread == 2 ||
          t->object_pairs_per_thread == 4) &&
         (t->grad_waves == 4 || t->grad_waves == 8) &&
         (t->grad_splits == 0 || t->grad_splits == 1 || t->grad_splits == 2 ||
          t->grad_splits == 4 || t->grad_splits == 8) &&
         (t->grad_row_tiles == 0 ||
          (t->grad_waves == 4 ? t->grad_row_tiles >= 2 && t->grad_row_tiles <= 4
                              : t->grad_row_tiles == 2)) &&
         (t->object_fused == 0 || t->object_fused == 1);
}

int momfbd_plan_set_tuning(momfbd_plan plan, const momfbd_tuning* t) {
  if (!plan || !tuning_ok(t)) return MOMFBD_EINVAL;
  // the automatic phase block, as get_tuning reports it, is accepted too
  Dims dauto = plan->d;
  dauto.phase_ct = dauto.phase_waves = 0;
  int act = 0, awaves = 0;
  phase_shape_of(dauto, plan->Mq, &act, &awaves);
  const bool phase_auto = (t->phase_col_tiles == 0 && t->phase_waves == 0) ||
                          (t->phase_col_tiles == act && t->phase_waves == awaves);
  if (!phase_auto && !phase_shape_fits(t->phase_col_tiles, t->phase_waves, plan->Mq))
    return MOMFBD_EINVAL;
  plan->d.phase_ct = phase_auto ? 0 : t->phase_col_tiles;
  plan->d.phase_waves = phase_auto ? 0 : t->phase_waves;
  plan->d.xcd_fwd = t->xcd_forward;
  plan->d.xcd_adj = t->xcd_adjoint;
  plan->d.obj_ppt = t->object_pairs_per_thread;
  plan->d.grad_waves = t->grad_waves;
  plan->d.grad_splits = t->grad_splits;
  plan->d.grad_rt = t->grad_row_tiles == 3 || t->grad_row_tiles == 2 ? t->grad_row_tiles : 0;
  plan->d.fuse_obj = t->object_fused;
  return MOMFBD_OK;
}

int momfbd_plan_get_tuning(momfbd_plan plan, momfbd_tuning* t) {
  if (!plan || !t) return MOMFBD_EINVAL;
  t->xcd_forward = plan->d.xcd_fwd;
  t->xcd_adjoint = plan->d.xcd_adj;
  t->object_pairs_per_thread = plan->d.obj_ppt;
  t->grad_waves = plan->d.grad_waves;
  t->grad_splits = grad_splits_of(plan->d);
  t->grad_row_tiles = grad_row_tiles_of(plan->d);
  phase_shape_of(plan->d, plan->Mq, &t->phase_col_tiles, &t->phase_waves);
  t->object_fused = fused_object(plan->d) ? 1 : 0;
  return MOMFBD_OK;
}

int momfbd_plan_dims(momfbd_plan plan, int* N, int* P, int* C, int* K, int* J, int* M) {
  if (!plan) return MOMFBD_EINVAL;
  if (N) *N = plan->d.N;
  if (P) *P = plan->d.P;
  if (C) *C = plan->d.C;
  if (K) *K = plan->d.K;
  if (J) *J = plan->d.J;
  if (M) *M = plan->d.M;
  return MOMFBD_OK;
}

int momfbd_workspace_size(momfbd_plan plan, size_t* bytes) {
  if (!plan || !bytes) return MOMFBD_EINVAL;
  *bytes = workspace_bytes(plan->d);
  return MOMFBD_OK;
}

int momfbd_prepare_data(momfbd_plan plan, const float* frames, int H, int W, int stride,
                        const float* apod, void* D, void* ws, size_t ws_bytes, void* stream) {
  int st = check_call(plan, ws, ws_bytes);
  if (st) return st;
  if (!frames || !apod || !D || stride < 1) return MOMFBD_EINVAL;
  const int N = plan->d.N;
  if (H < N || W < N) return MOMFBD_EINVAL;
  const long ny = (H - N) / stride + 1, nx = (W - N) / stride + 1;
  if (ny * nx != plan->d.P) return MOMFBD_EINVAL;
  if ((st = pending_error())) return st;
  hipStream_t s = (hipStream_t)stream;
  return to_status(prof_launch(plan, KK_PREPARE, s, [&] {
    return launch_prepare(plan->d, frames, H, W, stride, apod, static_cast<float2*>(D), s);
  }));
}

int momfbd_forward(momfbd_plan plan, const float* alpha, float* psf, void* otf, void* ws,
                   size_t ws_bytes, void* stream) {
  int st = check_call(plan, ws, ws_bytes);
  if (st) return st;
  if (!alpha || (!psf && !otf)) return MOMFBD_EINVAL;
  if ((st = pending_error())) return st;
  const Workspace w = carve_workspace(plan->d, ws);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = prof_launch(plan, KK_PHASE, s, [&] {
    return launch_phase(plan->d, alpha, plan->ZsT, plan->Mq, plan->thetat, w.phi, s);
  });
  if (e == hipSuccess)
    e = prof_launch(plan, KK_FORWARD, s, [&] {
      return launch_forward(plan->d, plan->ct, nullptr, plan->Ab, w.phi, psf,
                            otf ? static_cast<float2*>(otf) : w.S, s);
    });
  return to_status(e);
}

// (sum_loss false: the per-patch loss sum is left to the gradient stage)
static int run_object(momfbd_plan plan, const float* alpha, const void* D, const float* gamma,
                      float gamma_scalar, const float* weights, const int* active, double* loss,
                      void* ws, hipStream_t s, Workspace* wout, bool sum_loss = true) {
  const Workspace w = carve_workspace(plan->d, ws);
  LossArgs la{static_cast<const float2*>(D), gamma, gamma_scalar, weights, plan->supp};
  hipError_t e = prof_launch(plan, KK_PHASE, s, [&] {
    return launch_phase(plan->d, alpha, plan->ZsT, plan->Mq, plan->thetat, w.phi, s);
  });
  if (e == hipSuccess && fused_object(plan->d)) {
    e = prof_launch(plan, KK_FWDOBJ, s, [&] {
      return launch_fwdobj64(plan->d, plan->ct, la, active, plan->Ab, w.phi, w.S, w.O,
                             w.loss_pk, s);
    });
    if (e == hipSuccess && sum_loss)
      e = launch_loss_sum(loss_sum_of(plan->d, active, w.loss_pk, loss), s);
    *wout = w;
    return to_status(e);
  }
  if (e == hipSuccess)
    e = prof_launch(plan, KK_FORWARD, s, [&] {
      return launch_forward(plan->d, plan->ct, active, plan->Ab, w.phi, nullptr, w.S, s);
    });
  if (e == hipSuccess)
    e = prof_launch(plan, KK_OBJECT, s, [&] {
      return launch_object(plan->d, plan->ct, la, active, w.S, w.O, w.loss_pk, loss, s,
                           sum_loss);
    });
  *wout = w;
  return to_status(e);
}

// Loss and (if grad) gradient of the patches selected by `active` (all when null).
static int run_loss_grad(momfbd_plan plan, const float* alpha, const void* D, const float* gamma,
                         float gamma_scalar, const float* weights, const int* active,
                         double* loss, float* grad, void* ws, hipStream_t s) {
  Workspace w;
  int st = run_object(plan, alpha, D, gamma, gamma_scalar, weights, active, loss, ws, s, &w,
                      grad == nullptr);
  if (st || !grad) return st;
  LossArgs la{static_cast<const float2*>(D), gamma, gamma_scalar, weights, plan->supp};
  hipError_t e = prof_launch(plan, KK_ADJOINT, s, [&] {
    return launch_adjoint(plan->d, plan->ct, la, active, plan->Ab, w.phi, w.S, w.O, w.gphi, s);
  });
  // the gradient stage also sums the per-patch loss (in its combine launch)
  const LossSum ls = loss_sum_of(plan->d, active, w.loss_pk, loss);
  if (e == hipSuccess)
    e = prof_launch(plan, KK_GRAD, s, [&] {
      return launch_grad(plan->d, plan->Zs, w.gphi, grad, w.gpart, s, &ls);
    });
  return to_status(e);
}

int momfbd_loss_grad(momfbd_plan plan, const float* alpha, const void* D, const float* gamma,
                     float gamma_scalar, const float* weights, double* loss, float* grad,
                     void* ws, size_t ws_bytes, void* stream) {
  int st = check_call(plan, ws, ws_bytes);
  if (st) return st;
  if (!alpha || !D || !loss) return MOMFBD_EINVAL;
  if ((st = pending_error())) return st;
  return run_loss_grad(plan, alpha, D, gamma, gamma_scalar, weights, nullptr, loss, grad, ws,
                       (hipStream_t)stream);
}

int momfbd_loss_grad_noalloc(momfbd_plan plan, const float* alpha, const void* D,
                             const float* gamma, float gamma_scalar, const float* weights,
                             double* loss, float* grad, void* stream) {
  if (!plan) return MOMFBD_EINVAL;
  if (!alpha || !D || !loss) return MOMFBD_EINVAL;
  const size_t need = workspace_bytes(plan->d);
  if (need > kNoallocScratchBytes) return MOMFBD_ESCRATCH;
  void* ws = scratch_of(plan->device);
  if (!ws) return MOMFBD_EDEVICE;
  int st = pending_error();
  if (st) return st;
  return run_loss_grad(plan, alpha, D, gamma, gamma_scalar, weights, nullptr, loss, grad, ws,
                       (hipStream_t)stream);
}

int momfbd_smoothness_gamma(momfbd_plan plan, const float* gamma0, const float* lambda,
                            float* gamma, void* stream) {
  if (!plan || !gamma0 || !lambda || !gamma) return MOMFBD_EINVAL;
  PriorTab t;
  std::memset(&t, 0, sizeof(t));
  for (int k = 0; k < plan->d.K; ++k) {
    if (!(gamma0[k] >= 0.f) || !(lambda[k] >= 0.f) || !std::isfinite(gamma0[k]) ||
        !std::isfinite(lambda[k]))
      return MOMFBD_EINVAL;
    t.gamma0[k] = gamma0[k];
    t.lambda[k] = lambda[k];
  }
  int st = pending_error();
  if (st) return st;
  return to_status(launch_smoothness(plan->d.N, plan->d.K, t, gamma, (hipStream_t)stream));
}

int momfbd_object_estimate(momfbd_plan plan, const float* alpha, const void* D,
                           const float* gamma, float gamma_scalar, const float* weights,
                           float* obj, void* ws, size_t ws_bytes, void* stream) {
  int st = check_call(plan, ws, ws_bytes);
  if (st) return st;
  if (!alpha || !D || !obj) return MOMFBD_EINVAL;
  if ((st = pending_error())) return st;
  hipStream_t s = (hipStream_t)stream;
  Workspace w;
  // the per-patch loss is produced on the way; it lands in the gphi scratch
  double* scratch_loss = reinterpret_cast<double*>(carve_workspace(plan->d, ws).gphi);
  st = run_object(plan, alpha, D, gamma, gamma_scalar, weights, nullptr, scratch_loss, ws, s, &w);
  if (st) return st;
  return to_status(
      prof_launch(plan, KK_OBJIMG, s, [&] { return launch_objimg(plan->d, w.O, obj, s); }));
}

int momfbd_object_filtered(momfbd_plan plan, const float* alpha, const void* D,
                           const float* gamma, float gamma_scalar, const float* weights,
                           const momfbd_filter* filters, float* obj, float* H, void* ws,
                           size_t ws_bytes, void* stream) {
  int st = check_call(plan, ws, ws_bytes);
  if (st) return st;
  if (!alpha || !D || !obj || !filters) return MOMFBD_EINVAL;
  FilterTab ft;
  std::memset(&ft, 0, sizeof(ft));
  for (int k = 0; k < plan->d.K; ++k) {
    const momfbd_filter& f = filters[k];
    if (f.kind == MOMFBD_FILTER_TOPHAT) {
      if (!(f.f_lo >= 0.f) || !(f.f_hi > f.f_lo) || !(f.diff_limit > 0.f) ||
          !std::isfinite(f.f_hi) || !std::isfinite(f.diff_limit))
        return MOMFBD_EINVAL;
    } else if (f.kind == MOMFBD_FILTER_SCHARMER) {
      if (!(f.noise_power >= 0.f) || !std::isfinite(f.noise_power)) return MOMFBD_EINVAL;
    } else if (f.kind != MOMFBD_FILTER_NONE) {
      return MOMFBD_EINVAL;
    }
    ft.f[k] = FilterSpec{f.kind, f.f_lo, f.f_hi, f.diff_limit, f.noise_power};
  }
  if ((st = pending_error())) return st;
  hipStream_t s = (hipStream_t)stream;
  Workspace w;
  double* scratch_loss = reinterpret_cast<double*>(carve_workspace(plan->d, ws).gphi);
  st = run_object(plan, alpha, D, gamma, gamma_scalar, weights, nullptr, scratch_loss, ws, s, &w);
  if (st) return st;
  // the filter scales O in place; momfbd_profile_repeat refuses its kind
  hipError_t e = prof_launch(plan, KK_FILTER, s, [&] {
    return launch_filter(plan->d, plan->ct, ft, static_cast<const float2*>(D), weights, w.S, w.O,
                         H, s);
  });
  if (e != hipSuccess) return to_status(e);
  return to_status(
      prof_launch(plan, KK_OBJIMG, s, [&] { return launch_objimg(plan->d, w.O, obj, s); }));
}

int momfbd_synthesize(momfbd_plan plan, const float* alpha, const void* O, const float* noise,
                      const float* sigma, const float* apod, float* frames, void* D, void* ws,
                      size_t ws_bytes, void* stream) {
  int st = check_call(plan, ws, ws_bytes);
  if (st) return st;
  if (!alpha || !O || !noise || !sigma || !apod || !frames || !D) return MOMFBD_EINVAL;
  if ((st = pending_error())) return st;
  hipStream_t s = (hipStream_t)stream;
  const Workspace w = carve_workspace(plan->d, ws);
  const int N = plan->d.N;
  hipError_t e = launch_phase(plan->d, alpha, plan->ZsT, plan->Mq, plan->thetat, w.phi, s);
  if (e == hipSuccess) e = launch_forward(plan->d, plan->ct, nullptr, plan->Ab, w.phi, nullptr, w.S, s);
  if (e == hipSuccess)
    e = launch_synth(plan->d, plan->ct, static_cast<const float2*>(O), w.S, noise, sigma, frames,
                     s);
  if (e == hipSuccess)
    e = launch_prepare(plan->d, frames, plan->d.P * N, N, N, apod, static_cast<float2*>(D), s);
  return to_status(e);
}

int momfbd_mosaic(momfbd_plan plan, const float* obj, int ny, int nx, int stride, int border,
                  float* out, void* stream) {
  if (!plan || !obj || !out) return MOMFBD_EINVAL;
  const int N = plan->d.N;
  if (ny < 1 || nx < 1 || (long)ny * nx != plan->d.P || stride < 1 || stride > N || border < 0 ||
      border > N / 2)
    return MOMFBD_EINVAL;
  int st = pending_error();
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  return to_status(prof_launch(plan, KK_MOSAIC, s, [&] {
    return launch_mosaic(plan->d, obj, ny, nx, stride, border, out, s);
  }));
}

}  // extern "C"

static bool lbfgs_params_ok(const momfbd_lbfgs_params* pr) {
  return pr && pr->m >= 1 && pr->m <= 32 && pr->max_evals >= 1 && pr->max_evals <= 1000 &&
         pr->c1 > 0.0 && pr->c1 < pr->c2 && pr->c2 < 1.0 && pr->ftol >= 0.0;
}

extern "C" {

int momfbd_lbfgs_state_size(momfbd_plan plan, const momfbd_lbfgs_params* params, size_t* bytes) {
  if (!plan || !bytes || !lbfgs_params_ok(params)) return MOMFBD_EINVAL;
  *bytes = lbfgs_layout(plan->d, params->m, params->max_evals).total;
  return MOMFBD_OK;
}

int momfbd_lbfgs_init(momfbd_plan plan, const momfbd_lbfgs_params* params, void* state,
                      size_t state_bytes, const float* alpha, const void* D, const float* gamma,
                      float gamma_scalar, const float* weights, double* loss, void* ws,
                      size_t ws_bytes, void* stream) {
  int st = check_call(plan, ws, ws_bytes);
  if (st) return st;
  if (!lbfgs_params_ok(params) || !alpha || !D) return MOMFBD_EINVAL;
  const LbfgsLayout L = lbfgs_layout(plan->d, params->m, params->max_evals);
  if ((st = check_state(state, state_bytes, L.total))) return st;
  if ((st = pending_error())) return st;
  hipStream_t s = (hipStream_t)stream;
  char* b = static_cast<char*>(state);
  st = run_loss_grad(plan, alpha, D, gamma, gamma_scalar, weights, nullptr,
                     reinterpret_cast<double*>(b + L.ft), reinterpret_cast<float*>(b + L.g), ws, s);
  if (st) return st;
  return to_status(launch_lbfgs_init(plan->d, L, state, loss, s));
}

int momfbd_lbfgs_step(momfbd_plan plan, const momfbd_lbfgs_params* params, void* state,
                      size_t state_bytes, float* alpha, const void* D, const float* gamma,
                      float gamma_scalar, const float* weights, double* loss, int* status,
                      void* ws, size_t ws_bytes, void* stream) {
  int st = check_call(plan, ws, ws_bytes);
  if (st) return st;
  if (!lbfgs_params_ok(params) || !alpha || !D) return MOMFBD_EINVAL;
  const LbfgsLayout L = lbfgs_layout(plan->d, params->m, params->max_evals);
  if ((st = check_state(state, state_bytes, L.total))) return st;
  if ((st = pending_error())) return st;
  hipStream_t s = (hipStream_t)stream;
  char* b = static_cast<char*>(state);
  const int* active = reinterpret_cast<const int*>(b + L.active);
  const int* counter = reinterpret_cast<const int*>(b + L.counter);
  hipError_t e = launch_lbfgs_begin(plan->d, L, state, alpha, params->max_evals, s);
  for (int ev = 0; e == hipSuccess && ev < params->max_evals; ++ev) {
    st = run_loss_grad(plan, alpha, D, gamma, gamma_scalar, weights, active,
                       reinterpret_cast<double*>(b + L.ft), reinterpret_cast<float*>(b + L.gt), ws,
                       s);
    if (st) return st;
    e = launch_lbfgs_search(plan->d, L, state, alpha, ev, params->c1, params->c2,
                            params->max_evals, params->ftol, s);
    if (e != hipSuccess) break;
    // how many patches still search: decides whether another evaluation is needed
    e = hipMemcpyAsync(plan->hflag, counter + ev, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && *plan->hflag == 0) break;
  }
  if (e == hipSuccess) e = launch_lbfgs_finish(plan->d, L, state, loss, status, s);
  return to_status(e);
}

int momfbd_lbfgs_rounds(momfbd_plan plan, const momfbd_lbfgs_params* params, void* state,
                        size_t state_bytes, float* alpha, const void* D, const float* gamma,
                        float gamma_scalar, const float* weights, int rounds, double* loss,
                        int* status, float* alpha_accepted, void* ws, size_t ws_bytes,
                        void* stream) {
  int st = check_call(plan, ws, ws_bytes);
  if (st) return st;
  if (!lbfgs_params_ok(params) || !alpha || !D || rounds < 0) return MOMFBD_EINVAL;
  const LbfgsLayout L = lbfgs_layout(plan->d, params->m, params->max_evals);
  if ((st = check_state(state, state_bytes, L.total))) return st;
  if ((st = pending_error())) return st;
  hipStream_t s = (hipStream_t)stream;
  char* b = static_cast<char*>(state);
  const int* active = reinterpret_cast<const int*>(b + L.active);
  hipError_t e = hipSuccess;
  for (int r = 0; e == hipSuccess && r < rounds; ++r) {
    e = launch_lbfgs_prep(plan->d, L, state, alpha, s);
    if (e != hipSuccess) break;
    st = run_loss_grad(plan, alpha, D, gamma, gamma_scalar, weights, active,
                       reinterpret_cast<double*>(b + L.ft), reinterpret_cast<float*>(b + L.gt), ws,
                       s);
    if (st) return st;
    e = launch_lbfgs_search(plan->d, L, state, alpha, -1, params->c1, params->c2,
                            params->max_evals, params->ftol, s);
  }
  if (e == hipSuccess && alpha_accepted)
    e = launch_lbfgs_publish(plan->d, L, state, alpha, alpha_accepted, s);
  if (e == hipSuccess) e = launch_lbfgs_finish(plan->d, L, state, loss, status, s);
  return to_status(e);
}

// Greedy search over the launch schedules, one knob at a time, timing whole
// loss+gradient evaluations on the caller's data with events on `stream`.
int momfbd_plan_autotune(momfbd_plan plan, const float* alpha, const void* D, const float* gamma,
                         float gamma_scalar, const float* weights, int reps, double* loss,
                         float* grad, void* ws, size_t ws_bytes, void* stream,
                         momfbd_tuning* chosen) {
  int st = check_call(plan, ws, ws_bytes);
  if (st) return st;
  if (!alpha || !D || !loss || !grad || reps < 1) return MOMFBD_EINVAL;
  if ((st = pending_error())) return st;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreateWithFlags(&e0, hipEventReleaseToDevice) != hipSuccess ||
      hipEventCreateWithFlags(&e1, hipEventReleaseToDevice) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return MOMFBD_EDEVICE;
  }
  // A knob changes one kernel's launch only, so a candidate is timed by
  // that kernel alone: one whole evaluation under the candidate's schedule
  // fills the workspace, then the kernel runs 4 reps times back to back
  // (every kernel overwrites its outputs from unchanged inputs).
  const Workspace w = carve_workspace(plan->d, ws);
  const LossArgs la{static_cast<const float2*>(D), gamma, gamma_scalar, weights, plan->supp};
  auto launch_knob = [&](int knob) -> hipError_t {
    switch (knob) {
      case 0:
        return launch_adjoint(plan->d, plan->ct, la, nullptr, plan->Ab, w.phi, w.S, w.O, w.gphi,
                              s);
      case 1: return launch_forward(plan->d, plan->ct, nullptr, plan->Ab, w.phi, nullptr, w.S, s);
      case 2: return launch_object(plan->d, plan->ct, la, nullptr, w.S, w.O, w.loss_pk, loss, s);
      case 3: return launch_grad(plan->d, plan->Zs, w.gphi, grad, w.gpart, s);
      case 4: return launch_phase(plan->d, alpha, plan->ZsT, plan->Mq, plan->thetat, w.phi, s);
      default: {
        // the forward and object pass, in one launch or two
        if (fused_object(plan->d))
          return launch_fwdobj64(plan->d, plan->ct, la, nullptr, plan->Ab, w.phi, w.S, w.O,
                                 w.loss_pk, s);
        const hipError_t e =
            launch_forward(plan->d, plan->ct, nullptr, plan->Ab, w.phi, nullptr, w.S, s);
        return e != hipSuccess ? e
                               : launch_object(plan->d, plan->ct, la, nullptr, w.S, w.O,
                                               w.loss_pk, loss, s);
      }
    }
  };
  auto timed = [&](int knob, float* ms) -> int {
    int r = run_loss_grad(plan, alpha, D, gamma, gamma_scalar, weights, nullptr, loss, grad, ws, s);
    if (r) return r;
    if (hipEventRecord(e0, s) != hipSuccess) return MOMFBD_EDEVICE;
    for (int i = 0; i < 4 * reps; ++i)
      if (launch_knob(knob) != hipSuccess) return MOMFBD_EDEVICE;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess)
      return MOMFBD_EDEVICE;
    return MOMFBD_OK;
  };
  // Every candidate of a knob is timed once per round, the rounds
  // interleaved, and keeps its fastest round: a clock that is still rising,
  // or a transient slowdown, then favours no candidate.  The first value of
  // each knob is the library default; another value replaces the best so
  // far only when at least 1% faster, so that timing noise between
  // near-equal schedules does not decide (the XCD-grouped orders read less
  // from HBM at equal speed).
  // The gradient's shape is one knob: 4 waves with 4, 3 or 2 row tiles, or
  // 8 waves with 2 (each with its automatic split count); its split count
  // is the next knob, starting from the automatic one for the chosen shape,
  // the others following in increasing order.  After the last knob, one
  // whole evaluation under the chosen schedules leaves the loss and
  // gradient outputs of that schedule.  Knobs 0-5 time the adjoint, the
  // forward, the object kernel, (3, 4) the gradient contraction and (5) the
  // phase contraction, whose candidates are its automatic block and the
  // selectable blocks (4 x 8, 8 x 16 tiles x waves) that fit; knob 6, where
  // the plan allows it, the forward and object pass in two launches (the
  // default, under the schedules chosen for them) against one.
  constexpr int kRounds = 3;
  static const int kShapes[4][2] = {{4, 0}, {4, 3}, {4, 2}, {8, 0}};
  static const int kPhaseShapes[3][2] = {{0, 0}, {4, 8}, {8, 16}};
  auto set_knob = [&](int k, int v) {
    switch (k) {
      case 0: plan->d.xcd_adj = v; break;
      case 1: plan->d.xcd_fwd = v; break;
      case 2: plan->d.obj_ppt = v; break;
      case 3:
        plan->d.grad_waves = kShapes[v][0];
        plan->d.grad_rt = kShapes[v][1];
        plan->d.grad_splits = 0;
        break;
      case 4: plan->d.grad_splits = v; break;
      case 5:
        plan->d.phase_ct = kPhaseShapes[v][0];
        plan->d.phase_waves = kPhaseShapes[v][1];
        break;
      default: plan->d.fuse_obj = v; break;
    }
  };
  const Dims keep_d = plan->d;
  std::vector<int> values[7] = {{1, 0}, {0, 1}, {1, 2, 4}, {0, 1, 2, 3}, {}, {0}, {}};
  if (plan->d.fuse_ok) values[6] = {0, 1};
  for (int v = 1; v < 3; ++v)
    if (phase_shape_fits(kPhaseShapes[v][0], kPhaseShapes[v][1], plan->Mq)) values[5].push_back(v);
  for (int k = 0; k < 7 && st == MOMFBD_OK; ++k) {
    if (k == 6 && values[6].empty()) break;
    if (k == 4) {
      plan->d.grad_splits = 0;
      const int a = grad_splits_auto(plan->d);
      values[4] = {a};
      for (int v = 1; v <= kMaxGradSplits; v *= 2)
        if (v != a) values[4].push_back(v);
    }
    std::vector<float> fastest(values[k].size(), 0.f);
    for (int r = 0; r < kRounds && st == MOMFBD_OK; ++r) {
      for (size_t i = 0; i < values[k].size(); ++i) {
        set_knob(k, values[k][i]);
        float ms = 0.f;
        if ((st = timed(k < 3 ? k : k < 5 ? 3 : k - 1, &ms))) break;
        if (r == 0 || ms < fastest[i]) fastest[i] = ms;
      }
    }
    if (st) {
      plan->d = keep_d;
      break;
    }
    size_t best = 0;
    for (size_t i = 1; i < values[k].size(); ++i)
      if (fastest[i] < 0.99f * fastest[best]) best = i;
    set_knob(k, values[k][best]);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  st = run_loss_grad(plan, alpha, D, gamma, gamma_scalar, weights, nullptr, loss, grad, ws, s);
  if (st) return st;
  if (chosen) momfbd_plan_get_tuning(plan, chosen);
  return MOMFBD_OK;
}

}  // extern "C"

static void profile_free(Profiler& pr) {
  for (auto e : pr.ev0) (void)hipEventDestroy(e);
  for (auto e : pr.ev1) (void)hipEventDestroy(e);
  pr.ev0.clear();
  pr.ev1.clear();
  pr.kind.clear();
  pr.count.clear();
  pr.on = false;
  pr.used = 0;
  pr.rep_kind = -1;
  pr.reps = 1;
}

extern "C" {

int momfbd_profile_start(momfbd_plan plan, int max_launches) {
  if (!plan || max_launches < 1) return MOMFBD_EINVAL;
  profile_free(plan->prof);
  Profiler& pr = plan->prof;
  pr.ev0.resize(max_launches);
  pr.ev1.resize(max_launches);
  pr.kind.assign(max_launches, -1);
  pr.count.assign(max_launches, 0);
  pr.rep_kind = -1;
  pr.reps = 1;
  for (int i = 0; i < max_launches; ++i)
    if (hipEventCreateWithFlags(&pr.ev0[i], hipEventReleaseToDevice) != hipSuccess ||
        hipEventCreateWithFlags(&pr.ev1[i], hipEventReleaseToDevice) != hipSuccess) {
      pr.ev0.resize(i);
      pr.ev1.resize(i);
      profile_free(pr);
      return MOMFBD_EDEVICE;
    }
  pr.on = true;
  return MOMFBD_OK;
}

int momfbd_profile_repeat(momfbd_plan plan, const char* kind, int reps) {
  if (!plan || !kind || reps < 1 || !plan->prof.on) return MOMFBD_EINVAL;
  for (int k = 0; k < KK_COUNT; ++k) {
    if (std::strcmp(kind, kKernelNames[k]) != 0) continue;
    if (k == KK_FILTER) return MOMFBD_EINVAL;
    plan->prof.rep_kind = k;
    plan->prof.reps = reps;
    return MOMFBD_OK;
  }
  return MOMFBD_EINVAL;
}

int momfbd_profile_stop(momfbd_plan plan, int cap, const char** names, double* total_ms,
                        int* launches) {
  if (!plan || cap < 0 || (cap > 0 && (!names || !total_ms || !launches))) return MOMFBD_EINVAL;
  Profiler& pr = plan->prof;
  double tot[KK_COUNT] = {0};
  int cnt[KK_COUNT] = {0};
  int st = MOMFBD_OK;
  for (int i = 0; i < pr.used; ++i) {
    if (hipEventSynchronize(pr.ev1[i]) != hipSuccess) { st = MOMFBD_EDEVICE; break; }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pr.ev0[i], pr.ev1[i]) != hipSuccess) { st = MOMFBD_EDEVICE; break; }
    tot[pr.kind[i]] += ms;
    cnt[pr.kind[i]] += pr.count[i];
  }
  int n = 0;
  for (int k = 0; k < KK_COUNT && n < cap; ++k) {
    if (!cnt[k]) continue;
    names[n] = kKernelNames[k];
    total_ms[n] = tot[k];
    launches[n] = cnt[k];
    ++n;
  }
  profile_free(pr);
  return st ? st : n;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Groups: fields of one patch size solved together, one launch per stage.
// ---------------------------------------------------------------------------

struct momfbd_group_s {
  int n = 0, N = 0, device = -1;
  bool solver = false;
  momfbd_lbfgs_params params{};
  FieldDesc* fd_eval = nullptr;   // device [n]: evaluation into the bound loss/grad
  FieldDesc* fd_solve = nullptr;  // device [n]: solver trial (state ft/gt, active flags)
  int2* items = nullptr;          // device: the item maps of all stages, one after another
  size_t item_off[kGsCount] = {};  // offset of each stage's map in `items`
  int item_count[kGsCount] = {};   // work items of each stage
  std::vector<char> has_eval;     // per field: loss and grad bound
  int zc_max = 1, Mq_max = 32, mt_max = 1;
  long rows = 0;                  // (patch, frame) rows of all fields
  int xcd_fwd = 0, xcd_adj = 1, grad_rt = 4, grad_splits = 0;
};

namespace {

GroupArgs group_args(const momfbd_group_s* g, const FieldDesc* fd, int stage) {
  GroupArgs a;
  a.fd = fd;
  a.item = g->items + g->item_off[stage];
  a.total = g->item_count[stage];
  return a;
}

int group_default_rt(int mt_max) { return mt_max <= 10 ? 4 : mt_max <= 13 ? 3 : 2; }

int group_splits(const momfbd_group_s* g) {
  if (g->grad_splits > 0) return g->grad_splits;
  // the automatic count of a plan with all the group's rows
  Dims d{g->N, (int)std::min<long>(g->rows, 1L << 30), 1, 1, 1, 1};
  d.grad_waves = 4;
  d.grad_rt = g->grad_rt == 4 ? 0 : g->grad_rt;
  d.zc = g->zc_max;
  return grad_splits_auto(d);
}

// One loss+gradient evaluation of every field (fd: evaluation or solver table).
hipError_t group_chain(const momfbd_group_s* g, const FieldDesc* fd, hipStream_t s) {
  hipError_t e = launch_phase_group(group_args(g, fd, kGsPhaseTiles), g->zc_max, g->Mq_max, s);
  if (e == hipSuccess) e = launch_forward_group(g->N, group_args(g, fd, kGsUnits), g->xcd_fwd, s);
  if (e == hipSuccess)
    e = launch_object_group(g->N, group_args(g, fd, kGsObjBlocks),
                            group_args(g, fd, kGsPatchBlocks), s);
  if (e == hipSuccess) e = launch_adjoint_group(g->N, group_args(g, fd, kGsUnits), g->xcd_adj, s);
  if (e == hipSuccess)
    e = launch_grad_group(group_args(g, fd, g->grad_rt == 3   ? kGsGradTiles3
                                            : g->grad_rt == 2 ? kGsGradTiles2
                                                              : kGsGradTiles4),
                          group_args(g, fd, kGsElemBlocks), g->mt_max, g->grad_rt,
                          group_splits(g), s);
  return e;
}

void group_free(momfbd_group_s* g) {
  if (g->fd_eval) (void)hipFree(g->fd_eval);
  if (g->fd_solve) (void)hipFree(g->fd_solve);
  if (g->items) (void)hipFree(g->items);
  delete g;
}

}  // namespace

extern "C" {

int momfbd_group_create(const momfbd_field* fields, int n, const momfbd_lbfgs_params* params,
                        momfbd_group* out) {
  if (!out || !fields || n < 1) return MOMFBD_EINVAL;
  if (params && !lbfgs_params_ok(params)) return MOMFBD_EINVAL;
  const int N = fields[0].plan ? fields[0].plan->d.N : 0;
  const int dev = fields[0].plan ? fields[0].plan->device : -1;
  std::vector<FieldDesc> ev(n), so(n);
  std::vector<int2> maps[kGsCount];
  std::vector<char> has_eval(n, 0);
  int zc_max = 1, Mq_max = 32, mt_max = 1;
  long rows = 0;
  for (int f = 0; f < n; ++f) {
    const momfbd_field& a = fields[f];
    const momfbd_plan pl = a.plan;
    if (!pl || !a.alpha || !a.D) return MOMFBD_EINVAL;
    if (pl->d.N != N || pl->device != dev) return MOMFBD_EINVAL;
    if (!a.ws || reinterpret_cast<uintptr_t>(a.ws) % 256 || a.ws_bytes < workspace_bytes(pl->d))
      return MOMFBD_EWORKSPACE;
    const Dims& d = pl->d;
    FieldDesc F;
    std::memset(&F, 0, sizeof(F));
    F.d = d;
    F.Mq = pl->Mq;
    F.ct = pl->ct;
    F.la = LossArgs{static_cast<const float2*>(a.D), a.gamma, a.gamma_scalar, a.weights, pl->supp};
    F.Ab = pl->Ab;
    F.Zs = pl->Zs;
    F.ZsT = pl->ZsT;
    F.thetat = pl->thetat;
    F.alpha = a.alpha;
    F.w = carve_workspace(d, a.ws);
    F.loss = a.loss;
    F.grad = a.grad;
    has_eval[f] = a.loss && a.grad;
    ev[f] = F;
    if (params) {
      const LbfgsLayout L = lbfgs_layout(d, params->m, params->max_evals);
      const int st = check_state(a.state, a.state_bytes, L.total);
      if (st) return st;
      char* b = static_cast<char*>(a.state);
      F.state = a.state;
      F.L = L;
      F.active = reinterpret_cast<const int*>(b + L.active);
      F.loss = reinterpret_cast<double*>(b + L.ft);
      F.grad = reinterpret_cast<float*>(b + L.gt);
      F.loss_accepted = a.loss_accepted;
      F.status = a.status;
      F.alpha_accepted = a.alpha_accepted;
    }
    so[f] = F;
    const long R = (long)d.P * d.J;
    const long items[kGsCount] = {(long)d.P * d.C * d.J,
                                  d.P,
                                  (R + kPhaseCols - 1) / kPhaseCols,
                                  (long)d.P * d.K * object_blocks(N, 1),
                                  (R + 255) / 256,
                                  (R + 191) / 192,
                                  (R + 127) / 128,
                                  (d.P + 255) / 256,
                                  (R * d.M + 255) / 256};
    for (int s = 0; s < kGsCount; ++s) {
      if ((long)maps[s].size() + items[s] > (1L << 28)) return MOMFBD_EUNSUPPORTED;
      for (long i = 0; i < items[s]; ++i) maps[s].push_back(make_int2(f, (int)i));
    }
    zc_max = std::max(zc_max, d.zc > 0 ? d.zc : d.C);
    Mq_max = std::max(Mq_max, pl->Mq);
    mt_max = std::max(mt_max, (d.M + 15) / 16);
    rows += R;
  }
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return MOMFBD_EDEVICE;
  if (cur != dev) return MOMFBD_EINVAL;
  if (int st = pending_error()) return st;
  momfbd_group_s* g = new (std::nothrow) momfbd_group_s();
  if (!g) return MOMFBD_EDEVICE;
  g->n = n;
  g->N = N;
  g->device = dev;
  g->solver = params != nullptr;
  if (params) g->params = *params;
  g->has_eval = has_eval;
  std::vector<int2> all;
  for (int st = 0; st < kGsCount; ++st) {
    g->item_off[st] = all.size();
    g->item_count[st] = (int)maps[st].size();
    all.insert(all.end(), maps[st].begin(), maps[st].end());
  }
  g->zc_max = zc_max;
  g->Mq_max = Mq_max;
  g->mt_max = mt_max;
  // default row tiles per wave: fewer for the widest mode counts, where
  // four tiles of 16 x mt_max accumulators would spill (176 modes and up)
  g->grad_rt = group_default_rt(mt_max);
  g->rows = rows;
  const bool ok =
      hipMalloc(&g->fd_eval, n * sizeof(FieldDesc)) == hipSuccess &&
      hipMalloc(&g->fd_solve, n * sizeof(FieldDesc)) == hipSuccess &&
      hipMalloc(&g->items, all.size() * sizeof(int2)) == hipSuccess &&
      hipMemcpy(g->fd_eval, ev.data(), n * sizeof(FieldDesc), hipMemcpyHostToDevice) ==
          hipSuccess &&
      hipMemcpy(g->fd_solve, so.data(), n * sizeof(FieldDesc), hipMemcpyHostToDevice) ==
          hipSuccess &&
      hipMemcpy(g->items, all.data(), all.size() * sizeof(int2), hipMemcpyHostToDevice) ==
          hipSuccess;
  if (!ok) {
    group_free(g);
    return MOMFBD_EDEVICE;
  }
  *out = g;
  return MOMFBD_OK;
}

int momfbd_group_destroy(momfbd_group g) {
  if (!g) return MOMFBD_OK;
  group_free(g);
  return MOMFBD_OK;
}

int momfbd_group_loss_grad(momfbd_group g, void* stream) {
  if (!g) return MOMFBD_EINVAL;
  for (int f = 0; f < g->n; ++f)
    if (!g->has_eval[f]) return MOMFBD_EINVAL;
  if (int st = pending_error()) return st;
  return to_status(group_chain(g, g->fd_eval, (hipStream_t)stream));
}

int momfbd_group_lbfgs_rounds(momfbd_group g, int rounds, void* stream) {
  if (!g || !g->solver || rounds < 0) return MOMFBD_EINVAL;
  if (int st = pending_error()) return st;
  hipStream_t s = (hipStream_t)stream;
  const FieldDesc* fd = g->fd_solve;
  hipError_t e = hipSuccess;
  for (int r = 0; e == hipSuccess && r < rounds; ++r) {
    e = launch_lbfgs_prep_group(group_args(g, fd, kGsPatches), s);
    if (e == hipSuccess) e = group_chain(g, fd, s);
    if (e == hipSuccess)
      e = launch_lbfgs_search_group(group_args(g, fd, kGsPatches), g->params.c1, g->params.c2,
                                    g->params.max_evals, g->params.ftol, s);
  }
  if (e == hipSuccess) e = launch_lbfgs_publish_group(group_args(g, fd, kGsElemBlocks), s);
  if (e == hipSuccess) e = launch_lbfgs_finish_group(group_args(g, fd, kGsPatchBlocks), s);
  return to_status(e);
}

int momfbd_group_set_tuning(momfbd_group g, const momfbd_tuning* t) {
  if (!g || !tuning_ok(t) || t->grad_waves != 4) return MOMFBD_EINVAL;
  g->xcd_fwd = t->xcd_forward;
  g->xcd_adj = t->xcd_adjoint;
  g->grad_rt = t->grad_row_tiles == 0 ? group_default_rt(g->mt_max)
                : t->grad_row_tiles == 3 || t->grad_row_tiles == 2 ? t->grad_row_tiles : 4;
  g->grad_splits = t->grad_splits;
  return MOMFBD_OK;
}

int momfbd_group_get_tuning(momfbd_group g, momfbd_tuning* t) {
  if (!g || !t) return MOMFBD_EINVAL;
  t->xcd_forward = g->xcd_fwd;
  t->xcd_adjoint = g->xcd_adj;
  t->object_pairs_per_thread = 1;
  t->grad_waves = 4;
  t->grad_splits = group_splits(g);
  t->grad_row_tiles = g->grad_rt;
  t->phase_col_tiles = kPhaseCols / 16;
  t->phase_waves = kPhaseWaves;
  t->object_fused = 0;
  return MOMFBD_OK;
}

int momfbd_group_autotune(momfbd_group g, int reps, void* stream, momfbd_tuning* chosen) {
  if (!g || reps < 1) return MOMFBD_EINVAL;
  for (int f = 0; f < g->n; ++f)
    if (!g->has_eval[f]) return MOMFBD_EINVAL;
  if (int st = pending_error()) return st;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreateWithFlags(&e0, hipEventReleaseToDevice) != hipSuccess ||
      hipEventCreateWithFlags(&e1, hipEventReleaseToDevice) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return MOMFBD_EDEVICE;
  }
  int st = MOMFBD_OK;
  auto timed = [&](float* ms) -> int {
    if (group_chain(g, g->fd_eval, s) != hipSuccess) return MOMFBD_EDEVICE;
    if (hipEventRecord(e0, s) != hipSuccess) return MOMFBD_EDEVICE;
    for (int i = 0; i < reps; ++i)
      if (group_chain(g, g->fd_eval, s) != hipSuccess) return MOMFBD_EDEVICE;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess)
      return MOMFBD_EDEVICE;
    return MOMFBD_OK;
  };
  // the plan tuner's method: one knob at a time, candidates interleaved over
  // three rounds, each keeping its fastest; the default first, replaced only
  // by a value at least 1% faster
  int* knobs[4] = {&g->xcd_adj, &g->xcd_fwd, &g->grad_rt, &g->grad_splits};
  const int rt0 = group_default_rt(g->mt_max);
  std::vector<int> values[4] = {{1, 0}, {0, 1}, {rt0}, {}};
  for (int v = 4; v >= 2; --v)
    if (v != rt0) values[2].push_back(v);
  for (int k = 0; k < 4 && st == MOMFBD_OK; ++k) {
    if (k == 3) {
      g->grad_splits = 0;
      const int a = group_splits(g);
      values[3] = {a};
      for (int v = 1; v <= kMaxGradSplits; v *= 2)
        if (v != a) values[3].push_back(v);
    }
    const int keep = *knobs[k];
    std::vector<float> fastest(values[k].size(), 0.f);
    for (int r = 0; r < 3 && st == MOMFBD_OK; ++r)
      for (size_t i = 0; i < values[k].size(); ++i) {
        *knobs[k] = values[k][i];
        float ms = 0.f;
        if ((st = timed(&ms))) break;
        if (r == 0 || ms < fastest[i]) fastest[i] = ms;
      }
    if (st) {
      *knobs[k] = keep;
      break;
    }
    size_t best = 0;
    for (size_t i = 1; i < values[k].size(); ++i)
      if (fastest[i] < 0.99f * fastest[best]) best = i;
    *knobs[k] = values[k][best];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  if (chosen) momfbd_group_get_tuning(g, chosen);
  return MOMFBD_OK;
}

}  // extern "C"
