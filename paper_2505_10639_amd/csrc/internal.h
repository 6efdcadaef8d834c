// Internal declarations shared by the C-ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace mfbd {

constexpr int kMaxC = 32;
constexpr int kMaxK = 32;
constexpr int kMaxM = 256;
constexpr int kBand = 32;            // band width for N = 64
constexpr int kBandPix = kBand * kBand;
constexpr int kPhaseCols = 64;       // (patch, frame) columns per group phase-contraction block
constexpr int kPhaseWaves = 8;       // and its waves

// Blocks of 256 threads, `ppt` frequency pairs per thread, covering one
// half spectrum of side n.
__host__ __device__ constexpr int object_blocks(int n, int ppt = 1) {
  return (n * (n / 2 + 1) / 2 + 256 * ppt - 1) / (256 * ppt);
}

struct Dims {
  int N, P, C, K, J, M;
  // launch schedules (chosen by momfbd_plan_autotune): XCD-grouped unit
  // order of the forward / adjoint grids, frequency pairs per thread of the
  // object kernel, waves per row tile of the gradient contraction and the
  // number of blocks its pixel sum is split over (0: grad_splits_auto) and
  // its row tiles per block (0: 4 with 4 waves; 3 is the other 4-wave choice;
  // 8 waves always take 2)
  int xcd_fwd = 0, xcd_adj = 1, obj_ppt = 1, grad_waves = 4, grad_splits = 0, grad_rt = 0;
  // the phase contraction's block: 16-column tiles and waves per workgroup
  // (0, 0: the widest block whose staged coefficients fit; phase_shape_of)
  int phase_ct = 0, phase_waves = 0;
  // the object pass in the forward launch (k_fwdobj64) where it applies
  // (fuse_ok, set at plan creation: 64x64 patches, at most 12 units per
  // (patch, object)); fuse_obj is the schedule, 0 by default: measured
  // slower than the two launches at the 64x64 full-field workload
  int fuse_obj = 0;
  bool fuse_ok = false;
  // distinct modal bases on the band: 1 when every channel's band-sampled
  // basis is the same (the contractions then run once for all channels),
  // else C; 0 is read as C
  int zc = 0;
  __host__ __device__ int band() const { return N / 2; }                 // pupil band width
  __host__ __device__ int bandpix() const { return (N / 2) * (N / 2); }  // pixels of the band
  __host__ __device__ int half() const { return N * (N / 2 + 1); }  // complex values of a half spectrum
};

// Loads of data a kernel reads once per launch (the object kernel's data
// and OTF spectra): nontemporal, so that they do not displace cached lines.
// (In the adjoint kernels the same hint made the step slower.)
typedef float mfbd_fx4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 stream_load(const float4* p) {
  const mfbd_fx4 v = __builtin_nontemporal_load(reinterpret_cast<const mfbd_fx4*>(p));
  return make_float4(v[0], v[1], v[2], v[3]);
}

// Channel tables passed by value to kernels.
struct ChanTab {
  int chan_obj[kMaxC];     // object of each channel
  float kappa[kMaxC];      // 1 / (N^2 sum A^2) per channel
  int obj_first[kMaxK + 1];// channels of object k: obj_chans[obj_first[k] .. obj_first[k+1])
  int obj_chans[kMaxC];
};

// Loss/gradient inputs common to several kernels.
struct LossArgs {
  const float2* D;         // [P][C][J][N][N/2+1]
  const float* gamma;      // [K][N][N/2+1] or null
  float gamma_scalar;
  const float* weights;    // [C][J] or null (= 1)
  const int* supp;         // [K][N/2+1] spectral support of each object (plan table)
};

// conj(O) (D - O S) at one frequency, the residual D - O S formed with two
// FMAs per component (the 96x96 and 128x128 adjoint kernels' input; the
// factor -2 w of the frame is applied after the inverse transform, which is
// linear).  The 64x64 adjoint keeps the product form: its FMA form, at 9
// more registers, ran 1% slower.
__device__ __forceinline__ float2 adjoint_input(float2 d, float2 s, float2 o) {
  const float rx = fmaf(o.y, s.y, fmaf(-o.x, s.x, d.x));
  const float ry = fmaf(-o.y, s.x, fmaf(-o.x, s.y, d.y));
  return make_float2(o.x * rx + o.y * ry, o.x * ry - o.y * rx);
}

// Spectral support of an object.  A channel's OTF is the autocorrelation of
// its pupil, so it vanishes outside the pupil's difference set; supp[k][kx]
// is the largest |ky| (ky taken in (-N/2, N/2]) at which any channel of
// object k can have a nonzero OTF in column kx of the half spectrum (-1:
// none).  Outside it the Wiener object is zero, the residual is D and G =
// -2 w conj(O) R vanishes, so the object kernel needs no S and the adjoint
// no D, S or O there.
__device__ __forceinline__ bool in_support(int ky, int n, int fmax) {
  return (ky <= n / 2 ? ky : n - ky) <= fmax;
}

// Raw buffer view of `bytes` bytes at `base` (gfx9 descriptor, 32-bit
// elements): a load at an offset at or beyond `bytes` returns zero without
// a memory access, which skips the spectrum outside the support without a
// branch.
// The resource lives in scalar registers.  Every caller passes one base per
// wave, so the base is read from the first active lane: a pointer the
// compiler holds in vector registers (read from a field descriptor in a
// group kernel) then costs two readfirstlane, not a loop over the distinct
// lanes around every load.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_buffer(const void* base, int bytes) {
  const unsigned long long a = reinterpret_cast<unsigned long long>(base);
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a >> 32));
  void* const p = reinterpret_cast<void*>((static_cast<unsigned long long>(hi) << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(p, 0, __builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}
typedef unsigned int mfbd_u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int mfbd_u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float2 buffer_load_f2(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
// 16 bytes with the nontemporal hint (data read once per launch)
__device__ __forceinline__ float4 buffer_load_f4_stream(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 2));
}

// FP64 sums of one frequency pair of a (patch, object) plane over its
// units: N = sum w D conj(S), Q = gamma + sum w |S|^2, E = sum w |D|^2.
// Products of FP32 inputs are exact in FP64.  The object kernel and the
// fused forward/object kernel both use these two functions, in the same
// unit order, so that their results agree bit for bit.
struct Acc2 {
  double nr[2], ni[2], q[2], e[2];
};
__device__ __forceinline__ void acc_unit(Acc2& a, double w, float4 d, float4 s) {
  const double dx0 = d.x, dy0 = d.y, sx0 = s.x, sy0 = s.y;
  const double dx1 = d.z, dy1 = d.w, sx1 = s.z, sy1 = s.w;
  a.nr[0] += w * (dx0 * sx0 + dy0 * sy0);
  a.ni[0] += w * (dy0 * sx0 - dx0 * sy0);
  a.q[0] += w * (sx0 * sx0 + sy0 * sy0);
  a.e[0] += w * (dx0 * dx0 + dy0 * dy0);
  a.nr[1] += w * (dx1 * sx1 + dy1 * sy1);
  a.ni[1] += w * (dy1 * sx1 - dx1 * sy1);
  a.q[1] += w * (sx1 * sx1 + sy1 * sy1);
  a.e[1] += w * (dx1 * dx1 + dy1 * dy1);
}
// The Wiener object O = N / Q of the pair (f, f + 1) and its loss term
// E - |N|^2 / Q, columns 1..N/2-1 of the half spectrum counting twice.
__device__ __forceinline__ float4 wiener_pair(const Acc2& a, int f, int hc, double& loss) {
  const double inv0 = 1.0 / a.q[0], inv1 = 1.0 / a.q[1];
  const int kx0 = f % hc, kx1 = (f + 1) % hc;
  const double h0 = (kx0 == 0 || kx0 == hc - 1) ? 1.0 : 2.0;
  const double h1 = (kx1 == 0 || kx1 == hc - 1) ? 1.0 : 2.0;
  loss += h0 * (a.e[0] - (a.nr[0] * a.nr[0] + a.ni[0] * a.ni[0]) * inv0) +
          h1 * (a.e[1] - (a.nr[1] * a.nr[1] + a.ni[1] * a.ni[1]) * inv1);
  return make_float4((float)(a.nr[0] * inv0), (float)(a.ni[0] * inv0), (float)(a.nr[1] * inv1),
                     (float)(a.ni[1] * inv1));
}

// Frequency pair f2 (frequencies f = 2 f2 and f + 1 of the half spectrum)
// of the (patch p, object k) plane: N, Q and E over the object's units in
// order (its channels in order, each channel's frames in order), reading D
// and, within the object's spectral support, S; writes the pair of O and
// returns its loss term.  Outside the support every S of the pair is zero
// and is not read (N = 0, Q = gamma, O = 0, loss term E).
template <int NN>
__device__ __forceinline__ double object_pair(int f2, int p, int k, int C, int J, int K,
                                              const ChanTab& ct, const LossArgs& la,
                                              const float2* __restrict__ S,
                                              float2* __restrict__ O) {
  constexpr int HC = NN / 2 + 1;
  constexpr int kUnitF2 = NN * HC;
  const int f = 2 * f2;
  Acc2 a;
  for (int i = 0; i < 2; ++i) {
    a.nr[i] = a.ni[i] = a.e[i] = 0.0;
    a.q[i] = la.gamma ? (double)la.gamma[(size_t)k * kUnitF2 + f + i] : (double)la.gamma_scalar;
  }
  const bool sup = in_support(f / HC, NN, la.supp[k * HC + f % HC]) ||
                   in_support((f + 1) / HC, NN, la.supp[k * HC + (f + 1) % HC]);
  const int c0 = ct.obj_first[k], c1 = ct.obj_first[k + 1];
  for (int ci = c0; ci < c1; ++ci) {
    const int c = ct.obj_chans[ci];
    const float4* Dc =
        reinterpret_cast<const float4*>(la.D + ((size_t)(p * C + c) * J) * kUnitF2 + f);
    const int s_bytes = J * kUnitF2 * 8;
    const __amdgpu_buffer_rsrc_t rS =
        raw_buffer(S + ((size_t)(p * C + c) * J) * kUnitF2, s_bytes);
    const int s_off = sup ? f * 8 : s_bytes;
    constexpr int kStep = kUnitF2 * 8;   // bytes between frames
    const float* wc = la.weights ? la.weights + c * J : nullptr;
    int j = 0;
    for (; j + 6 <= J; j += 6) {
      float4 d[6], s[6];
#pragma unroll
      for (int u = 0; u < 6; ++u) {
        d[u] = stream_load(Dc + (size_t)(j + u) * (kUnitF2 / 2));
        s[u] = buffer_load_f4_stream(rS, sup ? s_off + (j + u) * kStep : s_bytes);
      }
#pragma unroll
      for (int u = 0; u < 6; ++u) acc_unit(a, wc ? (double)wc[j + u] : 1.0, d[u], s[u]);
    }
    for (; j < J; ++j)
      acc_unit(a, wc ? (double)wc[j] : 1.0, stream_load(Dc + (size_t)j * (kUnitF2 / 2)),
               buffer_load_f4_stream(rS, sup ? s_off + j * kStep : s_bytes));
  }
  double loss = 0.0;
  const float4 o = wiener_pair(a, f, HC, loss);
  reinterpret_cast<float4*>(O + ((size_t)p * K + k) * kUnitF2)[f2] = o;
  return loss;
}

// Smoothness prior constants per object.
struct PriorTab {
  float gamma0[kMaxK];
  float lambda[kMaxK];
};
hipError_t launch_smoothness(int N, int K, const PriorTab& t, float* gamma, hipStream_t s);

// Fourier filter of one object's restored spectrum.
constexpr int kFilterNone = 0, kFilterTophat = 1, kFilterScharmer = 2;
struct FilterSpec {
  int kind;
  float f_lo, f_hi, diff_limit;   // top-hat (units of the diffraction limit; bins)
  float noise_power;              // Loefdahl-Scharmer
};
struct FilterTab {
  FilterSpec f[kMaxK];
};
hipError_t launch_filter(const Dims& d, const ChanTab& ct, const FilterTab& ft, const float2* D,
                         const float* weights, const float2* S, float2* O, float* H,
                         hipStream_t s);
hipError_t launch_mosaic(const Dims& d, const float* obj, int ny, int nx, int stride, int border,
                         float* out, hipStream_t s);

// Workspace carve-up.
struct Workspace {
  float* phi;              // [P][C][J][N/2][N/2]  phase in turns on the pupil band
  float2* S;               // [P][C][J][N][N/2+1] OTF half spectra
  float2* O;               // [P][K][N][N/2+1]    object spectra
  float* gphi;             // [P][C][J][N/2][N/2]  dL/dphi (rad^-1) on the band
  double* loss_pk;         // [P][K][object_blocks(N)] partial loss terms
  float* gpart;            // [kMaxGradSplits][P][J][M] partial sums of the gradient
};

struct LbfgsLayout {
  int m;              // history pairs
  int n;              // variables per patch (J*M)
  size_t hdr, rho, x0, g, d, gt, S, Y, ft, active, counter, total;   // byte offsets
};

// A group: fields of one patch size whose loss/gradient chain and solver
// rounds run together, one launch per stage for all of them.  Each field
// keeps its own plan tables, data, workspace and solver state; FieldDesc
// holds every per-field argument of the kernels in device memory.  Per
// stage the group keeps an item map: work item g of a launch (a block, or
// a unit) is item map[g].y of field map[g].x, one load away.
struct FieldDesc {
  Dims d;
  int Mq;                  // modes rounded up to 32 (k extent of the phase contraction)
  ChanTab ct;
  LossArgs la;
  const float* Ab;
  const uint4* Zs;         // split basis tables (bf16split.h, contract_mfma.h)
  const uint4* ZsT;
  const float* thetat;
  float* alpha;            // [P][J][M] coefficients (solver trial point)
  Workspace w;
  const int* active;       // [P] patches inside a line search (solver), or null
  double* loss;            // [P] loss output of the evaluation
  float* grad;             // [P][J][M] gradient output of the evaluation
  void* state;             // solver state, or null
  LbfgsLayout L;
  double* loss_accepted;   // [P] or null
  int* status;             // [P] or null
  float* alpha_accepted;   // [P][J][M] or null
};
// work items per field: units P C J; patches P; phase tiles of 32 (patch,
// frame) rows; object blocks P K object_blocks(N); gradient blocks of 256,
// 192 or 128 rows (4 waves of 4, 3 or 2 row tiles); blocks of 256 patches;
// blocks of 256 coefficients (P J M)
enum GroupStage { kGsUnits, kGsPatches, kGsPhaseTiles, kGsObjBlocks, kGsGradTiles4,
                  kGsGradTiles3, kGsGradTiles2, kGsPatchBlocks, kGsElemBlocks, kGsCount };
struct GroupArgs {
  const FieldDesc* fd;     // [fields] (device)
  const int2* item;        // [total] (field, item of that field) per work item (device)
  int total;
};

// The gradient contraction's pixel sum may be split over up to this many
// blocks per row tile; grad_splits_of gives the plan's split count.
constexpr int kMaxGradSplits = 8;
int grad_splits_auto(const Dims& d);
int grad_splits_of(const Dims& d);
int grad_row_tiles_of(const Dims& d);
// The phase contraction's block in use (column tiles, waves), and whether a
// selectable one (8 x 8, 4 x 8 or 8 x 16) fits the LDS for Mq staged modes.
void phase_shape_of(const Dims& d, int Mq, int* ct, int* waves);
bool phase_shape_fits(int ct, int waves, int Mq);

size_t workspace_bytes(const Dims& d);
Workspace carve_workspace(const Dims& d, void* base);

// Launchers (return hipSuccess or the launch error); dispatch on d.N.
// ZsT: [C][(N/2)^2][Mq/8][3] and Zs: [C][Mp][(N/2)^2/8][3], the band bases in
// turns split into three bf16 parts (eight values per uint4; contract_mfma.h).
hipError_t launch_phase(const Dims& d, const float* alpha, const uint4* ZsT, int Mq,
                        const float* thetat, float* phi, hipStream_t s);
// `active` (nullable, [P]) restricts the unit kernels to patches with a
// nonzero entry; the others are neither computed nor written.
hipError_t launch_forward(const Dims& d, const ChanTab& ct, const int* active, const float* Ab,
                          const float* phi, float* psf, float2* S, hipStream_t s);
// The per-patch loss: the object kernel's FP64 block partials summed per
// patch in block order.  launch_object sums them itself unless asked to
// leave them (sum_loss false) to launch_grad, which then folds the sum into
// its combine launch (or launches it after the contraction).
struct LossSum {
  int P, nper;               // patches, partials per patch
  const int* active;         // nullable patch mask
  const double* loss_part;   // [P][nper]
  double* loss;              // [P]
};
__device__ __forceinline__ void loss_sum_patch(int p, int nper, const int* __restrict__ active,
                                               const double* __restrict__ loss_part,
                                               double* __restrict__ loss) {
  if (active && !active[p]) return;
  double s = 0.0;
  // in order; unrolled so that eight loads are in flight before the adds
#pragma unroll 8
  for (int i = 0; i < nper; ++i) s += loss_part[(size_t)p * nper + i];
  loss[p] = s;
}
LossSum loss_sum_of(const Dims& d, const int* active, const double* loss_pk, double* loss);
hipError_t launch_loss_sum(const LossSum& ls, hipStream_t s);
hipError_t launch_object(const Dims& d, const ChanTab& ct, const LossArgs& la, const int* active,
                         const float2* S, float2* O, double* loss_pk, double* loss,
                         hipStream_t s, bool sum_loss = true);
// Forward and object pass in one launch (64x64 patches, one workgroup per
// (patch, object)): S, O and the loss partials equal those of launch_forward
// followed by launch_object with one pair per thread, bit for bit.
constexpr int kFusedWaves = 12;   // units per (patch, object) it takes at most
inline bool fused_object(const Dims& d) { return d.fuse_ok && d.fuse_obj; }
hipError_t launch_fwdobj64(const Dims& d, const ChanTab& ct, const LossArgs& la,
                           const int* active, const float* Ab, const float* phi, float2* S,
                           float2* O, double* loss_pk, hipStream_t s);
hipError_t launch_adjoint(const Dims& d, const ChanTab& ct, const LossArgs& la, const int* active,
                          const float* Ab, const float* phi, const float2* S, const float2* O,
                          float* gphi, hipStream_t s);
hipError_t launch_grad(const Dims& d, const uint4* Zs, const float* gphi, float* grad,
                       float* gpart, hipStream_t s, const LossSum* ls = nullptr);
hipError_t launch_prepare(const Dims& d, const float* frames, int H, int W, int stride,
                          const float* apod, float2* D, hipStream_t s);
hipError_t launch_objimg(const Dims& d, const float2* O, float* obj, hipStream_t s);
// frames IDFT(D)/N^2 of `items` half spectra: item it is spectrum
// (it / per) * stride + it % per of D (channel 0 of bursts [B][C][J]: per = J,
// stride = C J)
hipError_t launch_frames(int N, int items, int per, int stride, const float2* D, float* out,
                         hipStream_t s);
hipError_t launch_synth(const Dims& d, const ChanTab& ct, const float2* O, const float2* S,
                        const float* noise, const float* sigma, float* field, hipStream_t s);
hipError_t launch_frames64(int items, int per, int stride, const float2* D, float* out,
                           hipStream_t s);
hipError_t launch_frames96(int items, int per, int stride, const float2* D, float* out,
                           hipStream_t s);
hipError_t launch_frames128(int items, int per, int stride, const float2* D, float* out,
                            hipStream_t s);
hipError_t launch_synth96(const Dims& d, const ChanTab& ct, const float2* O, const float2* S,
                          const float* noise, const float* sigma, float* field, hipStream_t s);
hipError_t launch_synth128(const Dims& d, const ChanTab& ct, const float2* O, const float2* S,
                           const float* noise, const float* sigma, float* field, hipStream_t s);

// per-size implementations
hipError_t launch_forward64(const Dims& d, const ChanTab& ct, const int* active, const float* Ab,
                            const float* phi, float* psf, float2* S, hipStream_t s);
hipError_t launch_adjoint64(const Dims& d, const ChanTab& ct, const LossArgs& la,
                            const int* active, const float* Ab, const float* phi, const float2* S,
                            const float2* O, float* gphi, hipStream_t s);
hipError_t launch_prepare64(const Dims& d, const float* frames, int H, int W, int stride,
                            const float* apod, float2* D, hipStream_t s);
hipError_t launch_objimg64(const Dims& d, const float2* O, float* obj, hipStream_t s);
hipError_t launch_synth64(const Dims& d, const ChanTab& ct, const float2* O, const float2* S,
                          const float* noise, const float* sigma, float* field, hipStream_t s);
hipError_t launch_forward96(const Dims& d, const ChanTab& ct, const int* active, const float* Ab,
                            const float* phi, float* psf, float2* S, hipStream_t s);
hipError_t launch_adjoint96(const Dims& d, const ChanTab& ct, const LossArgs& la,
                            const int* active, const float* Ab, const float* phi, const float2* S,
                            const float2* O, float* gphi, hipStream_t s);
hipError_t launch_prepare96(const Dims& d, const float* frames, int H, int W, int stride,
                            const float* apod, float2* D, hipStream_t s);
hipError_t launch_objimg96(const Dims& d, const float2* O, float* obj, hipStream_t s);
hipError_t launch_forward128(const Dims& d, const ChanTab& ct, const int* active, const float* Ab,
                             const float* phi, float* psf, float2* S, hipStream_t s);
hipError_t launch_adjoint128(const Dims& d, const ChanTab& ct, const LossArgs& la,
                             const int* active, const float* Ab, const float* phi, const float2* S,
                             const float2* O, float* gphi, hipStream_t s);
hipError_t launch_prepare128(const Dims& d, const float* frames, int H, int W, int stride,
                             const float* apod, float2* D, hipStream_t s);
hipError_t launch_objimg128(const Dims& d, const float2* O, float* obj, hipStream_t s);

// L-BFGS (per-patch solver state lives in a caller-provided buffer)
LbfgsLayout lbfgs_layout(const Dims& d, int m, int max_evals);
hipError_t launch_lbfgs_init(const Dims& d, const LbfgsLayout& L, void* state, double* loss_out,
                             hipStream_t s);
hipError_t launch_lbfgs_begin(const Dims& d, const LbfgsLayout& L, void* state, float* alpha,
                              int max_evals, hipStream_t s);
hipError_t launch_lbfgs_prep(const Dims& d, const LbfgsLayout& L, void* state, float* alpha,
                             hipStream_t s);
hipError_t launch_lbfgs_publish(const Dims& d, const LbfgsLayout& L, void* state,
                                const float* alpha, float* out, hipStream_t s);
hipError_t launch_lbfgs_search(const Dims& d, const LbfgsLayout& L, void* state, float* alpha,
                               int eval, double c1, double c2, int max_evals, double ftol,
                               hipStream_t s);
hipError_t launch_lbfgs_finish(const Dims& d, const LbfgsLayout& L, void* state, double* loss_out,
                               int* status_out, hipStream_t s);

// Group launches: one launch per stage over every field of a group (all of
// one patch size).  `ga` carries the stage's prefix sums; the schedules
// (XCD order, gradient row tiles and splits) are the group's.
hipError_t launch_phase_group(const GroupArgs& ga, int zc_max, int Mq_max, hipStream_t s);
hipError_t launch_forward_group(int N, const GroupArgs& ga, int xcd, hipStream_t s);
hipError_t launch_object_group(int N, const GroupArgs& ga_blocks, const GroupArgs& ga_patches,
                               hipStream_t s);
hipError_t launch_adjoint_group(int N, const GroupArgs& ga, int xcd, hipStream_t s);
hipError_t launch_grad_group(const GroupArgs& ga_tiles, const GroupArgs& ga_elems, int mt_max,
                             int row_tiles, int splits, hipStream_t s);
hipError_t launch_forward64_group(const GroupArgs& ga, int xcd, hipStream_t s);
hipError_t launch_adjoint64_group(const GroupArgs& ga, int xcd, hipStream_t s);
hipError_t launch_forward96_group(const GroupArgs& ga, int xcd, hipStream_t s);
hipError_t launch_adjoint96_group(const GroupArgs& ga, int xcd, hipStream_t s);
hipError_t launch_forward128_group(const GroupArgs& ga, int xcd, hipStream_t s);
hipError_t launch_adjoint128_group(const GroupArgs& ga, int xcd, hipStream_t s);
hipError_t launch_lbfgs_prep_group(const GroupArgs& ga, hipStream_t s);
hipError_t launch_lbfgs_search_group(const GroupArgs& ga, double c1, double c2, int max_evals,
                                     double ftol, hipStream_t s);
hipError_t launch_lbfgs_publish_group(const GroupArgs& ga_elems, hipStream_t s);
hipError_t launch_lbfgs_finish_group(const GroupArgs& ga_patches, hipStream_t s);

}  // namespace mfbd
