// Batched per-patch L-BFGS with a strong-Wolfe line search (gfx950).
//
// The patches are independent (no coefficient is shared between patches), so
// every patch runs its own quasi-Newton iteration: the two-loop recursion of
// limited-memory BFGS for the direction, then a bracketing/zoom line search
// enforcing the strong Wolfe conditions (Nocedal & Wright, Numerical
// Optimization, Algorithms 7.4, 3.5 and 3.6).  Trial steps inside the zoom are
// the minimiser of the cubic through the bracket ends, clamped to its central
// 80% (bisection when the cubic has no real minimiser).  The first trial step
// is min(1, 1/||g||_inf) when the history is empty and 1 otherwise.
//
// One block of 256 threads per patch; dot products are accumulated in FP64
// in a fixed order; every scalar of the line search is FP64.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace mfbd {

namespace {

struct Hdr {
  double f, f0, dphi0, t, t_prev, f_prev, g_prev, lo, flo, glo, hi, fhi, ghi;
  int phase, n_eval, count, head, iter, status, first, pad;
};

struct View {
  Hdr* hdr;
  double* rho;
  float *x0, *g, *d, *gt, *S, *Y;
  double* ft;
  int* active;
  int* counter;
};

__device__ __forceinline__ View view(const LbfgsLayout& L, void* state) {
  char* b = static_cast<char*>(state);
  View v;
  v.hdr = reinterpret_cast<Hdr*>(b + L.hdr);
  v.rho = reinterpret_cast<double*>(b + L.rho);
  v.x0 = reinterpret_cast<float*>(b + L.x0);
  v.g = reinterpret_cast<float*>(b + L.g);
  v.d = reinterpret_cast<float*>(b + L.d);
  v.gt = reinterpret_cast<float*>(b + L.gt);
  v.S = reinterpret_cast<float*>(b + L.S);
  v.Y = reinterpret_cast<float*>(b + L.Y);
  v.ft = reinterpret_cast<double*>(b + L.ft);
  v.active = reinterpret_cast<int*>(b + L.active);
  v.counter = reinterpret_cast<int*>(b + L.counter);
  return v;
}

constexpr int kThreads = 256;

// Sum over the block in a fixed order: a butterfly of shuffles inside each
// wave (every lane ends with the same bits, as each stage adds the same two
// values in either order), then the wave sums in wave order.  Every thread
// receives the result.
constexpr int kWaves = kThreads / 64;
__device__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < kWaves; ++w) r += red[w];
  __syncthreads();
  return r;
}

__device__ double block_max(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < kWaves; ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

__device__ double dot(const float* a, const float* b, int n, double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) s += (double)a[i] * (double)b[i];
  return block_sum(s, red);
}

__device__ double cubic_min(double a, double fa, double ga, double b, double fb, double gb) {
  const double lo = fmin(a, b), hi = fmax(a, b), w = hi - lo;
  const double d1 = ga + gb - 3.0 * (fa - fb) / (a - b);
  const double disc = d1 * d1 - ga * gb;
  if (disc >= 0.0 && w > 0.0) {
    const double d2 = copysign(sqrt(disc), b - a);
    const double den = gb - ga + 2.0 * d2;
    if (den != 0.0) {
      const double t = b - (b - a) * (gb + d2 - d1) / den;
      if (isfinite(t)) return fmin(fmax(t, lo + 0.1 * w), hi - 0.1 * w);
    }
  }
  return 0.5 * (lo + hi);
}

__global__ __launch_bounds__(kThreads) void k_lbfgs_init(int P, LbfgsLayout L, void* state,
                                                         double* loss_out) {
  View v = view(L, state);
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= P) return;
  Hdr& h = v.hdr[p];
  h.f = v.ft[p];
  h.count = 0;
  h.head = 0;
  h.iter = 0;
  h.status = 0;
  h.phase = 0;
  h.n_eval = 0;
  v.active[p] = 0;
  if (loss_out) loss_out[p] = h.f;
}

// Two-loop recursion with the direction q held in registers (E elements per
// thread, n <= 256 E) and each history pair loaded one step ahead, so that
// the chain of dependent block sums does not also wait on memory.  Same
// arithmetic and summation order as the in-memory loop in begin_patch.
// Leaves -H g in q_out.
template <int E>
__device__ void two_loop_regs(int n, int m, int count, int head, const float* __restrict__ g,
                              float* __restrict__ q_out, const float* __restrict__ S,
                              const float* __restrict__ Y, const double* __restrict__ rho,
                              double* red, double* coef) {
  const int tid = threadIdx.x;
  float q[E], s[E], y[E], sn[E], yn[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = tid + e * kThreads;
    q[e] = i < n ? g[i] : 0.f;
  }
  auto load = [&](int k, float (&sv)[E], float (&yv)[E]) {
    const size_t slot = (size_t)((head + k) % m);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = tid + e * kThreads;
      sv[e] = i < n ? S[slot * n + i] : 0.f;
      yv[e] = i < n ? Y[slot * n + i] : 0.f;
    }
  };
  auto slot_of = [&](int k) { return (head + k) % m; };
  // newest pair first
  if (count > 0) load(count - 1, s, y);
  for (int k = count - 1; k >= 0; --k) {
    if (k > 0) load(k - 1, sn, yn);
    double part = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) part += (double)s[e] * (double)q[e];
    const double ak = rho[slot_of(k)] * block_sum(part, red);
    if (tid == 0) coef[k] = ak;
#pragma unroll
    for (int e = 0; e < E; ++e) q[e] = (float)((double)q[e] - ak * (double)y[e]);
    if (k > 0) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        s[e] = sn[e];
        y[e] = yn[e];
      }
    }
  }
  if (count > 0) {
    load(count - 1, s, y);
    double psy = 0.0, pyy = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      psy += (double)s[e] * (double)y[e];
      pyy += (double)y[e] * (double)y[e];
    }
    const double sy = block_sum(psy, red);
    const double gam = sy / block_sum(pyy, red);
#pragma unroll
    for (int e = 0; e < E; ++e) q[e] = (float)((double)q[e] * gam);
    load(0, s, y);
  }
  __syncthreads();   // coef[] written by thread 0 above
  for (int k = 0; k < count; ++k) {
    if (k + 1 < count) load(k + 1, sn, yn);
    double part = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) part += (double)y[e] * (double)q[e];
    const double beta = rho[slot_of(k)] * block_sum(part, red);
    const double ak = coef[k];
#pragma unroll
    for (int e = 0; e < E; ++e) q[e] = (float)((double)q[e] + (ak - beta) * (double)s[e]);
    if (k + 1 < count) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        s[e] = sn[e];
        y[e] = yn[e];
      }
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = tid + e * kThreads;
    if (i < n) q_out[i] = -q[e];
  }
  __syncthreads();
}

// Start the next iteration of patch p (status 0): two-loop direction, first
// trial step, x0 = alpha, alpha = x0 + t0 d, active = 1.
__device__ void begin_patch(const LbfgsLayout& L, View& v, int p, float* __restrict__ alpha,
                            double* red, double* coef) {
  const int n = L.n, m = L.m, tid = threadIdx.x;
  Hdr& h = v.hdr[p];
  const float* g = v.g + (size_t)p * n;
  float* q = v.d + (size_t)p * n;
  float* x0 = v.x0 + (size_t)p * n;
  float* a = alpha + (size_t)p * n;
  const size_t hb = (size_t)p * m;
  const int count = h.count, head = h.head;
  if (n <= kThreads * 8) {
    two_loop_regs<8>(n, m, count, head, g, q, v.S + hb * n, v.Y + hb * n, v.rho + hb, red, coef);
  } else {
    for (int i = tid; i < n; i += kThreads) q[i] = g[i];
    __syncthreads();
    // two-loop recursion, newest pair first
    for (int k = count - 1; k >= 0; --k) {
      const int slot = (head + k) % m;
      const float* s = v.S + (hb + slot) * n;
      const float* y = v.Y + (hb + slot) * n;
      const double ak = v.rho[hb + slot] * dot(s, q, n, red);
      if (tid == 0) coef[k] = ak;
      for (int i = tid; i < n; i += kThreads) q[i] = (float)((double)q[i] - ak * (double)y[i]);
      __syncthreads();
    }
    if (count > 0) {
      const int last = (head + count - 1) % m;
      const float* s = v.S + (hb + last) * n;
      const float* y = v.Y + (hb + last) * n;
      const double gam = dot(s, y, n, red) / dot(y, y, n, red);
      for (int i = tid; i < n; i += kThreads) q[i] = (float)((double)q[i] * gam);
      __syncthreads();
    }
    for (int k = 0; k < count; ++k) {
      const int slot = (head + k) % m;
      const float* s = v.S + (hb + slot) * n;
      const float* y = v.Y + (hb + slot) * n;
      const double beta = v.rho[hb + slot] * dot(y, q, n, red);
      const double ak = coef[k];
      for (int i = tid; i < n; i += kThreads)
        q[i] = (float)((double)q[i] + (ak - beta) * (double)s[i]);
      __syncthreads();
    }
    for (int i = tid; i < n; i += kThreads) q[i] = -q[i];
    __syncthreads();
  }
  double dphi0 = dot(g, q, n, red);
  bool reset = !(dphi0 < 0.0);
  if (reset) {          // not a descent direction: restart from steepest descent
    for (int i = tid; i < n; i += kThreads) q[i] = -g[i];
    __syncthreads();
    dphi0 = -dot(g, g, n, red);
  }
  double gl = 0.0;
  for (int i = tid; i < n; i += kThreads) gl = fmax(gl, fabs((double)g[i]));
  const double gmax = block_max(gl, red);
  if (gmax == 0.0) {
    if (tid == 0) {
      h.status = 1;
      v.active[p] = 0;
    }
    return;
  }
  const int cnt = reset ? 0 : count;
  const double t0 = (cnt == 0) ? fmin(1.0, 1.0 / gmax) : 1.0;
  for (int i = tid; i < n; i += kThreads) {
    x0[i] = a[i];
    a[i] = (float)((double)a[i] + t0 * (double)q[i]);
  }
  if (tid == 0) {
    if (reset) {
      h.count = 0;
      h.head = 0;
    }
    h.f0 = h.f;
    h.dphi0 = dphi0;
    h.t = t0;
    h.t_prev = 0.0;
    h.f_prev = h.f;
    h.g_prev = dphi0;
    h.phase = 0;
    h.first = 1;
    h.n_eval = 0;
    v.active[p] = 1;
  }
}

__global__ __launch_bounds__(kThreads) void k_lbfgs_begin(LbfgsLayout L, void* state,
                                                          float* __restrict__ alpha,
                                                          int max_evals) {
  __shared__ double red[kThreads];
  __shared__ double coef[32];
  View v = view(L, state);
  const int p = blockIdx.x, tid = threadIdx.x;
  if (p == 0)
    for (int i = tid; i <= max_evals; i += kThreads) v.counter[i] = 0;
  if (v.hdr[p].status != 0) {
    if (tid == 0) v.active[p] = 0;
    return;
  }
  if (v.active[p]) {
    // left inside a line search by round mode: restart from the accepted point
    const int n = L.n;
    for (int i = tid; i < n; i += kThreads)
      alpha[(size_t)p * n + i] = v.x0[(size_t)p * n + i];
    __syncthreads();
  }
  begin_patch(L, v, p, alpha, red, coef);
}

// Round mode: a patch that is still running and not inside a line search
// starts its next iteration; a patch inside a search keeps its trial point.
__device__ __forceinline__ void prep_patch(int p, const LbfgsLayout& L, void* state,
                                           float* __restrict__ alpha) {
  __shared__ double red[kThreads];
  __shared__ double coef[32];
  View v = view(L, state);
  const int tid = threadIdx.x;
  if (v.hdr[p].status != 0) {
    if (tid == 0) v.active[p] = 0;
    return;
  }
  if (v.active[p]) return;
  begin_patch(L, v, p, alpha, red, coef);
}

__global__ __launch_bounds__(kThreads) void k_lbfgs_prep(LbfgsLayout L, void* state,
                                                         float* __restrict__ alpha) {
  prep_patch(blockIdx.x, L, state, alpha);
}

// Every patch of every field of a group.
__global__ __launch_bounds__(kThreads) void k_lbfgs_prep_group(GroupArgs ga) {
  const int2 it = ga.item[blockIdx.x];
  const FieldDesc& F = ga.fd[it.x];
  prep_patch(it.y, F.L, F.state, F.alpha);
}

__device__ __forceinline__ void search_patch(int p, const LbfgsLayout& L, void* state,
                                             float* __restrict__ alpha, int eval, double c1,
                                             double c2, int max_evals, double ftol) {
  __shared__ double red[kThreads];
  __shared__ int action;          // 0 accept, 1 next trial, 2 failed
  __shared__ double t_next;
  View v = view(L, state);
  const int n = L.n, m = L.m, tid = threadIdx.x;
  if (!v.active[p]) return;
  Hdr& h = v.hdr[p];
  const float* d = v.d + (size_t)p * n;
  const float* gt = v.gt + (size_t)p * n;
  float* g = v.g + (size_t)p * n;
  const float* x0 = v.x0 + (size_t)p * n;
  float* a = alpha + (size_t)p * n;
  const double ft = v.ft[p];
  const double dt = dot(gt, d, n, red);
  if (tid == 0) {
    const double t = h.t, f0 = h.f0, dphi0 = h.dphi0;
    const bool armijo_fail = !isfinite(ft) || ft > f0 + c1 * t * dphi0;
    int act = 1;
    double tn = t;
    h.n_eval += 1;
    if (h.phase == 0) {
      if (armijo_fail || (!h.first && ft >= h.f_prev)) {
        h.lo = h.t_prev; h.flo = h.f_prev; h.glo = h.g_prev;
        h.hi = t; h.fhi = ft; h.ghi = dt;
        h.phase = 1;
        tn = cubic_min(h.lo, h.flo, h.glo, h.hi, h.fhi, h.ghi);
      } else if (fabs(dt) <= -c2 * dphi0) {
        act = 0;
      } else if (dt >= 0.0) {
        h.lo = t; h.flo = ft; h.glo = dt;
        h.hi = h.t_prev; h.fhi = h.f_prev; h.ghi = h.g_prev;
        h.phase = 1;
        tn = cubic_min(h.lo, h.flo, h.glo, h.hi, h.fhi, h.ghi);
      } else {
        h.t_prev = t; h.f_prev = ft; h.g_prev = dt;
        h.first = 0;
        tn = 2.0 * t;
      }
    } else {
      if (armijo_fail || ft >= h.flo) {
        h.hi = t; h.fhi = ft; h.ghi = dt;
      } else {
        if (fabs(dt) <= -c2 * dphi0) {
          act = 0;
        } else {
          if (dt * (h.hi - h.lo) >= 0.0) {
            h.hi = h.lo; h.fhi = h.flo; h.ghi = h.glo;
          }
          h.lo = t; h.flo = ft; h.glo = dt;
        }
      }
      if (act) tn = cubic_min(h.lo, h.flo, h.glo, h.hi, h.fhi, h.ghi);
    }
    if (act == 1 && h.n_eval >= max_evals) act = 2;
    action = act;
    t_next = tn;
  }
  __syncthreads();
  if (action == 0) {
    // accepted: history update with s = t d, y = g_new - g.  The header is
    // read by every thread before the reductions' barriers; thread 0 writes
    // it only after them.
    const double t = h.t;
    const int count = h.count, head = h.head;
    double sy = 0.0, yy = 0.0;
    for (int i = tid; i < n; i += kThreads) {
      const double si = (double)(float)(t * (double)d[i]);
      const double yi = (double)gt[i] - (double)g[i];
      sy += si * yi;
      yy += yi * yi;
    }
    sy = block_sum(sy, red);
    yy = block_sum(yy, red);
    const bool store = sy > 1e-12 * yy;
    const int slot = (count < m) ? (head + count) % m : head;
    const size_t hb = (size_t)p * m;
    float* S = v.S + (hb + slot) * n;
    float* Y = v.Y + (hb + slot) * n;
    for (int i = tid; i < n; i += kThreads) {
      if (store) {
        S[i] = (float)(t * (double)d[i]);
        Y[i] = gt[i] - g[i];
      }
      g[i] = gt[i];
    }
    if (tid == 0) {
      if (store) {
        v.rho[hb + slot] = 1.0 / sy;
        if (count < m) h.count = count + 1; else h.head = (head + 1) % m;
      }
      const double df = h.f - ft;
      h.f = ft;
      h.iter += 1;
      if (ftol > 0.0 && df <= ftol * fmax(fabs(ft), 1e-300)) h.status = 1;
      v.active[p] = 0;
    }
  } else if (action == 1) {
    const double tn = t_next;
    for (int i = tid; i < n; i += kThreads) a[i] = (float)((double)x0[i] + tn * (double)d[i]);
    if (tid == 0) {
      h.t = tn;
      if (eval >= 0) atomicAdd(v.counter + eval, 1);
    }
  } else {
    // line search failed: keep the starting point and stop this patch
    for (int i = tid; i < n; i += kThreads) a[i] = x0[i];
    if (tid == 0) {
      h.status = 2;
      v.active[p] = 0;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_lbfgs_search(LbfgsLayout L, void* state,
                                                           float* __restrict__ alpha, int eval,
                                                           double c1, double c2, int max_evals,
                                                           double ftol) {
  search_patch(blockIdx.x, L, state, alpha, eval, c1, c2, max_evals, ftol);
}

__global__ __launch_bounds__(kThreads) void k_lbfgs_search_group(GroupArgs ga, double c1,
                                                                 double c2, int max_evals,
                                                                 double ftol) {
  const int2 it = ga.item[blockIdx.x];
  const FieldDesc& F = ga.fd[it.x];
  search_patch(it.y, F.L, F.state, F.alpha, -1, c1, c2, max_evals, ftol);
}

// The accepted point of every patch: x0 while inside a line search.
__global__ __launch_bounds__(kThreads) void k_lbfgs_publish(int P, LbfgsLayout L, void* state,
                                                            const float* __restrict__ alpha,
                                                            float* __restrict__ out) {
  View v = view(L, state);
  const long i = (long)blockIdx.x * kThreads + threadIdx.x;
  const long n = L.n;
  if (i >= (long)P * n) return;
  const int p = (int)(i / n);
  out[i] = v.active[p] ? v.x0[i] : alpha[i];
}

__global__ __launch_bounds__(kThreads) void k_lbfgs_finish(int P, LbfgsLayout L, void* state,
                                                           double* loss_out, int* status_out) {
  View v = view(L, state);
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= P) return;
  if (loss_out) loss_out[p] = v.hdr[p].f;
  if (status_out) status_out[p] = v.hdr[p].status;
}

// The accepted point of the group's coefficients, blocks of 256 of one field.
__global__ __launch_bounds__(kThreads) void k_lbfgs_publish_group(GroupArgs ga) {
  const int2 it = ga.item[blockIdx.x];
  const FieldDesc& F = ga.fd[it.x];
  const long i = (long)it.y * kThreads + threadIdx.x;
  if (!F.alpha_accepted || i >= (long)F.d.P * F.L.n) return;
  View v = view(F.L, F.state);
  const int p = (int)(i / F.L.n);
  F.alpha_accepted[i] = v.active[p] ? v.x0[i] : F.alpha[i];
}

// blocks of 256 patches of one field
__global__ __launch_bounds__(kThreads) void k_lbfgs_finish_group(GroupArgs ga) {
  const int2 it = ga.item[blockIdx.x];
  const FieldDesc& F = ga.fd[it.x];
  const int p = it.y * kThreads + threadIdx.x;
  if (p >= F.d.P) return;
  View v = view(F.L, F.state);
  if (F.loss_accepted) F.loss_accepted[p] = v.hdr[p].f;
  if (F.status) F.status[p] = v.hdr[p].status;
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

LbfgsLayout lbfgs_layout(const Dims& d, int m, int max_evals) {
  LbfgsLayout L;
  L.m = m;
  L.n = d.J * d.M;
  const size_t P = d.P, n = L.n;
  size_t o = 0;
  L.hdr = o;     o = a256(o + P * sizeof(Hdr));
  L.rho = o;     o = a256(o + P * m * sizeof(double));
  L.x0 = o;      o = a256(o + P * n * sizeof(float));
  L.g = o;       o = a256(o + P * n * sizeof(float));
  L.d = o;       o = a256(o + P * n * sizeof(float));
  L.gt = o;      o = a256(o + P * n * sizeof(float));
  L.S = o;       o = a256(o + P * m * n * sizeof(float));
  L.Y = o;       o = a256(o + P * m * n * sizeof(float));
  L.ft = o;      o = a256(o + P * sizeof(double));
  L.active = o;  o = a256(o + P * sizeof(int));
  L.counter = o; o = a256(o + (size_t)(max_evals + 1) * sizeof(int));
  L.total = o;
  return L;
}

hipError_t launch_lbfgs_init(const Dims& d, const LbfgsLayout& L, void* state, double* loss_out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_lbfgs_init, dim3((d.P + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                     d.P, L, state, loss_out);
  return hipGetLastError();
}

hipError_t launch_lbfgs_begin(const Dims& d, const LbfgsLayout& L, void* state, float* alpha,
                              int max_evals, hipStream_t s) {
  hipLaunchKernelGGL(k_lbfgs_begin, dim3(d.P), dim3(kThreads), 0, s, L, state, alpha, max_evals);
  return hipGetLastError();
}

hipError_t launch_lbfgs_prep(const Dims& d, const LbfgsLayout& L, void* state, float* alpha,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_lbfgs_prep, dim3(d.P), dim3(kThreads), 0, s, L, state, alpha);
  return hipGetLastError();
}

hipError_t launch_lbfgs_publish(const Dims& d, const LbfgsLayout& L, void* state,
                                const float* alpha, float* out, hipStream_t s) {
  const long n = (long)d.P * L.n;
  hipLaunchKernelGGL(k_lbfgs_publish, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, d.P, L, state, alpha, out);
  return hipGetLastError();
}

hipError_t launch_lbfgs_search(const Dims& d, const LbfgsLayout& L, void* state, float* alpha,
                               int eval, double c1, double c2, int max_evals, double ftol,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_lbfgs_search, dim3(d.P), dim3(kThreads), 0, s, L, state, alpha, eval, c1,
                     c2, max_evals, ftol);
  return hipGetLastError();
}

hipError_t launch_lbfgs_prep_group(const GroupArgs& ga, hipStream_t s) {
  hipLaunchKernelGGL(k_lbfgs_prep_group, dim3(ga.total), dim3(kThreads), 0, s, ga);
  return hipGetLastError();
}

hipError_t launch_lbfgs_search_group(const GroupArgs& ga, double c1, double c2, int max_evals,
                                     double ftol, hipStream_t s) {
  hipLaunchKernelGGL(k_lbfgs_search_group, dim3(ga.total), dim3(kThreads), 0, s, ga, c1, c2,
                     max_evals, ftol);
  return hipGetLastError();
}

hipError_t launch_lbfgs_publish_group(const GroupArgs& ga_elems, hipStream_t s) {
  hipLaunchKernelGGL(k_lbfgs_publish_group, dim3(ga_elems.total), dim3(kThreads), 0, s,
                     ga_elems);
  return hipGetLastError();
}

hipError_t launch_lbfgs_finish_group(const GroupArgs& ga_patches, hipStream_t s) {
  hipLaunchKernelGGL(k_lbfgs_finish_group, dim3(ga_patches.total), dim3(kThreads), 0, s,
                     ga_patches);
  return hipGetLastError();
}

hipError_t launch_lbfgs_finish(const Dims& d, const LbfgsLayout& L, void* state, double* loss_out,
                               int* status_out, hipStream_t s) {
  hipLaunchKernelGGL(k_lbfgs_finish, dim3((d.P + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                     d.P, L, state, loss_out, status_out);
  return hipGetLastError();
}

}  // namespace mfbd
