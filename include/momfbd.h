/*
 * libmomfbd -- C-ABI of the MOMFBD hot path on AMD Instinct MI355X (gfx950).
 *
 * What is computed (Asensio Ramos et al., "torchmfbd: a flexible multi-object
 * multi-frame blind deconvolution code"):
 *   for every patch p, channel c (an object/diversity pair) and frame j
 *     phi   = sum_m alpha[p][j][m] Z_c,m + theta_c           (Eq. wavefront)
 *     P     = A_c exp(i phi)                                  (Sect. "Wavefronts")
 *     s     = kappa_c |IDFT(P)|^2, kappa_c = 1/(N^2 sum A_c^2) (Eq. pupil_func;
 *             unit integral of the PSF, Sect. "PSF")
 *     S     = DFT(s)
 *   for every object k (channels c with channel_object[c] == k)
 *     O_k   = sum w D conj(S) / (sum w |S|^2 + gamma_k)       (Eq. object_optimization)
 *     L_p   = sum_k sum_u [ sum_{c,j} w |D - O_k S|^2 + gamma_k |O_k|^2 ]
 *           = Eq. loss_momfbd evaluated at the Wiener object
 *   and dL/dalpha by the adjoint of that chain with the object held at its
 *   optimum.
 *
 * Conventions
 *   DFT(x)(u) = sum_r x(r) exp(-2 pi i u.r/N); IDFT is the same sum with +i
 *   and no 1/N^2.  No fftshift: the PSF of a flat wavefront peaks at pixel
 *   (0,0).  Half spectra are [N][N/2+1] arrays of interleaved complex64
 *   (kx fastest).  The loss sums over the full N x N frequency grid.
 *   Phases are in radians at the reference wavelength; a channel at another
 *   wavelength carries the lambda_0/lambda_c factor inside its basis.
 *   The frame weights w are the gamma_kj of Eq. log_posterior; "gamma" here
 *   is the Wiener constant S_n/S_0 of Eq. object_optimization.
 *
 * Memory and threading
 *   All array arguments of the per-call functions are DEVICE pointers owned
 *   by the caller, C-order and contiguous, on the device the plan was
 *   created on.  Plan creation reads HOST arrays and copies what it needs.
 *   Work is enqueued on `stream` (a hipStream_t; NULL = default stream) and
 *   nothing synchronises.  No function allocates device memory after plan
 *   creation; scratch comes from the caller's workspace.  A plan and its
 *   workspace may be used by one stream at a time.
 *
 * Workspace
 *   Every per-call function takes the caller's workspace as a device
 *   pointer `ws` and its length in bytes `ws_bytes`.  The pointer must be
 *   256-byte aligned and the length at least what the size query returns
 *   (momfbd_workspace_size, momfbd_cnn_sizes,
 *   momfbd_power_spectrum_workspace); otherwise the call returns
 *   MOMFBD_EWORKSPACE before anything is enqueued.  The solver calls take
 *   their state buffer the same way (`state`, `state_bytes`, at least
 *   momfbd_lbfgs_state_size).
 *
 * Errors
 *   Every function returns MOMFBD_OK or a negative status.  Argument errors
 *   (including a missing, misaligned or short workspace) are detected before
 *   any work is enqueued, and outputs are then left untouched.
 *   MOMFBD_EDEVICE reports a HIP error, including one left by an earlier
 *   asynchronous launch.  NaN or Inf in the inputs are not checked:
 *   they propagate into the loss of the affected patch.
 */
#ifndef MOMFBD_H
#define MOMFBD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MOMFBD_OK 0
#define MOMFBD_EINVAL (-1)        /* NULL pointer, bad size, bad channel map   */
#define MOMFBD_EUNSUPPORTED (-2)  /* patch size, mode count or pupil not supported */
#define MOMFBD_EWORKSPACE (-3)    /* workspace missing, misaligned or too small */
#define MOMFBD_EDEVICE (-4)       /* HIP error                                 */
#define MOMFBD_ESCRATCH (-5)      /* problem too large for the fixed scratch of
                                     momfbd_loss_grad_noalloc                  */

typedef struct momfbd_plan_s* momfbd_plan;

typedef struct {
  int N;   /* patch side in pixels: 64, 96 or 128                            */
  int P;   /* number of patches                                              */
  int C;   /* number of channels (object/diversity pairs), 1..32             */
  int K;   /* number of objects, 1..32                                       */
  int J;   /* frames per channel                                             */
  int M;   /* wavefront modes, 1..256; J*M <= 8192                           */
  const int* channel_object; /* HOST [C]: object of each channel, in [0,K);
                                every object must own at least one channel  */
} momfbd_desc;

/* Create a plan (Sect. "Wavefronts").
 *   pupil     HOST float [C][N][N]: aperture transmission A_c(v) >= 0.  Its
 *             support must fit in an (N/2) x (N/2) box (a pupil diameter below
 *             N/2 pixels, which also keeps the OTF free of aliasing); the plan
 *             translates it to the centre of the grid, which leaves the PSF
 *             unchanged.
 *   basis     HOST float [C][M][N][N]: modes Z_c,m in radians (already scaled
 *             by lambda_0/lambda_c).
 *   diversity HOST float [C][N][N] in radians, or NULL for none.
 *   out       receives the plan.
 * Allocates device tables on the current device.
 * Errors: EINVAL (NULL, sizes, channel map, zero pupil), EUNSUPPORTED (N,
 * M, J*M, pupil support), EDEVICE. */
int momfbd_plan_create(const momfbd_desc* desc, const float* pupil, const float* basis,
                       const float* diversity, momfbd_plan* out);

/* Release a plan (NULL is accepted).  The caller must have synchronised any
 * stream still using it. */
int momfbd_plan_destroy(momfbd_plan plan);

/* Bytes of device workspace needed by every per-call function of this plan.
 * The workspace must be 256-byte aligned. */
int momfbd_workspace_size(momfbd_plan plan, size_t* bytes);

/* Data preparation (Sect. "Division in patches and apodization").
 *   frames  DEVICE float [C][J][H][W] observed images.
 *   stride  patch step: corners y0 = i*stride, i = 0..(H-N)/stride, same
 *           for x; patches ordered row-major; their count must equal P.
 *   apod    DEVICE float [N][N] apodization window W.
 *   D       DEVICE complex64 [P][C][J][N][N/2+1] output:
 *           D = DFT(W (x - m) + m), m the mean of each patch frame.
 * Errors: EINVAL (NULL, H/W/stride inconsistent with P), EWORKSPACE, EDEVICE. */
int momfbd_prepare_data(momfbd_plan plan, const float* frames, int H, int W, int stride,
                        const float* apod, void* D, void* ws, size_t ws_bytes, void* stream);

/* Forward model only: PSFs and/or OTFs for coefficients alpha.
 *   alpha   DEVICE float [P][J][M].
 *   psf     DEVICE float [P][C][J][N][N] unit-sum PSFs, or NULL.
 *   otf     DEVICE complex64 [P][C][J][N][N/2+1] OTF half spectra, or NULL.
 * Errors: EINVAL, EWORKSPACE, EDEVICE. */
int momfbd_forward(momfbd_plan plan, const float* alpha, float* psf, void* otf, void* ws,
                   size_t ws_bytes, void* stream);

/* Loss and gradient (Eqs. object_optimization and loss_momfbd).
 *   alpha        DEVICE float [P][J][M]
 *   D            DEVICE complex64 [P][C][J][N][N/2+1] data spectra
 *   gamma        DEVICE float [K][N][N/2+1] per-frequency Wiener constant, or
 *                NULL to use gamma_scalar for every object and frequency
 *   weights      DEVICE float [C][J] frame weights w, or NULL for 1
 *   loss         DEVICE double [P]: L_p (FP64 reduction)
 *   grad         DEVICE float [P][J][M]: dL_p/dalpha, or NULL for loss only
 * Errors: EINVAL, EWORKSPACE, EDEVICE. */
int momfbd_loss_grad(momfbd_plan plan, const float* alpha, const void* D, const float* gamma,
                     float gamma_scalar, const float* weights, double* loss, float* grad,
                     void* ws, size_t ws_bytes, void* stream);

/* Loss and gradient without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): momfbd_loss_grad with the workspace taken
 * from a fixed scratch buffer inside the library instead of the caller.
 *   Every argument as momfbd_loss_grad; there is no ws argument.
 *   The scratch is one buffer per device of 64 MiB (67 108 864 bytes),
 *   created when the library is loaded and kept until the process ends; its device address is looked up once per device by
 *   momfbd_plan_create.  The call allocates nothing (no hipMalloc, no
 *   host allocation) and synchronises nothing.
 *   Every call on one device uses that device's buffer, which keeps the
 *   last call's intermediates: calls that may overlap on one device (other
 *   streams, other threads, other plans) race and must be serialised by the
 *   caller.  No part of the buffer needs clearing between calls (every
 *   kernel of the chain writes what it later reads).
 * Errors: EINVAL, ESCRATCH (momfbd_workspace_size of the plan exceeds
 * 64 MiB, e.g. more than about 100 patches of 64 x 64 with 24 frames over
 * two channels; use momfbd_loss_grad), EDEVICE. */
int momfbd_loss_grad_noalloc(momfbd_plan plan, const float* alpha, const void* D,
                             const float* gamma, float gamma_scalar, const float* weights,
                             double* loss, float* grad, void* stream);

/* Wiener object estimate in pixel space (Eq. object_optimization):
 *   obj  DEVICE float [P][K][N][N], o_k = Re IDFT(O_k) / N^2 -- the restored
 *        apodized patch in the units of the frames.
 * Other arguments as momfbd_loss_grad.  Errors: EINVAL, EWORKSPACE, EDEVICE. */
int momfbd_object_estimate(momfbd_plan plan, const float* alpha, const void* D,
                           const float* gamma, float gamma_scalar, const float* weights,
                           float* obj, void* ws, size_t ws_bytes, void* stream);

/* Object smoothness prior (Sect. "Smoothness", Eq. regularization_smoothness):
 * the penalty lambda_k ||grad o_k||^2, with periodic forward differences, added
 * to the pixel-domain misfit is, in the unnormalised Fourier sum of Eq.
 * loss_momfbd, the per-frequency Wiener constant
 *   gamma_k(u) = gamma0_k + lambda_k (4 sin^2(pi u_x/N) + 4 sin^2(pi u_y/N)),
 * so lambda_k does not depend on N.  Writes that table, float [K][N][N/2+1]
 * (device, caller-allocated), to be passed as `gamma` to loss_grad,
 * object_estimate and the solver.  gamma0, lambda: host [K], finite, >= 0.
 * Errors: EINVAL (NULL or out-of-range constant), EDEVICE. */
int momfbd_smoothness_gamma(momfbd_plan plan, const float* gamma0, const float* lambda,
                            float* gamma, void* stream);

/* Fourier filter of a restored object (Sect. "Fourier filtering"). */
#define MOMFBD_FILTER_NONE 0
#define MOMFBD_FILTER_TOPHAT 1     /* H = 1 for f <= f_lo, 0 for f >= f_hi, cosine between */
#define MOMFBD_FILTER_SCHARMER 2   /* Loefdahl-Scharmer, see momfbd_object_filtered */
typedef struct {
  int kind;            /* MOMFBD_FILTER_*                                           */
  float f_lo, f_hi;    /* top-hat: transition, in units of the diffraction limit     */
  float diff_limit;    /* top-hat: diffraction-limit frequency in DFT bins, > 0       */
  float noise_power;   /* Loefdahl-Scharmer: noise power of one data frame per
                          frequency bin (eta), >= 0                                  */
} momfbd_filter;

/* Restored objects after a Fourier filter per object (Sect. "Fourier
 * filtering"): the Wiener objects of momfbd_object_estimate, each spectrum
 * multiplied by H_k before the inverse transform.  Frequencies f = |u| in
 * bins with u in (-N/2, N/2].  Loefdahl-Scharmer: H = 1 - eta sum w|S|^2 /
 * |sum w D conj(S)|^2 over the channels of the object (the printed ratio is
 * eta = 1; H = 0 where the cross spectrum vanishes), values below 0.2 set to
 * 0 and above 1 to 1, then a 3x3 median on the periodic frequency grid, then
 * zero outside the region 4-connected to the zero frequency.  The filter does
 * not enter the loss.
 *   filters  host [K]
 *   obj      [P][K][N][N] float (device), as momfbd_object_estimate
 *   H        [P][K][N][N/2+1] float (device) receives the filters, or NULL
 * Errors: EINVAL (NULL, unknown kind, f_hi <= f_lo, diff_limit <= 0,
 * eta < 0), EWORKSPACE, EDEVICE. */
int momfbd_object_filtered(momfbd_plan plan, const float* alpha, const void* D,
                           const float* gamma, float gamma_scalar, const float* weights,
                           const momfbd_filter* filters, float* obj, float* H, void* ws,
                           size_t ws_bytes, void* stream);

/* Mosaic of restored patches (Sect. "Division in patches and apodization"):
 * out_k(y, x) = sum_p w(y - y_p, x - x_p) o_pk(y - y_p, x - x_p) / sum_p w(.)
 * over the patches covering the pixel, patch p = i*nx + k at
 * (y_p, x_p) = (i*stride, k*stride), with the separable cosine taper
 * w1(e) = (1 - cos(pi (e + 1/2)/border))/2 for e = min(x, N-1-x) < border,
 * else 1 (border = 0: equal weights).
 *   obj  [P][K][N][N] float (device), P = ny*nx
 *   out  [K][(ny-1)*stride+N][(nx-1)*stride+N] float (device)
 * Errors: EINVAL (ny*nx != P, stride outside [1, N], border outside
 * [0, N/2]), EDEVICE. */
int momfbd_mosaic(momfbd_plan plan, const float* obj, int ny, int nx, int stride, int border,
                  float* out, void* stream);

/* Power spectrum of an L x L image (L a power of two, 16..4096) and its
 * average over 30-degree sectors along the +-45 degree directions as a
 * function of the radial frequency (Sect. "Results"):
 *   power[u_y][u_x] = |DFT(w (x - mean x))|^2   (float, device, [L][L])
 *   sector[k] = mean of power over the sector frequencies with
 *               round(|u|) = k, k = 0..nbins-1 (double, device; 0 where no
 *               frequency falls), counts[k] their number (int, device, or NULL)
 * with u in (-L/2, L/2] and the sector 30..60 degrees from the axes in all
 * four quadrants.  window: [L][L] float (device) or NULL (= 1); sector NULL
 * skips the averaging.  Workspace from momfbd_power_spectrum_workspace
 * (device, 256-byte aligned).  1 <= nbins <= L.
 * Errors: EINVAL, EWORKSPACE, EDEVICE. */
int momfbd_power_spectrum_workspace(int L, int nbins, size_t* bytes);
int momfbd_power_spectrum(int L, const float* image, const float* window, float* power,
                          double* sector, int* counts, int nbins, void* ws, size_t ws_bytes,
                          void* stream);

/* Per-patch L-BFGS solver (the quasi-Newton alternative to the paper's Adam,
 * Sect. "Optimization and paralellization"; patches are independent).
 * Each patch runs the two-loop recursion of limited-memory BFGS and a
 * bracketing/zoom line search enforcing the strong Wolfe conditions
 * (Nocedal & Wright, Numerical Optimization, Algorithms 7.4, 3.5, 3.6);
 * zoom trials are the clamped cubic-interpolation minimiser; all scalars
 * FP64. */
typedef struct {
  int m;           /* stored correction pairs, 1..32 (10 is usual)              */
  int max_evals;   /* loss+gradient evaluations per line search, 1..1000 (20)  */
  double c1;       /* sufficient-decrease constant, 0 < c1 < c2 (1e-4)          */
  double c2;       /* curvature constant, c1 < c2 < 1 (0.9)                     */
  double ftol;     /* a patch stops when its loss falls by <= ftol*|loss| in one
                      iteration (0: never)                                      */
} momfbd_lbfgs_params;

/* Bytes of solver state (device memory, 256-byte aligned, owned by the
 * caller) for this plan and these parameters.  Errors: EINVAL.
 * The solver calls below take the state with its length (`state_bytes`):
 * a NULL or misaligned state is EINVAL, a shorter one EWORKSPACE. */
int momfbd_lbfgs_state_size(momfbd_plan plan, const momfbd_lbfgs_params* params, size_t* bytes);

/* Start a solve at alpha (DEVICE float [P][J][M]): evaluates loss and
 * gradient, clears the history.  loss (DEVICE double [P]) may be NULL.
 * Other arguments as momfbd_loss_grad.  Errors: EINVAL, EWORKSPACE, EDEVICE. */
int momfbd_lbfgs_init(momfbd_plan plan, const momfbd_lbfgs_params* params, void* state,
                      size_t state_bytes, const float* alpha, const void* D, const float* gamma,
                      float gamma_scalar, const float* weights, double* loss, void* ws,
                      size_t ws_bytes, void* stream);

/* One L-BFGS iteration for every patch that has not stopped.  alpha is
 * updated in place (DEVICE float [P][J][M], the same array the solve was
 * started with).  loss (DEVICE double [P], or NULL) receives each patch's
 * loss at its accepted point; status (DEVICE int [P], or NULL): 0 running,
 * 1 converged (relative decrease <= ftol, or zero gradient), 2 stopped
 * (line search found no strong-Wolfe point within max_evals; alpha is left
 * at the start of that search).  Evaluations run only for patches still
 * searching; after each, the call synchronises `stream` to read how many
 * remain.  Errors: EINVAL, EWORKSPACE, EDEVICE. */
int momfbd_lbfgs_step(momfbd_plan plan, const momfbd_lbfgs_params* params, void* state,
                      size_t state_bytes, float* alpha, const void* D, const float* gamma,
                      float gamma_scalar, const float* weights, double* loss, int* status,
                      void* ws, size_t ws_bytes, void* stream);

/* Solver rounds without host synchronisation, for HIP graph capture.  A
 * round gives every running patch one line-search trial: a patch that is
 * not inside a line search first starts its next iteration (two-loop
 * direction, first trial step), then the loss and gradient of all patches
 * inside a search are evaluated, then each advances its search (accept,
 * next trial, or fail after max_evals trials).  Patches advance
 * independently, so each follows the trajectory it follows under
 * momfbd_lbfgs_step; the call enqueues a fixed sequence of kernels
 * (rounds x (prep, evaluation, search), then publish and finish) with no
 * read-back and no memset.
 *   alpha           in/out: a patch inside a search holds its trial point
 *   loss, status    [P] (device, may be NULL): last accepted loss; 0 running,
 *                   1 converged (ftol), 2 line search failed
 *   alpha_accepted  [P][J][M] (device, may be NULL): the last accepted
 *                   coefficients of every patch
 * momfbd_lbfgs_step after rounds restarts searching patches from their
 * accepted point.  Errors: EINVAL, EWORKSPACE, EDEVICE. */
int momfbd_lbfgs_rounds(momfbd_plan plan, const momfbd_lbfgs_params* params, void* state,
                        size_t state_bytes, float* alpha, const void* D, const float* gamma,
                        float gamma_scalar, const float* weights, int rounds, double* loss,
                        int* status, float* alpha_accepted, void* ws, size_t ws_bytes,
                        void* stream);

/* Synthetic bursts through the forward model (Eq. generative_model):
 * per patch p, channel c, frame j the frame i = o_k * s_pcj + sigma_p n
 * (circular convolution of the object o_k of the channel with the PSF of
 * alpha[p][j]), then D = DFT(W(i - m) + m) as momfbd_prepare_data.
 *   alpha   [P][J][M] float (device)
 *   O       [P][K][N][N/2+1] complex64 (device): object spectra DFT(o)
 *   noise   [P][C][J][N][N] float (device): standard normal draws
 *   sigma   [P] float (device): noise standard deviation per patch
 *   apod    [N][N] float (device)
 *   frames  [C][J][P*N][N] float (device): receives the noisy frames
 *   D       [P][C][J][N][N/2+1] complex64 (device): receives the spectra
 * Every patch size and channel count of the plan.  Errors: EINVAL,
 * EWORKSPACE, EDEVICE. */
int momfbd_synthesize(momfbd_plan plan, const float* alpha, const void* O, const float* noise,
                      const float* sigma, const float* apod, float* frames, void* D, void* ws,
                      size_t ws_bytes, void* stream);

/* Standard normal draws for synthetic bursts (the noise of
 * momfbd_synthesize, the network's initial weights): Philox4x32-10 (Salmon
 * et al., SC 2011) with key = seed and counter = (counter0 + i/4, stream_id)
 * as 64-bit halves, low word first, and the Box-Muller transform of each
 * pair of words: draw i uses word i % 4 of block counter0 + i/4, paired with
 * its neighbour (words 0,1 give cos and sin of one pair, words 2,3 of the
 * next), u = ((x >> 8) + 1/2) 2^-24, r = sqrt(-2 ln u_first),
 * angle 2 pi u_second.  A call of n draws from counter0 continues exactly
 * where a call ending at counter0 stopped, when n is a multiple of 4.
 *   out   [n] float (device) receives the draws
 *   bits  [n] uint32 (device) receives the generator's word of each draw,
 *         or NULL
 * Errors: EINVAL (NULL, n = 0 or n > 2^40), EDEVICE. */
int momfbd_random_normal(unsigned long long seed, unsigned long long stream_id,
                         unsigned long long counter0, size_t n, float* out, unsigned int* bits,
                         void* stream);

/* Warm-start network: a 6-layer convolutional regressor from a burst of J
 * frames (N x N, N = 64, 96 or 128) to J x M modal coefficients (Noll
 * j = 2..M+1, the lowest M modes of the solve), with bfloat16 weights and
 * activations and FP32 accumulation on the matrix cores.  Layers: four 3x3
 * stride-2 convolutions (J->32->64->128->128 channels, ReLU), dense
 * 128 (N/16)^2 -> 512 (ReLU), dense 512->J*M, times mode_scale.
 * The input of every burst is the first channel of its data half spectra
 * D [B][C][J][N][N/2+1] (as for momfbd_loss_grad); the network sees the
 * apodized frames IDFT(D)/N^2, each divided by its mean.
 * Training loss per frame: sum over modes of mode_scale_m^2 / mean(
 * mode_scale^2) times the squared error in units of mode_scale, after
 * removing the burst mean of the two tilt modes, taking the smaller of the
 * errors to the target and to the target with its even-radial-order modes
 * negated (frames cannot tell these apart without diversity, Sect.
 * "Wavefronts"); the loss is the mean over bursts and frames.
 * Parameters are one FP32 vector (weights [out][3][3][in] or [out][in],
 * then biases, layer by layer); the workspace holds the bfloat16 copy used
 * by the kernels, refreshed by momfbd_cnn_init, momfbd_cnn_load and
 * momfbd_cnn_adam. */
typedef struct momfbd_cnn_s* momfbd_cnn;
/* mode_scale HOST [M] > 0; J <= 64, J*M <= 2048; batch_max bursts per call.
 * Errors: EINVAL, EUNSUPPORTED (N), EDEVICE. */
int momfbd_cnn_create(int N, int J, int M, int batch_max, const float* mode_scale,
                      momfbd_cnn* out);
int momfbd_cnn_destroy(momfbd_cnn net);
int momfbd_cnn_sizes(momfbd_cnn net, size_t* n_params, size_t* workspace_bytes);
/* params = normals * He standard deviation per weight (biases 0; the last
 * layer's weights 10x smaller); normals: [n_params] device draws. */
int momfbd_cnn_init(momfbd_cnn net, const float* normals, float* params, void* ws,
                    size_t ws_bytes, void* stream);
/* refresh the workspace's bfloat16 weights from FP32 params */
int momfbd_cnn_load(momfbd_cnn net, const float* params, void* ws, size_t ws_bytes,
                    void* stream);
/* alpha [B][J][M] float (device) predicted from D [B][C][J][N][N/2+1]
 * (channel 0 is read); B <= batch_max */
int momfbd_cnn_forward(momfbd_cnn net, const float* params, const void* D, int B, int C,
                       float* alpha, void* ws, size_t ws_bytes, void* stream);
/* The network's input for D (as momfbd_cnn_forward): x [B][N][N][J] float
 * (device, frames as channels), each frame of channel 0 (IDFT(D) / N^2)
 * divided by its mean, minus one, times ten, rounded to bfloat16 as the
 * first layer reads it (the values returned as floats).  For checking the
 * layers on exactly the values they read.  Errors: EINVAL, EWORKSPACE,
 * EDEVICE. */
int momfbd_cnn_input(momfbd_cnn net, const void* D, int B, int C, float* x, void* ws,
                     size_t ws_bytes, void* stream);
/* loss (one FP64, device) and grad [n_params] (device) for targets
 * [B][J][M] float (device); D as momfbd_cnn_forward */
int momfbd_cnn_loss_grad(momfbd_cnn net, const float* params, const void* D, int C,
                         const float* target, int B, double* loss, float* grad, void* ws,
                         size_t ws_bytes, void* stream);
/* one Adam step (FP32 moments m1, m2 [n_params]; step >= 1) */
int momfbd_cnn_adam(momfbd_cnn net, float* params, const float* grad, float* m1, float* m2,
                    int step, float lr, float beta1, float beta2, float eps, void* ws,
                    size_t ws_bytes, void* stream);

/* Kernel timing for measurement.  After momfbd_profile_start, every kernel
 * launched by this plan's calls (up to max_launches launches) is bracketed
 * by a pair of HIP events recorded on the call's stream.  Events are created
 * here, not in the calls, with a device-scope release (no system-scope cache
 * write-back between the timed kernels).  Errors: EINVAL, EDEVICE. */
int momfbd_profile_start(momfbd_plan plan, int max_launches);

/* Back-to-back timing of one kernel kind (after momfbd_profile_start): from
 * now until momfbd_profile_stop only the launches of `kind` are bracketed,
 * and each is issued `reps` times in a row inside its event pair, so the
 * kernel is timed without the idle gaps that per-launch events put in front
 * of it.  Every kernel overwrites its outputs, so results are unchanged;
 * "filter" (which scales the object spectrum in place) is refused.  The
 * reported launch count includes the repeats.  Errors: EINVAL (no timing
 * started, unknown kind, reps < 1). */
int momfbd_profile_repeat(momfbd_plan plan, const char* kind, int reps);

/* Synchronise on the recorded events, stop timing, and report per kernel
 * kind: a static name ("phase", "forward", "object", "adjoint", "grad",
 * "prepare", "objimg", "filter", "mosaic"), the summed milliseconds and the launch count, for at
 * most `cap` kinds.  Returns the number of kinds written (>= 0) or a
 * negative status. */
int momfbd_profile_stop(momfbd_plan plan, int cap, const char** names, double* total_ms,
                        int* launches);

/* Human-readable text of a status code. */
const char* momfbd_status_string(int status);

/* Launch schedules of a plan: how units and frequencies map to workgroups.
 * Results are the same for every schedule up to the order of floating-point
 * sums (the unit order changes nothing; the object kernel's pairs per
 * thread change the grouping of the FP64 loss partials, the gradient
 * contraction's waves and splits the grouping of its FP32 partial sums). */
typedef struct {
  int xcd_forward;              /* 1: units of a patch-object on one XCD (L2)   */
  int xcd_adjoint;              /* same for the adjoint kernel                  */
  int object_pairs_per_thread;  /* 1, 2 or 4 frequency pairs per thread         */
  int grad_waves;               /* gradient contraction: 4 waves x 4, 3 or 2
                                   row tiles, or 8 waves x 2 row tiles per
                                   workgroup; every wave owns its rows, and
                                   each basis chunk staged in LDS serves all
                                   the workgroup's rows                       */
  int grad_splits;              /* workgroups sharing one row block's pixel
                                   sum: 1, 2, 4 or 8; 0 on input picks the
                                   count from the number of row blocks and
                                   pixel chunks (get_tuning reports the count
                                   in use)                                    */
  int grad_row_tiles;           /* row tiles of 16 (patch, frame) rows per
                                   wave: 4, 3 or 2 with 4 waves (fewer: more,
                                   smaller workgroups, each basis chunk
                                   serving fewer rows), 2 with 8 waves; 0 on
                                   input is 4 or 2 (get_tuning reports the
                                   count in use)                              */
  int phase_col_tiles;          /* phase contraction (Eq. wavefront): 16-column
                                   tiles of (patch, frame) columns per
                                   workgroup, whose coefficients it stages in
                                   LDS, each basis part read serving them all */
  int phase_waves;              /* and its waves: 8 x 8, 4 x 8 or 8 x 16
                                   (tiles x waves) while the staged
                                   coefficients fit 128 KB of LDS; 0, 0 on
                                   input picks 8 x 8 where it fits, else 4 x 4
                                   or 2 x 4 (get_tuning reports the shape in
                                   use; set_tuning also takes the automatic
                                   shape as reported)                         */
  int object_fused;             /* 1: the forward transforms and the Wiener
                                   object and loss (Eqs. object_optimization,
                                   loss_momfbd) in one launch, a workgroup per
                                   (patch, object) that reads its own OTFs back
                                   from the caches; 0 (default): two launches.
                                   Applies to 64x64 patches with at most 12
                                   units (channels x frames) per object;
                                   results are the same bit for bit.
                                   get_tuning reports 1 only where in use    */
} momfbd_tuning;
/* Errors: EINVAL (NULL, a value out of range, or a phase shape whose
 * staged coefficients do not fit). */
int momfbd_plan_set_tuning(momfbd_plan plan, const momfbd_tuning* tuning);
int momfbd_plan_get_tuning(momfbd_plan plan, momfbd_tuning* tuning);
/* Choose the schedules by timing: one knob at a time, every candidate value
 * is timed on the caller's data (HIP events on `stream`, which this call
 * synchronises) by the one kernel the knob changes (object_fused: the
 * forward and object launches together), run 4 x `reps` times back to back
 * after a whole evaluation under that candidate's schedule,
 * in three interleaved rounds; each candidate keeps its fastest round, and
 * the fastest candidate is kept.  The first candidate of each knob is the
 * library default, and another value replaces the best so far only when at
 * least 1% faster.
 * loss [P] and grad [P][J][M] (device) receive an evaluation under the
 * chosen schedules.  The choice is stored in the plan and, if `chosen` is
 * not NULL, returned.  Errors: EINVAL, EWORKSPACE, EDEVICE. */
int momfbd_plan_autotune(momfbd_plan plan, const float* alpha, const void* D, const float* gamma,
                         float gamma_scalar, const float* weights, int reps, double* loss,
                         float* grad, void* ws, size_t ws_bytes, void* stream,
                         momfbd_tuning* chosen);

/* Groups: many independent fields of one patch size (for instance the
 * fields of an observing run, each with its own frame count, mode count,
 * objects, pupils and data) solved together, with one kernel launch per
 * stage of the loss/gradient chain and of the solver round covering every
 * patch of every field (Sect. "Optimization and paralellization": patches
 * are independent, and batching them fills the GPU).  Each field keeps its
 * own plan (created as usual), workspace and solver state; the results of
 * every field are those its own plan gives (the arithmetic per patch is the
 * same, and so is the order of every sum), only the launches are shared.
 *
 * A field binds its device arrays once, at group creation:
 *   plan           the field's plan; every plan of a group has the same N and
 *                  was created on the current device
 *   alpha          [P][J][M] coefficients, read (and, by the solver rounds,
 *                  updated in place: the trial point of running patches)
 *   D, gamma, gamma_scalar, weights   as momfbd_loss_grad
 *   ws, ws_bytes   the field's own workspace (momfbd_workspace_size of its
 *                  plan); fields must not share workspaces
 *   state, state_bytes   the field's solver state, started by
 *                  momfbd_lbfgs_init with the group's params (solver groups
 *                  only; else NULL)
 *   loss, grad     [P], [P][J][M] outputs of momfbd_group_loss_grad, or NULL
 *                  (then that call is refused)
 *   loss_accepted, status, alpha_accepted   outputs of the solver rounds
 *                  ([P], [P], [P][J][M]), each may be NULL
 * The arrays must stay valid, and in place, for the life of the group. */
typedef struct momfbd_group_s* momfbd_group;
typedef struct {
  momfbd_plan plan;
  float* alpha;
  const void* D;
  const float* gamma;
  float gamma_scalar;
  const float* weights;
  void* ws;
  size_t ws_bytes;
  void* state;
  size_t state_bytes;
  double* loss;
  float* grad;
  double* loss_accepted;
  int* status;
  float* alpha_accepted;
} momfbd_field;

/* Create a group of n >= 1 fields (host array `fields`, copied).  params:
 * the solver parameters the states were started with, or NULL for a group
 * that only evaluates.  Allocates the group's device tables.
 * Errors: EINVAL (NULL, mixed N or devices, bad params), EWORKSPACE (a
 * field's workspace or state missing, misaligned or short), EUNSUPPORTED
 * (more than 2^28 work items in one stage), EDEVICE. */
int momfbd_group_create(const momfbd_field* fields, int n, const momfbd_lbfgs_params* params,
                        momfbd_group* out);
int momfbd_group_destroy(momfbd_group group);

/* Loss and gradient of every field at its alpha into its loss and grad
 * (momfbd_loss_grad for each field, in one launch per stage).
 * Errors: EINVAL (a field without loss or grad outputs), EDEVICE. */
int momfbd_group_loss_grad(momfbd_group group, void* stream);

/* `rounds` solver rounds of every field (momfbd_lbfgs_rounds for each field,
 * in one launch per stage), then the accepted loss, status and coefficients
 * of every field into its bound outputs.  No host synchronisation, no
 * allocation: capturable in a HIP graph.  Errors: EINVAL (not a solver
 * group, rounds < 0), EDEVICE. */
int momfbd_group_lbfgs_rounds(momfbd_group group, int rounds, void* stream);

/* Launch schedules of a group (the fields of momfbd_tuning that apply:
 * xcd_forward, xcd_adjoint, grad_splits, grad_row_tiles 4, 3 or 2 (0: 4, or
 * 3 and 2 where the group's largest mode count reaches 176 and 224, whose
 * accumulators would not fit four tiles); grad_waves must be 4; the phase
 * fields are ignored: a group's phase blocks are 4 tiles x 8 waves; a group
 * runs the forward and object pass in two launches, object_fused is
 * ignored and reported 0).  The autotuner times momfbd_group_loss_grad over
 * `reps` evaluations per candidate with the plan autotuner's method and
 * keeps the fastest schedule.  Errors: EINVAL, EDEVICE. */
int momfbd_group_set_tuning(momfbd_group group, const momfbd_tuning* tuning);
int momfbd_group_get_tuning(momfbd_group group, momfbd_tuning* tuning);
int momfbd_group_autotune(momfbd_group group, int reps, void* stream, momfbd_tuning* chosen);

/* Sizes the plan was created with (any out pointer may be NULL). */
int momfbd_plan_dims(momfbd_plan plan, int* N, int* P, int* C, int* K, int* J, int* M);

#ifdef __cplusplus
}
#endif

#endif /* MOMFBD_H */
