/*
 * nlinv.h -- C-ABI of the MI355X (gfx950) NLINV hot path.
 *
 * NLINV (Sec. 2.2 of Schaetz, Voit, Frahm, Uecker, "Accelerated Computing in
 * MRI: Real-Time Imaging Using Non-Linear Inverse Reconstruction") jointly
 * estimates an image rho and J coil sensitivities c_j from multi-channel
 * radial k-space data y by minimising ||F x - y||^2 + alpha ||W (x - x_prev)||^2
 * (the objective of Sec. 2.2) with the iteratively regularised Gauss-Newton
 * method (the IRGNM update equation of Sec. 2.2), each Newton system being
 * solved by conjugate gradients on DF^H DF + alpha I (the normal-operator
 * equation of Sec. 2.2).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Sizes: G = grid side = 2 gamma N with 1 <= gamma <= 2 (Sec. 3.2,
 *    grid oversampling; 2N unless given), R = G/2 reconstructed side,
 *    G_c = G/4 coil-spectrum side (Sec. 3.2, coil cropping),
 *    S = K * S_r samples per channel, X = R*R + J*G_c*G_c unknowns.
 *    Supported grids: G in {64, 128, 256, 320, 384, 432, 448, 480, 512} with
 *    2N <= G <= 4N.
 *    Every array is on the R x R field of view; for gamma > 1 the N x N
 *    output image is its centre, rows and columns R/2 - floor(N/2) to
 *    R/2 + ceil(N/2) - 1.
 *  - complex64 is interleaved (re, im) float32 (nlinv_c64).
 *  - Images are R x R row-major [y][x]; pixel (0,0) sits at (x, y) =
 *    (-R/2, -R/2) pixels.  The unknown x_hat = W x is stored as the image rho
 *    [R][R] followed by J coil spectra c_hat_j [G_c][G_c] (row-major
 *    [kappa_y][kappa_x], DC at (G_c/2, G_c/2)); c_j = W^-1 c_hat_j.
 *  - Trajectories are float32 [K][S_r][2] (kx, ky) in cycles/pixel; radial
 *    data are [J][K*S_r].  The non-uniform Fourier transform is
 *    (F u)_s = (1/R) sum_r u(r) exp(-i 2 pi k_s . r), unitary when the samples
 *    are the R x R Cartesian frequencies of the field of view.
 *  - The batch dimension B (plan parameter `batch`) is outermost in every
 *    array: B independent problems of the same shape are processed per call.
 *  - All d_* pointers are device pointers owned by the caller; they must be
 *    8-byte aligned.  h_* pointers are host pointers read before the call
 *    returns.  Inputs and outputs must not overlap unless stated.
 *  - The plan owns only host metadata.  All device scratch memory (tables,
 *    PSF kernels, intermediate buffers, CG vectors, FP64 partial sums) lives
 *    in the caller-supplied workspace; no call allocates device memory.
 *  - Every call enqueues asynchronously on the plan's HIP stream and returns;
 *    nothing synchronises except nlinv_sync.  A plan is used by one host
 *    thread at a time; calls on one plan are ordered by its stream.
 *  - Errors: 0 = NLINV_OK, negative codes below.  Arguments are validated on
 *    the host before anything is enqueued, so a failing call has no side
 *    effects.  Launch failures are reported as NLINV_E_HIP; asynchronous
 *    device errors surface at the next call or at nlinv_sync.
 *    nlinv_last_error returns a description that stays valid until the next
 *    call on the same plan.
 */
#ifndef NLINV_H
#define NLINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nlinv_plan_s* nlinv_plan;
typedef struct { float re, im; } nlinv_c64;

enum {
  NLINV_OK = 0,
  NLINV_E_ARG = -1,        /* NULL / misaligned pointer, bad value          */
  NLINV_E_SIZE = -2,       /* unsupported size combination                 */
  NLINV_E_WORKSPACE = -3,  /* workspace missing or too small               */
  NLINV_E_HIP = -4,        /* HIP runtime / launch error                   */
  NLINV_E_STATE = -5,      /* call order violated (e.g. PSF not computed)  */
  NLINV_E_NONFINITE = -6,  /* NLINV_F_CHECK_FINITE: a result was NaN / Inf */
  NLINV_E_BUDGET = -7,     /* the device's workspace budget is exhausted    */
};

/* Plan flags.
 * NLINV_F_EXACT_GRID: nlinv_grid always forms the exact sum (see
 *   nlinv_grid); without it, calls that name the turns use Kaiser-Bessel
 *   gridding through per-turn tables.
 * NLINV_F_CHECK_FINITE: after every nlinv_reconstruct /
 *   nlinv_reconstruct_frames one more kernel checks the result x_hat for NaN
 *   and infinity and sets a device flag (no host synchronisation); the next
 *   nlinv_sync returns NLINV_E_NONFINITE if it is set, and clears it.
 * Precision (not a flag): every transform runs in float64 arithmetic with
 * float64 intermediates; the CG vectors, inner products and scalars and the
 * Newton update are float64; the data, the gridded data, the unknowns x_hat,
 * the coil images and the per-channel products are stored as complex64.
 * Bits 1 and 8 are not flags (rejected with NLINV_E_ARG). */
enum { NLINV_F_EXACT_GRID = 2, NLINV_F_CHECK_FINITE = 4 };

/* Plan parameters.  nlinv_params_default fills the defaults noted here. */
typedef struct {
  int32_t N;          /* image side (required)                                  */
  int32_t G;          /* grid side 2 gamma N, 2N..4N; 0 -> 2N (gamma = 1)       */
  int32_t J;          /* channels (virtual coils), 1..64                         */
  int32_t K;          /* spokes per frame, odd                                   */
  int32_t S_r;        /* samples per spoke; 0 -> 2N                              */
  int32_t U;          /* turns = number of cached PSF kernels, 1..64 (default 1) */
  int32_t batch;      /* B >= 1, <= 64 (default 1)                               */
  int32_t newton;     /* M Newton steps (default 7)                              */
  int32_t cg;         /* C CG iterations per Newton step (default 10)            */
  int32_t flags;      /* NLINV_F_* bits (default 0)                              */
  double alpha0;      /* first regularisation weight (default 1.0)               */
  double alpha_q;     /* alpha_{n+1} = max(alpha_n * alpha_q, alpha_min) (0.5)   */
  double alpha_min;   /* (default 0.0)                                           */
  double sob_a;       /* Sobolev weight (1 + a |k|^2)^l, Fig. weight_func: 880   */
  double sob_l;       /*                                                    : 16 */
  int32_t col_tile;   /* tile schedule: columns per block of the two column    */
                      /* passes of a CG iteration, 0 or 8 (default) or 4       */
                      /* (twice the blocks); results are identical bit for bit */
  int32_t cg_passes;  /* form of a CG iteration: 6 = coil rows with the        */
                      /* direction update, the four operator passes, the CG   */
                      /* vector step; 4 = the direction update, W^-1 p and the */
                      /* vector step folded into the operator's passes, with   */
                      /* Re<p, q> from the spectrum (Parseval; two dependent   */
                      /* kernels fewer, about 15 % more bytes); 0 (default) =  */
                      /* 6.  Both forms are the same CG in exact arithmetic;   */
                      /* they differ in rounding only                          */
  int32_t fft_split;  /* factorisation G = G1 G2 of the Toeplitz row pass's  */
                      /* team transforms: 0 (default) the grid's own (G1 = 16 */
                      /* for G >= 128), 1 an alternative (the swapped order,  */
                      /* e.g. 20 x 16 at G = 320; 32 x 8 at 256, 16 x 4 at   */
                      /* 64).  The same transform in exact arithmetic; the    */
                      /* faster one is a measurement (autotuner dimension)    */
} nlinv_params;

/* Fill `p` with the defaults above (N, K left 0).  Never fails for non-NULL p. */
int nlinv_params_default(nlinv_params* p);

/* Validate `p` and return the workspace size in bytes.  Host-only: needs no GPU. */
int nlinv_workspace_size(const nlinv_params* p, size_t* bytes);

/* The same call under the name nlinv_plan_workspace_size. */
int nlinv_plan_workspace_size(const nlinv_params* p, size_t* bytes);

/* Derived sizes of a parameter set (host-only).  Any output may be NULL. */
int nlinv_sizes(const nlinv_params* p, int32_t* R, int32_t* G, int32_t* Gc,
                int64_t* S, int64_t* X);

/* Create a plan on the current HIP device.  `stream` is a hipStream_t (NULL =
 * default stream).  `d_workspace` (>= nlinv_workspace_size bytes, 256-byte
 * aligned) is owned by the caller and must stay allocated until
 * nlinv_plan_destroy.  Uploads the FP64-computed tables (twiddles, Sobolev
 * weights) and waits for that upload before returning. */
int nlinv_plan_create(const nlinv_params* p, void* stream, void* d_workspace,
                      size_t ws_bytes, nlinv_plan* out);
int nlinv_plan_destroy(nlinv_plan plan);

/* Admission by device-memory budget (Sec. 3.1: several slices of a real-time
 * pipeline share one GPU).  With budget_bytes > 0, nlinv_plan_create and
 * nlinv_plan_create_static on HIP device `device` (0..63) fail with
 * NLINV_E_BUDGET, before touching the device, when the new plan's workspace
 * (nlinv_workspace_size) plus the workspaces of the live plans on that device
 * would exceed budget_bytes; nlinv_plan_destroy returns a plan's share.
 * budget_bytes = 0 (the default) removes the cap.  Lowering the budget below
 * what is in use affects only later plans.  nlinv_budget_used reports the
 * summed workspace bytes of the live plans on `device`.  Thread-safe; host-only. */
int nlinv_set_budget(int32_t device, size_t budget_bytes);
int nlinv_budget_used(int32_t device, size_t* used_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): a plan
 * exactly like nlinv_plan_create's, whose workspace is the library's static
 * device array of NLINV_STATIC_WORKSPACE_BYTES (128 MiB) instead of a
 * caller buffer.  Each GPU the library runs on holds its own array until the
 * process ends; it is set up on the first call on a device (that device
 * current).  The call allocates no device memory.
 *   - NLINV_E_WORKSPACE: the parameters need more workspace than the array
 *     holds (nlinv_workspace_size > NLINV_STATIC_WORKSPACE_BYTES; e.g. 160 px,
 *     10 coils, 5 turns, batch 1 needs 81 MiB and fits).
 *   - NLINV_E_STATE: another plan on the static workspace of the current
 *     device is still alive (one at a time per GPU; destroy it first).
 * The array keeps the last plan's contents; a new plan rebuilds every table
 * and PSF kernel it uses.  Plans on it launch eagerly: nlinv_set_graphs(1)
 * and nlinv_timer_enable return NLINV_E_STATE.  As for every plan, calls
 * that overlap in time on one plan race; since all static plans of a GPU
 * share one array, so would two of them, which is why only one may live. */
#define NLINV_STATIC_WORKSPACE_BYTES ((size_t)128 << 20)
int nlinv_plan_create_static(const nlinv_params* p, void* stream, nlinv_plan* out);
/* Make `stream` (a hipStream_t; NULL = the null stream) the plan's stream for
 * later calls.  Work already enqueued on the previous stream is not waited
 * for: the caller orders the two streams (an event) before the next call,
 * since every call reuses the plan's workspace. */
int nlinv_set_stream(nlinv_plan plan, void* stream);

/* PSF kernel of one turn (Sec. 2.2 footnote; Fig. flow: convolution with the
 * point-spread function on the twofold oversampled grid).
 * psf(d) = (1/R^2) sum_s exp(+i 2 pi k_s . d) over lags |d_x|,|d_y| <= R-1 (exact sum),
 * P = unnormalised 2D DFT of psf on the G-grid; P is real and is cached in the
 * workspace under `turn` (0 <= turn < U).  d_traj: [K][S_r][2]. */
int nlinv_psf(nlinv_plan plan, const float* d_traj, int32_t turn);
/* (also builds the turn's gridding table: kernels enqueued on the plan's
 * stream, which read d_traj there; the call does not wait for the device.
 * d_traj must stay valid until that work has run.) */

/* The same for a turn acquired with fewer spokes than the plan's K: only the
 * first `spokes` spokes of d_traj [K][S_r][2] count (1 <= spokes <= K,
 * NLINV_E_ARG otherwise); the PSF kernel and the gridding table of `turn`
 * are built from those samples alone, so a series with fewer spokes can
 * share a batched plan.  Its data keep the plan's layout [J][K * S_r] with
 * the spokes beyond `spokes` never read by the table-based gridding
 * (nlinv_grid with turns); the exact sum (no turns, or NLINV_F_EXACT_GRID)
 * reads every sample, so there those samples must be zero.
 * nlinv_psf(plan, d_traj, turn) is nlinv_psf_spokes(plan, d_traj, K, turn). */
int nlinv_psf_spokes(nlinv_plan plan, const float* d_traj, int32_t spokes, int32_t turn);

/* The same for a turn of any smaller acquisition: only the first `samples`
 * samples of d_traj (1 <= samples <= K * S_r, NLINV_E_ARG otherwise) count,
 * so a series with fewer samples per spoke (a smaller image side N' on this
 * plan's grid, gamma = G / (2 N') <= 2, Sec. 3.2) or fewer spokes packs its
 * K' * S_r' samples at the start of the plan's [J][K * S_r] layout and runs
 * in the same batched launch; with zero channels for a smaller coil count its
 * reconstruction equals that of its own plan of grid G bit for bit.  The
 * same zero-sample rule as nlinv_psf_spokes holds for the exact sum. */
int nlinv_psf_samples(nlinv_plan plan, const float* d_traj, int64_t samples, int32_t turn);

/* Gridding (Sec. 3.1, preprocessing): z_j = F^H y_j on the R x R field of view,
 * z_j(r) = (1/R) sum_s y_{j,s} exp(+i 2 pi k_s . r).
 * d_traj [B][K][S_r][2], d_y [B][J][S] -> d_z [B][J][R][R].
 * h_turn == NULL: the exact sum over the samples of d_traj[b].
 * h_turn != NULL (host [B]): item b is sampled on the trajectory of turn
 * h_turn[b].  The PSF kernel and the gridding table of every turn not yet
 * cached are computed from d_traj[b] (as nlinv_psf, enqueued on the stream).
 * Unless the plan has NLINV_F_EXACT_GRID, z is then formed by Kaiser-Bessel
 * gridding (width 9, oversampling G/R = 2; Beatty et al. 2005): gather onto
 * the G x G grid, inverse 2D FFT, crop, deapodise; relative error ~1e-8
 * against the exact sum, below float32 rounding. */
int nlinv_grid(nlinv_plan plan, const float* d_traj, const nlinv_c64* d_y,
               const int32_t* h_turn, nlinv_c64* d_z);

/* NLINV reconstruction (Sec. 2.2: IRGNM, M Newton steps, each solved with C CG
 * iterations on DF^H DF + alpha_n I applied through the PSF convolution).
 *   d_z     [B][J][R][R]  gridded data (nlinv_grid)
 *   h_turn  host [B]      PSF kernel per item (must have been computed)
 *   d_xprev [B][X]        regularisation target x_hat_prev; NULL -> (rho = 1, c = 0)
 *   d_xhat  [B][X]        in: initial guess (init = 0); out: result
 *   init    0: use d_xhat as given; 1: start from (rho = 1, c = 0);
 *           2: start from d_xprev (copied; d_xprev must not be NULL)
 *   d_img   [B][R][R] float32, |rho| sqrt(sum_j |c_j|^2), or NULL
 *   d_coils [B][J][R][R] coil images c_j = W^-1 c_hat_j of the result, or NULL
 * d_xhat must not overlap d_xprev or d_z. */
int nlinv_reconstruct(nlinv_plan plan, const nlinv_c64* d_z, const int32_t* h_turn,
                      const nlinv_c64* d_xprev, nlinv_c64* d_xhat, int32_t init,
                      float* d_img, nlinv_c64* d_coils);

/* Relaxed temporal coupling (Sec. 3.3, temporal decomposition, equation for
 * h(n, m)): reconstruct `count` consecutive frames n0 .. n0+count-1 of one
 * series (1 <= count <= batch) together.
 *   d_z     [count][J][R][R]  gridded data of the frames, in order
 *   h_turn  host [count]      PSF kernel of each frame's turn
 *   d_xprev [X]               result of frame n0-1 (the source frame, the most
 *                             recent finished one); NULL -> (rho = 1, c = 0)
 *   d_xhat  [count][X]        out: results
 *   d_img, d_coils            as nlinv_reconstruct ([count] items), or NULL
 * Newton steps m < M-1 of every frame start from, and are regularised
 * towards, d_xprev; they run as one batch (groups of 2 or 3 frames in the
 * four-pass CG form, not on the static workspace: as one chain per frame on
 * streams the plan creates on first use, forked from and joined back into its
 * stream, with the same results).  Step M-1 of frame n0+k is
 * regularised towards frame n0+k-1 (d_xprev for k = 0) and runs after it, one
 * frame at a time; with M = 1 that step also starts from frame n0+k-1.
 * count = 1 gives the strict per-frame order (nlinv_reconstruct with init =
 * 2, or init = 1 when d_xprev is NULL).  d_xhat must not overlap d_xprev or
 * d_z.  Uses the active-batch setting internally and restores it. */
int nlinv_reconstruct_frames(nlinv_plan plan, int32_t count, const nlinv_c64* d_z,
                             const int32_t* h_turn, const nlinv_c64* d_xprev,
                             nlinv_c64* d_xhat, float* d_img, nlinv_c64* d_coils);

/* Active batch: calls after nlinv_set_batch(plan, b) work on the first b
 * items (1 <= b <= batch); every [B] in this header then means [b].  A plan
 * starts with b = batch.  Lets one plan serve partial batches, e.g. frames
 * that have arrived so far.  nlinv_get_batch returns the setting (0 for a
 * NULL plan). */
int nlinv_set_batch(nlinv_plan plan, int32_t b);
int32_t nlinv_get_batch(nlinv_plan plan);

/* Operators at the linearisation point d_xhat [B][X] (Sec. 2.2), mapping
 * between the unknowns and the radial measurement space [B][J][S]:
 *   F_hat(x)_j    = F(rho . W^-1 c_hat_j)
 *   DF(dx)_j      = F(c_j d_rho + rho W^-1 d_c_hat_j)
 *   DF^H(dy)      = (sum_j conj(c_j) F^H dy_j ; W^-H (conj(rho) F^H dy_j))
 * F is the exact non-uniform DFT (no gridding approximation), so DF and DF^H
 * are adjoint up to float32 rounding. */
int nlinv_apply_F(nlinv_plan plan, const float* d_traj, const nlinv_c64* d_xhat,
                  nlinv_c64* d_y);
int nlinv_apply_DF(nlinv_plan plan, const float* d_traj, const nlinv_c64* d_xhat,
                   const nlinv_c64* d_dx, nlinv_c64* d_dy);
int nlinv_apply_DFH(nlinv_plan plan, const float* d_traj, const nlinv_c64* d_xhat,
                    const nlinv_c64* d_dy, nlinv_c64* d_dx);

/* The CG operator (normal-operator equation and t_j of Sec. 2.2):
 * d_q = DF^H DF d_p + alpha d_p, with F^H F applied as the PSF convolution of
 * turn h_turn[b].  d_xhat, d_p, d_q: [B][X]. */
int nlinv_apply_normal(nlinv_plan plan, const int32_t* h_turn, const nlinv_c64* d_xhat,
                       double alpha, const nlinv_c64* d_p, nlinv_c64* d_q);

/* One frame on each of several plans as one launch (Sec. 3.3, real-time
 * series of different image sides, channel and spoke counts, each on its own
 * plan and grid, without padding to one shape).  The launch sequences
 * nlinv_reconstruct would enqueue for the plans are captured once per argument
 * set into one HIP graph whose branches (one per plan) depend on nothing but
 * the graph's start, and the graph is launched on plans[0]'s stream; the
 * branches may run concurrently.  Each plan's result equals its own
 * nlinv_reconstruct bit for bit.
 *   count        1..NLINV_MAX_MULTI distinct plans, all on one device
 *   d_z[i], h_turn[i], d_xprev[i], d_xhat[i], init[i], d_img[i]
 *                plan i's arguments as nlinv_reconstruct takes them (d_xprev[i]
 *                and d_img[i] may be NULL; no coil-image output); the arrays
 *                themselves are host memory and not kept
 * Everything runs on plans[0]'s stream: work pending on the plans' own
 * streams must be ordered before the call by the caller.  The instantiated
 * graphs are kept per argument set (at most 64 sets in the process, then all
 * are dropped), and those of a plan are dropped when it is destroyed or its
 * coil weights change.  NLINV_E_STATE while a kernel timer is armed on one of
 * the plans or for a plan on the static workspace (those launch eagerly);
 * NLINV_E_ARG for a plan given twice or plans on different devices. */
#define NLINV_MAX_MULTI 8
int nlinv_reconstruct_multi(int32_t count, const nlinv_plan* plans, const nlinv_c64* const* d_z,
                            const int32_t* const* h_turn, const nlinv_c64* const* d_xprev,
                            nlinv_c64* const* d_xhat, const int32_t* init, float* const* d_img);

/* The CG operator of several plans of different grid sides in one go (the
 * same result as nlinv_apply_normal per plan, bit for bit): every plan's
 * passes run on plans[0]'s stream, and the Toeplitz row passes of all of
 * them are one persistent launch whose blocks work through one list of
 * tiles of every shape, each shape on its own grid (mixed image sides
 * without padding to one grid).
 *   count        1..3 plans, of grid sides 256, 320 and 384, at most one each
 *                (NLINV_E_SIZE for other sides), default factorisation,
 *                all on one device; their pending work on other streams must
 *                be ordered before this call by the caller
 *   h_turns[i]   host [B_i] turns of plan i; d_xhat[i], d_p[i], d_q[i] its
 *                [B_i][X_i] point, direction and output (complex64);
 *                alpha[i] host, finite */
int nlinv_apply_normal_multi(int32_t count, const nlinv_plan* plans, const int32_t* const* h_turns,
                             const nlinv_c64* const* d_xhat, const double* alpha, const nlinv_c64* const* d_p,
                             nlinv_c64* const* d_q);

/* The pieces of the IRGNM (Sec. 2.2) in the PSF-convolution form, for the
 * differentiable unrolled reconstruction.  E_x is the image-space part of the
 * derivative, DF_x = F E_x with E_x(p)_j = c_j d_rho + rho W^-1 d_c_hat_j
 * (c_j = W^-1 c_hat_j, rho of the linearisation point x), and T = F^H F the
 * PSF convolution of each item's turn.  Vectors in the unknowns' space are
 * complex128 ([B][X], interleaved double re, im); linearisation points x are
 * complex64 as everywhere; images [B][J][R][R] complex64.
 *   nlinv_apply_normal2: q = E_xa^H T E_xb p + alpha p (= DF_xa^H DF_xb p + alpha p;
 *                        xa = xb gives the CG operator of the normal-operator
 *                        equation; xa != xb the terms of its derivative in x).
 *   nlinv_apply_E:       img = E_x p.
 *   nlinv_apply_EH:      out = E_x^H img = (sum_j conj(c_j) img_j ; W^-H(conj(rho) img_j)).
 *   nlinv_nudft:         y = F img per channel, the exact non-uniform DFT (the
 *                        adjoint of the exact gridding nlinv_grid without turns);
 *                        R <= 256 (NLINV_E_SIZE otherwise). */
int nlinv_apply_normal2(nlinv_plan plan, const int32_t* h_turn, const nlinv_c64* d_xa, const nlinv_c64* d_xb,
                        double alpha, const double* d_p, double* d_q);
int nlinv_apply_E(nlinv_plan plan, const nlinv_c64* d_xhat, const double* d_p, nlinv_c64* d_img);
int nlinv_apply_EH(nlinv_plan plan, const nlinv_c64* d_xhat, const nlinv_c64* d_img, double* d_out);
int nlinv_nudft(nlinv_plan plan, const float* d_traj, const nlinv_c64* d_img, nlinv_c64* d_y);

/* One IRGNM update (Sec. 2.2, the update equation) with a given alpha and CG
 * count: d_xhat <- d_xhat + h, h from `cg` CG iterations (1 <= cg <= 100000)
 * from h = 0 on (DF^H DF + alpha) h = DF^H (y - F_hat(x_hat)) - alpha (x_hat -
 * x_prev), with the solver's own kernels (the plan's cg_passes form, FP64 CG
 * vectors and scalars).  d_z [B][J][R][R] gridded data, h_turn host [B] PSF
 * kernel per item, d_xprev [B][X] or NULL for (rho = 1, c = 0), d_xhat [B][X]
 * in/out (must not alias d_xprev); alpha finite and >= 0.  A step of
 * nlinv_reconstruct is this call with alpha_n and the plan's cg.  It serves
 * the forward pass of the differentiable unrolled reconstruction. */
int nlinv_newton_step(nlinv_plan plan, const int32_t* h_turn, const nlinv_c64* d_z, const nlinv_c64* d_xprev,
                      double alpha, int32_t cg, nlinv_c64* d_xhat);

/* Another Sobolev weight for every later call of this plan (Sec. 3.2, Fig.
 * weight_func: the weight is a choice).  d_winv: device [G_c][G_c] float32
 * table of 1 / (G w'(kappa)) in the layout of one coil spectrum block of
 * x_hat (centred kappa, kappa_y major); the plan's own table holds
 * 1 / (G (1 + sob_a |kappa/G|^2)^sob_l).  The caller owns d_winv and keeps it
 * valid and unchanged while it is set; NULL restores the plan's own table.
 * Captured HIP graphs of the plan are dropped when the table changes. */
int nlinv_set_coil_weights(nlinv_plan plan, const float* d_winv);

/* Channel compression (Sec. 3.1, preprocessing): virtual channels
 * d_y[b][j][s] = sum_p d_cc[j][p] d_yp[b][p][s] of the J_phys receive channels.
 *   d_cc [J][J_phys] (J of the plan), d_yp [B][J_phys][S], d_y [B][J][S];
 *   1 <= J_phys <= 128.  FP64 sums. */
int nlinv_compress(nlinv_plan plan, const nlinv_c64* d_cc, int32_t J_phys,
                   const nlinv_c64* d_yp, nlinv_c64* d_y);

/* Calibration of the compression (Sec. 3.1): d_cc [J][J_phys] gets, as rows,
 * the conjugated eigenvectors of the channel covariance y0 y0^H of one frame
 * d_y0 [J_phys][S] for its J largest eigenvalues (principal components; each
 * row is defined up to a phase).  The covariance is formed on the GPU in
 * FP64 and the Hermitian eigenproblem (J_phys x J_phys) solved there by
 * parallel cyclic Jacobi rotations in one block; the call only enqueues
 * (d_y0 must stay valid until the work has run).  J <= J_phys <= 128. */
int nlinv_compression_matrix(nlinv_plan plan, const nlinv_c64* d_y0, int32_t J_phys, nlinv_c64* d_cc);

/* Adjoint of the coil synthesis c_j = W^-1 c_hat_j (Sec. 2.2, Sec. 3.2):
 * d_xhat [B][X] gets the image block 0 and the coil blocks
 * W^-H c_j = D_W^-1 crop_{G_c} F_u pad_G c_j of d_coils [B][J][R][R].
 * Used as the backward pass of nlinv_coils in the differentiation form. */
int nlinv_apply_WH(nlinv_plan plan, const nlinv_c64* d_coils, nlinv_c64* d_xhat);

/* Coil images c_j = W^-1 c_hat_j [B][J][R][R] and/or the combined image
 * |rho| sqrt(sum_j |c_j|^2) [B][R][R] of d_xhat; either output may be NULL. */
int nlinv_coils(nlinv_plan plan, const nlinv_c64* d_xhat, nlinv_c64* d_coils, float* d_img);

/* HIP graphs for nlinv_reconstruct (default off).  When enabled, the launch
 * sequence of a reconstruction is captured once per distinct argument set
 * (pointers, turns, init, outputs; up to 64 cached, then the cache is
 * cleared) on an internal stream and replayed on the plan's stream, which
 * removes the per-kernel host launch cost.  Results are identical to the
 * uncaptured path.  Ignored while the kernel timer is enabled. */
int nlinv_set_graphs(nlinv_plan plan, int32_t enable);

/* Block until all work enqueued on the plan's stream has finished. */
int nlinv_sync(nlinv_plan plan);

/* Description of the last error on `plan` (or of the last plan-less error
 * when plan == NULL).  Never NULL. */
const char* nlinv_last_error(nlinv_plan plan);

/* Kernel timing for roofline measurement: while enabled, every launch of
 * kernel class `kernel_id` (NLINV_KT_*) on the plan stream is timed with HIP
 * events.  The classes of one kernel per launch carry the events in the
 * kernel's own dispatch (hipExtLaunchKernel), which times the kernel alone;
 * NLINV_KT_GRID (several kernels) has them recorded around the call.
 * nlinv_timer_read waits for the stream, returns the summed duration (ms) and
 * launch count since the last read, and resets them. */
enum { NLINV_KT_NONE = 0, NLINV_KT_TOEPLITZ_ROWS = 1, NLINV_KT_COIL_COLS = 2,
       NLINV_KT_BACK_COLS = 3, NLINV_KT_CG_UPDATE = 4, NLINV_KT_COIL_ROWS = 5,
       NLINV_KT_COILH_ROWS = 6, NLINV_KT_GRID = 7 };
int nlinv_timer_enable(nlinv_plan plan, int32_t kernel_id);
int nlinv_timer_read(nlinv_plan plan, double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* NLINV_H */
