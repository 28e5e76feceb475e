// Internal interface between the C-ABI (nlinv_abi.cpp) and the HIP kernel
// launchers.  Not part of the public API.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <math.h>
#include <stdint.h>

namespace nlv {

constexpr int ROWS = 8;       // lines per block in the row (x) passes
constexpr int TW = 8;         // columns per block in the column (y) passes (8 x 16 B = 128 B)
constexpr int CHUNK = 512;    // vector elements per block in the CG kernels
constexpr int RHOQ_E = 1;     // rho-block elements per thread of the q_rho blocks of the coil-adjoint rows
                              // (one: the channel sums of 64 pixels per wave, many short waves)
constexpr int VT = 256;       // threads per block in the vector / NUDFT kernels
constexpr int MAXB = 64;      // largest batch (turn table passed by value)
constexpr int KB_SHORT = 16;  // gridding rows up to this length take one thread
constexpr int KB_LONG_BLOCKS = 256;  // blocks per item of the long-row gridding kernels (grid-stride)

// Kaiser-Bessel gridding kernel (Beatty, Nishimura, Pauly 2005): width W grid
// cells at oversampling G / R = 2, shape beta = pi sqrt((W/2)^2 (2 - 1/2)^2 - 0.8).
// The same functions run on the host (deapodisation) and on the device (tables).
constexpr int KB_W = 9;
constexpr int KB_TAPS = KB_W + 1;   // grid points a sample can reach per axis

__host__ __device__ inline double kb_bessel_i0(double x) {   // sum_k ((x/2)^k / k!)^2
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 200; ++k) {
    term *= q / ((double)k * k);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

__host__ __device__ inline double kb_beta() {
  const double sigma = 2.0, hw = KB_W / sigma;
  return M_PI * sqrt(hw * hw * (sigma - 0.5) * (sigma - 0.5) - 0.8);
}

// kernel value at distance d (grid cells), normalised to 1 at d = 0
__host__ __device__ inline double kb_phi(double d, double beta) {
  const double t = 1.0 - (2.0 * d / KB_W) * (2.0 * d / KB_W);
  return t < 0.0 ? 0.0 : kb_bessel_i0(beta * sqrt(t)) / kb_bessel_i0(beta);
}

struct TurnArgs { int32_t t[MAXB]; };

// FP64 partial sums of one scalar, per batch item: p[b * stride + slot].
struct Partials {
  const double* cur;  int ncur;    // partials of rr_i = <r_i, r_i>
  const double* prev; int nprev;   // partials of rr_{i-1}
  int stride;
};

// Scalars of the four-pass CG iteration, reduced by one extra block per item
// of the column pass back: scal[b] = (Re<p, q>, rr) with
// Re<p, q> = sum of the Toeplitz partials (||DF p||^2) + alpha * sum of the
// direction partials (|p|^2) and rr = sum of the residual partials.
struct CGRed {
  double2* scal;                      // [B]; nullptr: no reduction
  const double* dfp; int ndfp, sdfp;  // Toeplitz-pass partials, count and stride per item
  const double* pp; int npp, spp;     // direction partials
  const double* rr; int nrr, srr;     // residual partials
  double alpha;
  int nbase;                          // blocks of the pass itself; block nbase + b reduces item b
};

// Sizes shared by all launches of a plan.
struct Shape {
  int B, J, G, R, GC, S, U;
  long long X;         // unknowns per item
  int NT;              // column tiles per channel (R / TW)
  int NX3;             // coil row blocks per item (ceil(J * GC / row_lines))
  int NRQ;             // q_rho blocks per item of the coil-adjoint rows (ceil(R*R / (64 * RHOQ_E)))
  int NCH;             // vector chunks (ceil(X / CHUNK))
  int stride;          // partial slots per item
  int gsplit;          // sample-range split of the gridding kernel (1 = none)
  bool kb;             // Kaiser-Bessel gridding tables present
  long long kbe_stride;  // table entries per turn
  int coltile;         // tile schedule of cols_fwd / cols_back: 0 (the library's), 4 or 8
  int NTB;             // Toeplitz-pass blocks per item of the four-pass CG (ceil(J G / row_lines))
  int NPP;             // direction-partial slots per item (J * R: one per channel and column)
  int split;           // factorisation of the Toeplitz row pass: 0 the grid's default, 1 its alternative
};

// Columns per block of a CG column pass (the plan's tile schedule; the
// library's choice is TW for both passes).  Four columns per block double
// the blocks of launches too small to fill the GPU; measured at 160 px they
// speed up the forward pass of a batch-1 launch alone, yet the whole solve
// runs slower (plain series 164.8 against 166.9 frames/s with four columns in
// the forward pass of small launches only; with the four-pass CG iteration
// 190.3 against 198.3, and 176.7 with four columns in both passes), so four
// is a schedule to measure, not a default.
inline int col_tile(const Shape& s, bool /*forward*/) { return s.coltile == 4 ? 4 : TW; }

// Gridding work decomposition (channels per block; sample-range split).
int grid_jg(int J);
int grid_nsplit(int B, int J, int R);

// Timing of one launch by the kernel timer: when `start` is set, the next
// single-kernel launch carries the two events in its own dispatch
// (hipExtLaunchKernel), so they time the kernel without the cost of
// separately recorded events, and marks `attached`.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
  bool attached = false;
};

// Device buffers carved from the caller's workspace.
struct Bufs {
  double2* tw;    // [G] twiddles (cos, sin)(2 pi m / G)
  float* dinv;    // [GC][GC] 1 / (G w(kappa))
  float* P;       // [U][G][G] PSF kernel / (G^2 R^2), natural DFT order
  double2* psf;   // [G][G] scratch for the PSF build
  float2* CO;     // [B][J][R][R] coil images c_j
  double2* U1;    // [B][J][GC][R] coil-spectrum lines (also the adjoint output)
  void* U2;       // [B][J][G][R] half-transformed grid (double2)
  float2* PR;     // [B][J][R][R] per-channel conj(c_j) t_j
  float2* IMG;    // [B][J][R][R] image-space scratch
  float2* GS;     // [gsplit][B][J][R][R] partial gridding sums (gsplit > 1 only)
  double2* H;     // [B][X] CG iterate increment h
  double2* Rv;    // [B][X] CG residual r
  double2* Pv[2]; // [B][X] CG directions p (ping-pong)
  double2* Q;     // [B][X] operator output (coil block)
  double* pq;     // [B][stride]
  double* rr[2];  // [B][stride] ping-pong
  int* kbr;       // [U][G*G+1] gridding table row starts (per grid point)
  int2* kbe;      // [U][kbe_stride] (sample index, weight bits) per table entry
  int* kbp;       // [U][G*G] grid points: short rows from the front, long rows from the back
  int2* kbn;      // [U] (short, long) point counts
  int2* kbs;      // [kbe_stride] staging of one turn's entries while its table is built
  int* kbq;       // [G*G] per-point fill cursors while a table is built
  float* kbc;     // [R] 1 / (sqrt(R) c(x)), deapodisation per axis
  float2* KG;     // [B][J][G][G] gridded samples
  double2* cov;   // [2][MAX_JP][MAX_JP] channel covariance and its eigenvectors (compression calibration)
  double2* Vr;    // [B][J][GC][R] x-stage of W^-1 applied to the residual's coil block
  double2* Vp;    // [B][J][GC][R] the same for the CG direction (carried by linearity)
  double* pdfp;   // [B][NTB] Toeplitz-pass partials ||DF p||^2
  double* ppp;    // [B][NPP] direction partials |p|^2
  double2* scal;  // [B] (Re<p, q>, rr) of the current CG iteration
  LaunchTiming* lt = nullptr;   // the plan's kernel-timer hook (host memory)
};

// Launch one kernel; with the timer hook armed, the hook's events are
// attached to this dispatch.
template <class... KArgs, class... Args>
inline hipError_t launch_timed(const Bufs& w, void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t shm,
                               hipStream_t st, Args... args) {
  if (w.lt && w.lt->start) {
    hipExtLaunchKernelGGL(kernel, grid, block, shm, st, w.lt->start, w.lt->stop, 0u, args...);
    w.lt->attached = true;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
  }
  return hipGetLastError();
}

// Grid-size specific launchers (one table per supported G).
struct GTable {
  // coil spectra of the float32 unknowns -> U1 (W^-1 along x)
  hipError_t (*coil_rows)(const Shape&, const Bufs&, hipStream_t, const float2* src);
  // same on a float64 CG direction; with rsrc != nullptr the update p = r + beta p_old
  // is fused (src = p_old, the whole new direction, rho block included, written to pdst)
  hipError_t (*coil_rows_cg)(const Shape&, const Bufs&, hipStream_t, const double2* src,
                             const double2* rsrc, double2* pdst, Partials sc);
  // column pass on U1.  mode 0: coils c_j -> co, u = rho c_j -> U2 (out may be null)
  // mode 1: u = c_j d_rho + rho d_c_j -> U2; mode 2: coils -> co, u = rho c_j -> out (image)
  // mode 3: u = c_j d_rho + rho d_c_j -> out (image).  pv: float64 direction (modes 1, 3).
  hipError_t (*cols_fwd)(const Shape&, const Bufs&, hipStream_t, int mode, float2* co, const float2* xh,
                         const double2* pv, void* out);
  // row pass: FFT, multiply by the PSF kernel of each item's turn, inverse FFT (in place on U2)
  hipError_t (*toep_rows)(const Shape&, const Bufs&, hipStream_t, const TurnArgs& turns);
  // column pass back: mode 0 normal, 1 residual (z - T u), 2 adjoint of an image-space
  // float32 input, 3 plain W^-H column stage of coil images.  Writes U1 (as the W^-H column
  // stage) and, except in mode 3, PR.
  hipError_t (*cols_back)(const Shape&, const Bufs&, hipStream_t, int mode, const void* in,
                          const float2* co, const float2* xh, const float2* z);
  // row pass: W^-H along x.  mode 0: q = W^-H(..) + alpha p -> out, and NRQ further blocks
  // per item form the image block q_rho = sum_j PR_j + alpha p_rho -> out (pq partials of
  // Re<p, q>: line blocks at slots [0, NX3), q_rho blocks at [NX3, NX3 + NRQ))
  // mode 1: b = W^-H(..) - alpha (x - xprev) -> out and out2 (rr[0] partials at slot 0)
  // mode 2: raw W^-H -> out.
  hipError_t (*coilh_rows)(const Shape&, const Bufs&, hipStream_t, int mode, const double2* pv,
                           const float2* xh, const float2* xprev, double alpha, double2* out,
                           double2* out2);
  // four-pass CG iteration (see nlinv_kernels.h): direction update and forward column
  // pass (Pold -> Pnew, Vr/Vp -> U2, direction partials); the Toeplitz row pass with
  // the Parseval partials; the column pass back (mode 0) with the scalar reduction;
  // the coil-adjoint rows with the CG vector updates (x += h on the last iteration)
  hipError_t (*cg_cols_fwd)(const Shape&, const Bufs&, hipStream_t, const float2* xh, const double2* pold,
                            double2* pnew, Partials sc, int first);
  hipError_t (*cg_toep_rows)(const Shape&, const Bufs&, hipStream_t, const TurnArgs& turns);
  hipError_t (*cg_cols_back)(const Shape&, const Bufs&, hipStream_t, const float2* xh, const CGRed& red);
  hipError_t (*cg_coilh)(const Shape&, const Bufs&, hipStream_t, const double2* pnew, float2* xh, double alpha,
                         double* rr_next, int first, int last);
  // PSF kernel: 2D FFT of the embedded PSF (w.psf) -> P (real part x scale)
  hipError_t (*psf_fft)(const Shape&, const Bufs&, hipStream_t, float* P, double scale);
  // Kaiser-Bessel gridding of y [B][J][S] into z [B][J][R][R] with the turn tables
  hipError_t (*kb_grid)(const Shape&, const Bufs&, hipStream_t, const TurnArgs& turns, const float2* y,
                        float2* z);
  int row_lines;   // lines per block of the coil row passes
  int row_lines_split;   // lines per block of the Toeplitz row pass under the alternative factorisation
};

// Table for grid size G, or nullptr if unsupported.
const GTable* table_for(int G);

// Grid-size independent launchers.
hipError_t launch_cg_update(const Shape& s, const Bufs& w, hipStream_t st, int iter, int last,
                            const double2* p, Partials rr, float2* xh);
// out (float32 [B][X]) = (sum_j PR_j + alpha p ; Q) ; p may be null; without the image
// block (image_block false) the image part is alpha p, or zero when p is null
hipError_t launch_finalize(const Shape& s, const Bufs& w, hipStream_t st, const double2* p,
                           double alpha, float2* out, bool image_block = true);
hipError_t launch_finalize(const Shape& s, const Bufs& w, hipStream_t st, const double2* p,
                           double alpha, double2* out, bool image_block = true);
hipError_t launch_to_double(const Shape& s, hipStream_t st, double2* dst, const float2* src);
// mode 1: (rho = 1, c = 0); 2: copy xprev [B][X]; 3: broadcast xprev [X] to every item
hipError_t launch_init_x(const Shape& s, hipStream_t st, float2* xh, const float2* xprev, int mode);
hipError_t launch_image(const Shape& s, hipStream_t st, const float2* xh, const float2* co, float* img);
hipError_t launch_grid(const Shape& s, const Bufs& w, hipStream_t st, const float* traj, const float2* y,
                       float2* z);
hipError_t launch_nudft_fwd(const Shape& s, hipStream_t st, const float* traj, const float2* u,
                            float2* y);
// PSF kernel of `turn` from the first S samples of traj (S <= s.S)
hipError_t launch_psf(const Shape& s, const Bufs& w, hipStream_t st, const float* traj, int S, int turn);
hipError_t launch_kb_table(const Shape& s, const Bufs& w, hipStream_t st, const float* traj, int S, int turn);
// One shape of a ragged Toeplitz row pass: a plan's half-transformed grid,
// PSF kernels, twiddles and turns, and its J and line count (B J G).
struct ToepShape {
  double2* U2;
  const float* P;
  const double2* tw;
  TurnArgs turns;
  int J, nlines;
};
hipError_t launch_toep_ragged(hipStream_t st, const ToepShape (&shapes)[3]);
// channel compression y [B][J][S] = cc [J][Jp] x yp [B][Jp][S]; covariance of one frame [Jp][S]
constexpr int MAX_JP = 128;
hipError_t launch_compress(const Shape& s, hipStream_t st, const float2* cc, int Jp, const float2* yp, float2* y);
hipError_t launch_channel_cov(const Shape& s, hipStream_t st, const float2* y0, int Jp, double2* cov);
hipError_t launch_compression_eig(hipStream_t st, double2* A, double2* V, int n, int J, float2* cc);

}  // namespace nlv
