// HIP kernels of the NLINV hot path for gfx950 (MI355X), templated on the grid size.
//
// The CG operator q = (DF^H DF + alpha) p of the normal-operator equation
// (Sec. 2.2) is applied per channel j as
//     d_c_j = W^-1 d_c_hat_j            (coil synthesis: weight, pad, iFFT, crop)
//     u_j   = c_j d_rho + rho d_c_j     (derivative of the coil product)
//     t_j   = F^H F u_j                 (PSF convolution: pad, FFT, x P, iFFT, crop)
//     q_rho = sum_j conj(c_j) t_j + alpha d_rho,   q_c_hat_j = W^-H(conj(rho) t_j) + alpha d_c_hat_j
// with every 2D FFT split into a row (x) and a column (y) pass and the
// pointwise steps fused into the pass that holds the data in registers:
//     coil_rows : direction update p = r + beta p, x-iFFT of the
//                 (weighted) coil spectra                           G_c rows  -> U1
//     cols_fwd  : y-iFFT -> u_j -> y-FFT                            R columns -> U2
//     toep_rows : x-FFT -> x P -> x-iFFT (in place)                 G rows
//     cols_back : y-iFFT -> conj(c_j) t_j, conj(rho) t_j -> y-FFT   R columns -> PR, U1
//     coilh_rows: x-FFT -> x weight (+ alpha p); channel sum of the
//                 image block; <p, q> partials                     G_c rows, R^2 pixels -> Q
//     cg_update : CG scalars, h and r updates
// Zero padding and cropping are never materialised: absent inputs are not
// loaded and unwanted outputs are not stored.
//
// Precision: the transforms run in float64 registers and float64 LDS; the
// half-transformed grid U2 and the small coil-row buffer U1 are stored in
// float64, the coil images and the per-channel products in float32.  CG
// iterates are far more sensitive to rounding that differs from one operator
// application to the next than to a fixed error of the operator, so the CG
// state (h, r, p, q) is float64 too.
// CG scalars stay on the device as FP64 partial sums reduced in a fixed order
// (deterministic, no atomics).
#pragma once

#include "nlinv_fft.h"
#include "nlinv_internal.h"

namespace nlv {

using C = double2;   // arithmetic type of every transform

// Blocks are padded to whole wavefronts; padding threads take part in barriers
// and reductions only (their team lane is set past the last real lane).
constexpr int pad64(int n) { return (n + 63) / 64 * 64; }
template <int G> constexpr int rows_threads() { return pad64(ROWS * Team<G>::SIZE); }
// Row passes of the solver run one wavefront per block: 64 / SIZE lines (3 at
// G = 320), so the exchanges synchronise a single wave and many small blocks
// share a CU (measured: Toeplitz pass 15 % faster than 8-line blocks).
template <int G> constexpr int row_lines() { return 64 / Team<G>::SIZE > 0 ? 64 / Team<G>::SIZE : 1; }
template <int G> constexpr int row_threads() { return pad64(row_lines<G>() * Team<G>::SIZE); }
template <int G, int TWC = TW> constexpr int cols_threads() { return pad64(TWC * Team<G>::SIZE); }

// ---------------------------------------------------------------------------
// reductions (FP64, fixed order, valid for blocks that are not whole waves)
// ---------------------------------------------------------------------------

constexpr int pow2_ceil(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Sum over the block; the result is returned to every thread.  sh: [NT] doubles.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  __syncthreads();   // sh may still be read by a previous call
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = pow2_ceil(NT) / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && (int)threadIdx.x + s < NT) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// Sum of p[0..n), returned to every thread.
template <int NT>
__device__ __forceinline__ double block_sum_array(const double* __restrict__ p, int n, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s += p[i];
  return block_sum<NT>(s, sh);
}

// Same for blocks made of whole wavefronts (NT a multiple of 64): shuffle within
// each wave, then every thread adds the per-wave sums in the same order.
template <int NT>
__device__ __forceinline__ double block_sum_waves(double v, double* sh) {
  static_assert(NT % 64 == 0, "whole wavefronts only");
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NT / 64; ++i) s += sh[i];
  return s;
}

// s += p[i0], p[i0 + NT], ... (i < n) in that order, the loads of 8 terms issued
// together so that their latencies overlap
template <int NT>
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int i0, int n) {
  constexpr int U = 8;
  double s = 0.0;
  for (int i = i0; i < n; i += NT * U) {
    double v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) v[k] = i + NT * k < n ? p[i + NT * k] : 0.0;
#pragma unroll
    for (int k = 0; k < U; ++k) s += v[k];
  }
  return s;
}

template <int NT>
__device__ __forceinline__ double block_sum_array_waves(const double* __restrict__ p, int n, double* sh) {
  return block_sum_waves<NT>(strided_sum<NT>(p, threadIdx.x, n), sh);
}

// Two block sums with one pair of barriers; sh holds at least 2 NT / 64 values.
// Each sum is formed in the same order as block_sum_waves would form it.
template <int NT>
__device__ __forceinline__ double2 block_sum2_waves(double u, double v, double* sh) {
  static_assert(NT % 64 == 0, "whole wavefronts only");
  constexpr int NW = NT / 64;
  for (int off = 32; off > 0; off >>= 1) {
    u += __shfl_down(u, off, 64);
    v += __shfl_down(v, off, 64);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6] = u;
    sh[NW + (threadIdx.x >> 6)] = v;
  }
  __syncthreads();
  double su = 0.0, sv = 0.0;
  for (int i = 0; i < NW; ++i) su += sh[i];
  for (int i = 0; i < NW; ++i) sv += sh[NW + i];
  return make_double2(su, sv);
}

// Sums of two partial arrays; all loads are issued before the reduction.
template <int NT>
__device__ __forceinline__ double2 block_sum2_arrays_waves(const double* __restrict__ p, int n,
                                                           const double* __restrict__ q, int m, double* sh) {
  return block_sum2_waves<NT>(strided_sum<NT>(p, threadIdx.x, n), strided_sum<NT>(q, threadIdx.x, m), sh);
}

// Sums of two partial arrays by the first wavefront of the block, broadcast to
// every thread through sh[0..1]: the same order whatever the block size, so
// that launches of different tile schedules reduce to the same bits.
__device__ __forceinline__ double2 wave0_sum2_arrays(const double* __restrict__ p, int n,
                                                     const double* __restrict__ q, int m, double* sh) {
  __syncthreads();   // sh may still be read by a previous call
  if (threadIdx.x < 64) {
    double s = strided_sum<64>(p, threadIdx.x, n), t = strided_sum<64>(q, threadIdx.x, m);
    for (int off = 32; off > 0; off >>= 1) {
      s += __shfl_down(s, off, 64);
      t += __shfl_down(t, off, 64);
    }
    if (threadIdx.x == 0) {
      sh[0] = s;
      sh[1] = t;
    }
  }
  __syncthreads();
  return make_double2(sh[0], sh[1]);
}

// partial sums per lane that a pass loads up front for beta (the rest, if
// any, in a loop after them)
constexpr int BETA_PRE = 12;

__device__ __forceinline__ double beta_wave0(const Partials& sc, int b, double* sh) {
  const double2 r = wave0_sum2_arrays(sc.cur + (size_t)b * sc.stride, sc.ncur, sc.prev + (size_t)b * sc.stride,
                                      sc.nprev, sh);
  return r.y != 0.0 ? r.x / r.y : 0.0;
}

template <int NT>
__device__ __forceinline__ double beta_of(const Partials& sc, int b, double* sh) {
  const double2 r = block_sum2_arrays_waves<NT>(sc.cur + (size_t)b * sc.stride, sc.ncur,
                                                sc.prev + (size_t)b * sc.stride, sc.nprev, sh);
  return r.y != 0.0 ? r.x / r.y : 0.0;
}


// Non-temporal access to the half-transformed grid U2 (the largest buffer: it
// is written once and read once per pass).  Keeping it out of the caches
// leaves them to the CG vectors, channel products and coil rows.  Measured
// on the whole solve: plain 158 -> 167 frames/s, batch 16 458 -> 480, although
// the Toeplitz pass alone gets slower (it no longer finds U2 cached).
template <class S2> struct NV;
template <> struct NV<double2> { typedef double T __attribute__((ext_vector_type(2))); };
template <> struct NV<float2> { typedef float T __attribute__((ext_vector_type(2))); };
template <class S2> __device__ __forceinline__ S2 nt_load(const S2* p) {
  using V = typename NV<S2>::T;
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  S2 o;
  o.x = v.x;
  o.y = v.y;
  return o;
}
template <class S2> __device__ __forceinline__ void nt_store(S2* p, S2 v) {
  using V = typename NV<S2>::T;
  V w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<V*>(p));
}

// ---------------------------------------------------------------------------
// coil_rows: W^-1 along x.  Line (b, j, i): G_c weighted coil coefficients of
// spectrum row i -> R image columns.  Optional fused p = r + beta p_old; the
// rho block of the direction is updated by nr further blocks per item, so the
// whole new direction is in pdst before the column pass reads it.
// ---------------------------------------------------------------------------
constexpr int RHO_PER_THREAD = 8;   // rho-block elements per thread of the update blocks

template <int G, class V>
__global__ void __launch_bounds__(row_threads<G>())
k_coil_rows(const V* __restrict__ src, const double2* __restrict__ rsrc, double2* __restrict__ pdst,
            Partials sc, const float* __restrict__ dinv, const double2* __restrict__ tw,
            double2* __restrict__ U1, int J, long long X, int nb, int nr) {
  using T = Team<G>;
  constexpr int R = G / 2, GC = G / 4, NTH = row_threads<G>(), RT = row_lines<G>();
  __shared__ C lds[RT * T::LDSN];
  __shared__ double sh[NTH];
  // nb line blocks then nr rho-update blocks per item, each line block RT of
  // the item's J * GC lines
  const int b = blockIdx.x / (nb + nr), chunk = blockIdx.x - b * (nb + nr);
  if constexpr (std::is_same<V, double2>::value) {
    if (chunk >= nb) {   // block-uniform
      constexpr int E = RHO_PER_THREAD;
      const double2* ps = src + (size_t)b * X;
      const double2* rs = rsrc + (size_t)b * X;
      double2* pd = pdst + (size_t)b * X;
      const int e0 = (chunk - nb) * NTH * E + (int)threadIdx.x;
      double2 po[E], ro[E];
      sfor<0, E>([&](auto c) {
        constexpr int k = decltype(c)::value;
        const int e = e0 + k * NTH;
        if (e < R * R) {
          po[k] = ps[e];
          ro[k] = rs[e];
        }
      });
      const double beta = beta_of<NTH>(sc, b, sh);
      sfor<0, E>([&](auto c) {
        constexpr int k = decltype(c)::value;
        const int e = e0 + k * NTH;
        if (e < R * R) pd[e] = make_double2(ro[k].x + beta * po[k].x, ro[k].y + beta * po[k].y);
      });
      return;
    }
  }
  const int rl0 = (int)threadIdx.x / T::SIZE, l0 = chunk * RT + rl0;
  const bool act = rl0 < RT && l0 < J * GC;
  const int tl = act ? (int)threadIdx.x % T::SIZE : T::SIZE, rl = act ? rl0 : 0;
  const int l = act ? l0 : 0;
  const int i = l % GC, j = l / GC, bj = b * J + j;
  const bool upd = rsrc != nullptr;
  const size_t off = (size_t)b * X + (size_t)R * R + ((size_t)j * GC + i) * GC;
  const float* dw = dinv + i * GC;
  // the element loads are issued before the scalar reduction, so that both
  // memory round trips overlap
  C a[T::G2], ra[T::G2];
  float wv[T::G2];
  if (tl < T::G1) {
    sfor<0, T::G2>([&](auto c) {
      constexpr int n2 = decltype(c)::value;
      a[n2] = czero<C>();
      if constexpr (cls_n<G, SET_COIL, n2>() != NEVER) {
        const int ic = coil_idx<G>(tl + T::G1 * n2);
        if (ic >= 0) {
          a[n2] = to_d(src[off + ic]);
          if (upd) ra[n2] = rsrc[off + ic];
          wv[n2] = dw[ic];
        }
      }
    });
  }
  const double beta = upd ? beta_of<NTH>(sc, b, sh) : 0.0;
  if (tl < T::G1) {
    sfor<0, T::G2>([&](auto c) {
      constexpr int n2 = decltype(c)::value;
      if constexpr (cls_n<G, SET_COIL, n2>() != NEVER) {
        const int ic = coil_idx<G>(tl + T::G1 * n2);
        if (ic >= 0) {
          double2 p = a[n2];
          if (upd) {
            p = make_double2(ra[n2].x + beta * p.x, ra[n2].y + beta * p.y);
            pdst[off + ic] = p;
          }
          a[n2] = cscale(p, (double)wv[n2]);
        }
      }
    });
  }
  C v[T::G1];
  fsA_regs<G, +1, SET_IMG>(tl, lds + rl * T::LDSN, tw, a, v);
  if (tl < T::G2) {
    double2* o = U1 + ((size_t)bj * GC + i) * R;
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      const int ix = img_idx<G>(T::G2 * k1 + tl);
      if (ix >= 0) o[ix] = v[k1];
    });
  }
}

// ---------------------------------------------------------------------------
// cols_fwd: W^-1 along y, coil product, forward FFT along y.
// MODE 0: coils -> co, u = rho c_j -> out (U2, may be null)
// MODE 1: u = c_j d_rho + rho d_c_j -> out (U2);  MODE 2 / 3: as 0 / 1 but u -> out (image, float32)
// pv: the direction (MODE 1 / 3), its rho block already updated by coil_rows.
// ---------------------------------------------------------------------------
// Block order of the column passes.  The blocks of a launch are dealt to the
// eight XCDs in turn (block i to XCD i mod 8), each with its own L2.  While
// the launch's half-transformed grid fits in the 256 MB Infinity Cache, block
// i takes the work item w(i) with the channel fastest, each XCD working
// through a contiguous run of work items: the J channel blocks of one column
// tile run on one XCD at about the same time and share its cached rho and
// direction columns.  Larger launches keep the plain order (tile fastest),
// whose eight XCDs advance through neighbouring columns.  Measured, one plan
// of the 160 px series, frames/s with the channel-fastest order against the
// plain one: batch 8 448 / 434, batch 16 535 / 513, batch 32 491 / 492,
// batch 64 487 / 500.
constexpr size_t INFINITY_CACHE_BYTES = size_t(256) << 20;
template <int G, int TWC>
__device__ __forceinline__ void col_order(int i, int n, int J, int& bj, int& tile) {
  constexpr int NT = G / 2 / TWC, NX = 8;
  if ((size_t)n * TWC * G * sizeof(double2) > INFINITY_CACHE_BYTES) {
    tile = i % NT;
    bj = i / NT;
    return;
  }
  const int k = i % NX, q = n / NX, r = n % NX;
  const int w = k * q + (k < r ? k : r) + i / NX;
  const int j = w % J, bt = w / J;
  tile = bt % NT;
  bj = (bt / NT) * J + j;
}

template <int G, int TWC, int MODE, class S2>
__global__ void __launch_bounds__((cols_threads<G, TWC>()))
k_cols_fwd(const double2* __restrict__ U1, float2* __restrict__ co, const float2* __restrict__ xh,
           const double2* __restrict__ pv, const double2* __restrict__ tw, void* __restrict__ outp, int J,
           long long X) {
  using T = Team<G>;
  constexpr int R = G / 2, GC = G / 4, NT = R / TWC;
  constexpr bool NORMAL = (MODE == 1 || MODE == 3);
  constexpr bool TO_IMG = (MODE == 2 || MODE == 3);
  __shared__ C lds[TWC * T::LDSC];
  const bool act = (int)threadIdx.x < TWC * T::SIZE;
  const int col = act ? (int)threadIdx.x % TWC : 0, tl = act ? (int)threadIdx.x / TWC : T::SIZE;
  int tile, bj;
  col_order<G, TWC>((int)blockIdx.x, (int)gridDim.x, J, bj, tile);
  const int b = bj / J;
  const int x = tile * TWC + col;
  C* L = lds + col * T::LDSC;

  // the coil-row, rho and coil-image loads are issued before the first exchange,
  // so that their latencies overlap; the float64 direction is loaded after the
  // first transform, which keeps the kernel at 160 VGPRs (3 waves per SIMD
  // instead of 2; measured 18 % faster at batch 16)
  const double2* u1 = U1 + (size_t)bj * GC * R + x;
  C a[T::G2];
  fsA_load<G, SET_COIL>(tl, a, [&](int n) -> C {
    const int i = coil_idx<G>(n);
    return i < 0 ? czero<C>() : u1[(size_t)i * R];
  });
  const float2* rho = xh + (size_t)b * X;
  float2* cj = co + (size_t)bj * R * R;
  float2 rv[T::G1], cv[T::G1];
  double2 dv[T::G1];
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      if constexpr (cls_k<G, SET_IMG, k1>() != NEVER) {
        const int iy = img_idx<G>(T::G2 * k1 + tl);
        if (iy >= 0) {
          const size_t e = (size_t)iy * R + x;
          rv[k1] = rho[e];
          if constexpr (NORMAL) cv[k1] = cj[e];
        }
      }
    });
  }
  C v[T::G1];
  fsA_regs<G, +1, SET_IMG>(tl, L, tw, a, v);
  if constexpr (NORMAL) {
    if (tl < T::G2) {
      sfor<0, T::G1>([&](auto c) {
        constexpr int k1 = decltype(c)::value;
        if constexpr (cls_k<G, SET_IMG, k1>() != NEVER) {
          const int iy = img_idx<G>(T::G2 * k1 + tl);
          if (iy >= 0) dv[k1] = pv[(size_t)b * X + (size_t)iy * R + x];
        }
      });
    }
  }

  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      const int iy = img_idx<G>(T::G2 * k1 + tl);
      C u = czero<C>();
      if (cls_k<G, SET_IMG, k1>() != NEVER && iy >= 0) {
        const size_t e = (size_t)iy * R + x;
        const C r = to_d(rv[k1]);
        if constexpr (!NORMAL) {
          const float2 cf = to_f(v[k1]);
          cj[e] = cf;
          u = cmul(r, to_d(cf));   // the stored (float32) coil image, as later passes read it
        } else {
          u = cadd(cmul(to_d(cv[k1]), dv[k1]), cmul(r, v[k1]));
        }
        if constexpr (TO_IMG) static_cast<float2*>(outp)[(size_t)bj * R * R + e] = to_f(u);
      }
      v[k1] = u;
    });
  }
  if constexpr (!TO_IMG) {
    if (outp == nullptr) return;   // uniform: coil synthesis only
    S2* o = static_cast<S2*>(outp) + (size_t)bj * G * R + x;
    fsB<G, -1, SET_IMG, SET_ALL>(tl, L, tw, v, [&](int n, C val) { nt_store(o + (size_t)n * R, store_as<S2>(val)); });
  }
}

// ---------------------------------------------------------------------------
// toep_rows: along x, FFT (R inputs) -> x P(ky, kx) -> iFFT (R outputs), in place.
// ---------------------------------------------------------------------------
// With PQ, the blocks are laid out per item (nbi blocks of RT lines over the
// item's J G lines, the last one partial) and each block also writes the
// partial sum_k P(k) |U(k)|^2 of its lines' spectra to part[b * pstride +
// block]: summed over an item it is <u, F^H F u> = ||DF p||^2 (Parseval), the
// operator part of Re<p, q> in the four-pass CG iteration.  KEY names the
// grid side and the factorisation of its team transform (nlinv_fft.h), so
// that the factorisation of this pass can be chosen per plan.
//
// toep_lines transforms the RT = row_lines<KEY>() lines base .. base+RT-1 of
// U2 (those below base + nvalid; the other teams only take part in the
// barriers); every thread of the block calls it.  With PQ, the group's
// partial goes to *part.  The kernels below map blocks to line groups.
template <int KEY, class S2, bool PQ>
__device__ __forceinline__ void toep_lines(C* __restrict__ lds, double* __restrict__ sh, S2* __restrict__ U2,
                                           const float* __restrict__ P, const TurnArgs& turns,
                                           const double2* __restrict__ tw, int J, int base, int nvalid,
                                           double* __restrict__ part) {
  using T = Team<KEY>;
  constexpr int G = grid_of(KEY), R = G / 2, RT = row_lines<KEY>();
  const int rl0 = (int)threadIdx.x / T::SIZE;
  // lanes past the last team, or of a team past the last line, only take part in barriers
  const bool act = rl0 < RT && rl0 < nvalid;
  const int tl = act ? (int)threadIdx.x % T::SIZE : T::SIZE, rl = act ? rl0 : 0;
  const int row = act ? base + rl0 : 0;
  const int ky = row % G, b = row / G / J;
  // the turn of each line's item: a group's lines belong to at most two
  // consecutive items, whose turns are read from the kernel arguments with
  // block-uniform indices (scalar loads, not a per-lane memory round trip
  // ahead of the PSF row loads)
  const int b0 = __builtin_amdgcn_readfirstlane(base / G / J);
  const int t0 = turns.t[b0], t1 = turns.t[b0 + 1 < MAXB ? b0 + 1 : b0];
  S2* line = U2 + (size_t)row * R;
  const float* prow = P + ((size_t)(b == b0 ? t0 : t1) * G + ky) * G;
  C* L = lds + rl * T::LDSN;
  // every load of the group is issued before the first wait: the line, the
  // twiddle value and the PSF kernel values of this thread's spectrum outputs
  C a[T::G2];
  fsA_load<KEY, SET_IMG>(tl, a, [&](int n) -> C {
    const int ix = img_idx<G>(n);
    return ix < 0 ? czero<C>() : to_d(nt_load(line + ix));
  });
  const double2 tv = twiddle_of<KEY>(tw, tl);
  float pk[T::G1];
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      pk[k1] = prow[T::G2 * k1 + tl];
    });
  }
  C v[T::G1];
  fsA_regs<KEY, -1, SET_ALL>(tl, L, tv, a, v);
  double acc = 0.0;
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      if constexpr (PQ) acc += (double)pk[k1] * (v[k1].x * v[k1].x + v[k1].y * v[k1].y);
      v[k1] = cscale(v[k1], (double)pk[k1]);
    });
  }
  if constexpr (PQ) {
    static_assert(row_threads<KEY>() == 64, "one wavefront per block");
    const double s = block_sum_waves<64>(acc, sh);
    if (threadIdx.x == 0) *part = s;
  }
  fsB<KEY, +1, SET_ALL, SET_IMG>(tl, L, tv, v, [&](int n, C val) {
    const int ix = img_idx<G>(n);
    if (ix >= 0) nt_store(line + ix, store_as<S2>(val));
  });
}

template <int KEY, class S2, bool PQ = false>
__global__ void __launch_bounds__(row_threads<KEY>())
k_toep_rows(S2* __restrict__ U2, const float* __restrict__ P, TurnArgs turns,
            const double2* __restrict__ tw, int J, int nlines, double* __restrict__ part, int pstride, int nbi) {
  using T = Team<KEY>;
  constexpr int G = grid_of(KEY), RT = row_lines<KEY>();
  __shared__ C lds[RT * T::LDSN];
  __shared__ double sh[64];
  if constexpr (PQ) {
    // blocks per item: nbi groups of RT lines over the item's J G lines, the last one partial
    const int ib = blockIdx.x / nbi, lb = blockIdx.x - ib * nbi;
    toep_lines<KEY, S2, true>(lds, sh, U2, P, turns, tw, J, ib * J * G + lb * RT, J * G - lb * RT,
                              part + (size_t)ib * pstride + lb);
  } else {
    toep_lines<KEY, S2, false>(lds, sh, U2, P, turns, tw, J, blockIdx.x * RT, nlines - blockIdx.x * RT, nullptr);
  }
}

// One Toeplitz row pass over the plans of several grid sides in a single
// persistent launch: the line groups of every shape (shape k on its own grid
// and team, key Kk) form one list of tiles, shape 0's first, and block b of
// the launch's resident blocks takes tiles b, b + gridDim.x, ... until the
// list is done.  A shape with no lines is absent.  (A dynamic queue, blocks
// taking tiles from an atomic counter, was measured slower: the atomics on
// the one counter serialise, 0.61 against 0.39 ms for the mixed shapes.)
template <int K0, int K1, int K2>
constexpr int ragged_lds() {
  constexpr int a = row_lines<K0>() * Team<K0>::LDSN, b = row_lines<K1>() * Team<K1>::LDSN;
  constexpr int c = row_lines<K2>() * Team<K2>::LDSN;
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

template <int K0, int K1, int K2>
__global__ void __launch_bounds__(64)
k_toep_rows_ragged(ToepShape s0, ToepShape s1, ToepShape s2) {
  static_assert(row_threads<K0>() == 64 && row_threads<K1>() == 64 && row_threads<K2>() == 64,
                "one wavefront per tile");
  __shared__ C lds[ragged_lds<K0, K1, K2>()];
  __shared__ double sh[64];
  constexpr int R0 = row_lines<K0>(), R1 = row_lines<K1>(), R2 = row_lines<K2>();
  const int n0 = (s0.nlines + R0 - 1) / R0, n1 = (s1.nlines + R1 - 1) / R1, n2 = (s2.nlines + R2 - 1) / R2;
  const int total = n0 + n1 + n2;
  for (int t = blockIdx.x; t < total; t += gridDim.x) {      // block-uniform
    if (t < n0) {
      toep_lines<K0, double2, false>(lds, sh, s0.U2, s0.P, s0.turns, s0.tw, s0.J, t * R0, s0.nlines - t * R0,
                                     nullptr);
    } else if (t < n0 + n1) {
      const int u = t - n0;
      toep_lines<K1, double2, false>(lds, sh, s1.U2, s1.P, s1.turns, s1.tw, s1.J, u * R1, s1.nlines - u * R1,
                                     nullptr);
    } else {
      const int u = t - n0 - n1;
      toep_lines<K2, double2, false>(lds, sh, s2.U2, s2.P, s2.turns, s2.tw, s2.J, u * R2, s2.nlines - u * R2,
                                     nullptr);
    }
  }
}

// ---------------------------------------------------------------------------
// cols_back: iFFT along y (or an image-space input), channel terms, FFT along y
// to the coil rows.  MODE 0 normal, 1 residual z - t, 2 adjoint of `in` (image, float32),
// 3 plain W^-H column stage of coil images `in` (no channel products, no rho).
// ---------------------------------------------------------------------------
// EARLY (the four-pass CG form, whose batch-1 chain is latency-bound): the
// coil image and rho values are loaded together with the column, so that the
// pass has one memory round trip before its first transform and none after it
// (at G = 320 still within 3 waves per SIMD: 152 VGPRs)
template <int G, int TWC, int MODE, class S2, bool EARLY = false>
__global__ void __launch_bounds__((cols_threads<G, TWC>()))
k_cols_back(const void* __restrict__ inp, const float2* __restrict__ co, const float2* __restrict__ xh,
            const float2* __restrict__ z, const double2* __restrict__ tw, float2* __restrict__ PR,
            double2* __restrict__ U4, int J, long long X, CGRed red) {
  using T = Team<G>;
  constexpr int R = G / 2, GC = G / 4, NT = R / TWC, NTH = cols_threads<G, TWC>();
  __shared__ C lds[TWC * T::LDSC];
  if constexpr (MODE == 0) {
    // four-pass CG: one extra block per item, after the pass's own blocks,
    // reduces the partials of the passes before it to (Re<p, q>, rr) in a
    // fixed order while the pass runs (block-uniform branch)
    if (red.scal && (int)blockIdx.x >= red.nbase) {
      __shared__ double shr[2];
      const int bi = (int)blockIdx.x - red.nbase;
      const double2 d = wave0_sum2_arrays(red.dfp + (size_t)bi * red.sdfp, red.ndfp,
                                          red.pp + (size_t)bi * red.spp, red.npp, shr);
      const double2 r = wave0_sum2_arrays(red.rr + (size_t)bi * red.srr, red.nrr, red.rr, 0, shr);
      if (threadIdx.x == 0) red.scal[bi] = make_double2(d.x + red.alpha * d.y, r.x);
      return;
    }
  }
  const bool act = (int)threadIdx.x < TWC * T::SIZE;
  const int col = act ? (int)threadIdx.x % TWC : 0, tl = act ? (int)threadIdx.x / TWC : T::SIZE;
  // the four-pass form (batch 1: every block resident at once) keeps the
  // plain order (channel-fastest there, with its forward pass: plain series
  // 197.5 against 198.3 frames/s)
  int tile = (int)blockIdx.x % NT, bj = (int)blockIdx.x / NT;
  if constexpr (!EARLY) {
    const int n = (MODE == 0 && red.scal) ? red.nbase : (int)gridDim.x;
    col_order<G, TWC>((int)blockIdx.x, n, J, bj, tile);
  }
  const int b = bj / J;
  const int x = tile * TWC + col;
  C* L = lds + col * T::LDSC;
  const size_t img = (size_t)bj * R * R;

  const double2 tv = twiddle_of<G>(tw, tl);
  const float2* rho = xh + (size_t)b * X;
  C v[T::G1];
  float2 cov[T::G1], rov[T::G1];
  if constexpr (MODE < 2) {
    const S2* c0 = static_cast<const S2*>(inp) + (size_t)bj * G * R + x;
    C a[T::G2];
    fsA_load<G, SET_ALL>(tl, a, [&](int n) -> C { return to_d(nt_load(c0 + (size_t)n * R)); });
    if constexpr (EARLY) {
      static_assert(MODE == 0, "the early loads serve the normal operator");
      // every lane loads (rows outside the image clamped to row 0, never
      // used): a value defined on every path is converted where it is used,
      // so no conversion waits on a load while other loads are still to issue
      sfor<0, T::G1>([&](auto c) {
        constexpr int k1 = decltype(c)::value;
        if constexpr (cls_k<G, SET_IMG, k1>() != NEVER) {
          const int iy = img_idx<G>(T::G2 * k1 + tl);
          const size_t e = (size_t)(iy >= 0 ? iy : 0) * R + x;
          cov[k1] = co[img + e];
          rov[k1] = rho[e];
        }
      });
    }
    fsA_regs<G, +1, SET_IMG>(tl, L, tv, a, v);
  } else {
    const float2* in = static_cast<const float2*>(inp);
    if (tl < T::G2) {
      sfor<0, T::G1>([&](auto c) {
        constexpr int k1 = decltype(c)::value;
        const int iy = img_idx<G>(T::G2 * k1 + tl);
        v[k1] = iy < 0 ? czero<C>() : to_d(in[img + (size_t)iy * R + x]);
      });
    }
  }

  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      const int iy = img_idx<G>(T::G2 * k1 + tl);
      C s = czero<C>();
      if (iy >= 0) {
        const size_t e = (size_t)iy * R + x;
        C t = v[k1];
        if constexpr (MODE == 3) {
          s = t;   // plain W^-H of a coil image: no channel products
        } else {
          if constexpr (MODE == 1) t = csub(to_d(z[img + e]), t);
          const float2 pv = to_f(cjmul(to_d(EARLY ? cov[k1] : co[img + e]), t));
          if constexpr (EARLY) nt_store(PR + img + e, pv);
          else PR[img + e] = pv;
          s = cjmul(to_d(EARLY ? rov[k1] : rho[e]), t);
        }
      }
      v[k1] = s;
    });
  }
  double2* o = U4 + (size_t)bj * GC * R + x;
  fsB<G, -1, SET_IMG, SET_COIL>(tl, L, tv, v, [&](int n, C val) {
    const int i = coil_idx<G>(n);
    if (i >= 0) {
      if constexpr (EARLY) nt_store(o + (size_t)i * R, val);
      else o[(size_t)i * R] = val;
    }
  });
}

// ---------------------------------------------------------------------------
// coilh_rows: W^-H along x plus the regularisation term.
// MODE 0: q = W^-H(.) + alpha p  (partials Re<p, q> -> part at slot_off + block);
//         nr further blocks per item form the image block of q,
//         q_rho = sum_j PR_j + alpha p_rho (channel sum in channel order, FP64)
// MODE 1: b = W^-H(.) - alpha (x - x_prev) -> out, out2 (partials |b|^2);
//         nr further blocks per item form the image block of b,
//         b_rho = sum_j PR_j - alpha (rho - rho_prev)
// MODE 2: raw W^-H(.) -> out
// ---------------------------------------------------------------------------
template <int G, int MODE>
__global__ void __launch_bounds__(row_threads<G>())
k_coilh_rows(const double2* __restrict__ U4, const float* __restrict__ dinv, const double2* __restrict__ tw,
             const double2* __restrict__ pv, const float2* __restrict__ xh, const float2* __restrict__ xprev,
             const float2* __restrict__ PR, double alpha, double2* __restrict__ out, double2* __restrict__ out2,
             double* __restrict__ part, int stride, int slot_off, int J, long long X, int nb, int nr,
             double2* __restrict__ vr) {
  using T = Team<G>;
  constexpr int R = G / 2, GC = G / 4, NTH = row_threads<G>(), RT = row_lines<G>();
  static_assert(NTH == 64, "the q_rho block count assumes one wavefront per block");
  __shared__ C lds[RT * T::LDSN];
  __shared__ double sh[NTH];
  // nb line blocks, each RT of the item's J * GC lines, then nr q_rho blocks per
  // item; one partial per block
  const int b = blockIdx.x / (nb + nr), chunk = blockIdx.x - b * (nb + nr);
  if constexpr (MODE == 0) {
    if (chunk >= nb) {   // block-uniform: image block of q
      constexpr int E = RHOQ_E;
      const int e0 = (chunk - nb) * NTH * E + (int)threadIdx.x;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const int e = e0 + k * NTH;
        if (e < R * R) {
          const size_t ve = (size_t)b * X + e;
          const double2 p = pv[ve];
          double qx = 0.0, qy = 0.0;
          for (int j = 0; j < J; ++j) {
            const float2 pr = PR[((size_t)b * J + j) * R * R + e];
            qx += pr.x;
            qy += pr.y;
          }
          qx += alpha * p.x;
          qy += alpha * p.y;
          out[ve] = make_double2(qx, qy);
          acc += p.x * qx + p.y * qy;
        }
      }
      const double s = block_sum_waves<NTH>(acc, sh);
      if (threadIdx.x == 0) part[(size_t)b * stride + slot_off + chunk] = s;
      return;
    }
  }
  if constexpr (MODE == 1) {
    if (chunk >= nb) {   // block-uniform: image block of the right-hand side,
      // b_rho = sum_j PR_j - alpha (rho - rho_prev) (channel sum in channel
      // order), one pixel per lane, into out and out2, |b|^2 partials beside
      // those of the coil block; the channel products are loaded up front
      // (indices clamped to J - 1, only k < J summed), the rest after them
      const int e = (chunk - nb) * NTH + (int)threadIdx.x;
      double acc = 0.0;
      if (e < R * R) {
        constexpr int JP = 16;
        float2 prv[JP];
        sfor<0, JP>([&](auto c) {
          constexpr int k = decltype(c)::value;
          prv[k] = PR[((size_t)b * J + (k < J ? k : J - 1)) * R * R + e];
        });
        const size_t ve = (size_t)b * X + e;
        const float2 rho = xh[ve];
        const float2 rp = xprev ? xprev[ve] : make_float2(1.f, 0.f);
        double sx = 0.0, sy = 0.0;
        sfor<0, JP>([&](auto c) {
          constexpr int k = decltype(c)::value;
          if (k < J) {
            sx += prv[k].x;
            sy += prv[k].y;
          }
        });
        for (int jj = JP; jj < J; ++jj) {
          const float2 pr = PR[((size_t)b * J + jj) * R * R + e];
          sx += pr.x;
          sy += pr.y;
        }
        const double2 bv = make_double2(sx - alpha * ((double)rho.x - rp.x), sy - alpha * ((double)rho.y - rp.y));
        out[ve] = bv;
        out2[ve] = bv;
        acc = bv.x * bv.x + bv.y * bv.y;
      }
      const double s = block_sum_waves<NTH>(acc, sh);
      if (threadIdx.x == 0) part[(size_t)b * stride + slot_off + chunk] = s;
      return;
    }
  }
  const int rl0 = (int)threadIdx.x / T::SIZE, l0 = chunk * RT + rl0;
  const bool act = rl0 < RT && l0 < J * GC;
  const int tl = act ? (int)threadIdx.x % T::SIZE : T::SIZE, rl = act ? rl0 : 0;
  const int l = act ? l0 : 0;
  const int i = l % GC, j = l / GC, bj = b * J + j;
  const double2* line = U4 + ((size_t)bj * GC + i) * R;
  const size_t base = (size_t)b * X + (size_t)R * R + ((size_t)j * GC + i) * GC;
  const float* dw = dinv + i * GC;
  // loads of the output terms are issued together with the line loads
  float wv[T::G1];
  double2 pvv[T::G1];
  float2 xv[T::G1], xpv[T::G1];
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      if constexpr (cls_k<G, SET_COIL, k1>() != NEVER) {
        const int ic = coil_idx<G>(T::G2 * k1 + tl);
        if (ic >= 0) {
          wv[k1] = dw[ic];
          if constexpr (MODE == 0) pvv[k1] = pv[base + ic];
          if constexpr (MODE == 1) {
            xv[k1] = xh[base + ic];
            xpv[k1] = xprev ? xprev[base + ic] : make_float2(0.f, 0.f);
          }
        }
      }
    });
  }
  C v[T::G1];
  fsA<G, -1, SET_IMG, SET_COIL>(tl, lds + rl * T::LDSN, tw, [&](int n) -> C {
    const int ix = img_idx<G>(n);
    return ix < 0 ? czero<C>() : line[ix];
  }, v);
  double acc = 0.0;
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      const int ic = coil_idx<G>(T::G2 * k1 + tl);
      if (cls_k<G, SET_COIL, k1>() != NEVER && ic >= 0) {
        const size_t e = base + ic;
        const double2 w = cscale(v[k1], (double)wv[k1]);
        if constexpr (MODE == 0) {
          const double2 p = pvv[k1];
          const double2 q = make_double2(w.x + alpha * p.x, w.y + alpha * p.y);
          out[e] = q;
          acc += p.x * q.x + p.y * q.y;
        } else if constexpr (MODE == 1) {
          const double2 bv = make_double2(w.x - alpha * ((double)xv[k1].x - xpv[k1].x),
                                          w.y - alpha * ((double)xv[k1].y - xpv[k1].y));
          out[e] = bv;
          if (out2) out2[e] = bv;
          acc += bv.x * bv.x + bv.y * bv.y;
          v[k1] = cscale(bv, (double)wv[k1]);   // input of the x-stage of W^-1 b
        } else {
          out[e] = w;
        }
      } else if constexpr (MODE == 1) {
        v[k1] = czero<C>();
      }
    });
  }
  if constexpr (MODE == 1) {
    // x-stage of W^-1 applied to the right-hand side's coil row: the first
    // residual's row transform of the four-pass CG iteration
    if (vr) {
      double2* o = vr + ((size_t)bj * GC + i) * R;
      fsB<G, +1, SET_COIL, SET_IMG>(tl, lds + rl * T::LDSN, tw, v, [&](int n, C val) {
        const int ix = img_idx<G>(n);
        if (ix >= 0) o[ix] = val;
      });
    }
  }
  if constexpr (MODE != 2) {
    const double s = block_sum_waves<NTH>(acc, sh);
    if (threadIdx.x == 0) part[(size_t)b * stride + slot_off + chunk] = s;
  }
}

// ---------------------------------------------------------------------------
// Four-pass CG iteration.  The direction update, the coil synthesis of the
// direction and the CG vector updates are folded into the passes of the
// operator, so that one iteration is four dependent kernels instead of six:
//   cg_cols_fwd : beta = rr_i / rr_{i-1}; p_i = r_i + beta p_{i-1} (image block
//                 written by the channel-0 blocks, coil row i by the lanes of
//                 columns 2i and 2i + 1); the x-stage of W^-1 p_i by linearity,
//                 V_p = V_r + beta V_p (V_r: x-stage of W^-1 r_i from the pass
//                 before); y-iFFT -> dc, u = c dp_rho + rho dc, y-FFT -> U2;
//                 partials |p_i|^2, one per channel and column
//   toep_rows   : the plain pass plus the partials sum_k P(k)|U(k)|^2, which sum
//                 to ||DF p_i||^2 = <u, F^H F u> (Parseval)
//   cols_back   : the plain pass; the first block of each item reduces
//                 Re<p, q> = ||DF p||^2 + alpha |p|^2 and rr_i
//   cg_coilh    : a = rr_i / Re<p, q>; x-FFT (W^-H) -> q = W^-H(..) + alpha p_i,
//                 h += a p_i, r_{i+1} = r_i - a q, the x-stage of W^-1 r_{i+1}
//                 -> V_r; the image block q_rho = sum_j PR_j + alpha p_rho
//                 likewise; partials |r_{i+1}|^2.  Last iteration: x += h.
// Re<p, q> comes from the spectrum instead of the vector q, so a is known
// before q is formed; in exact arithmetic both are the same number.
// ---------------------------------------------------------------------------

template <int G, int TWC, class S2>
__global__ void __launch_bounds__((cols_threads<G, TWC>()))
k_cg_cols_fwd(const double2* __restrict__ Vr, double2* __restrict__ Vp, const float2* __restrict__ co,
              const float2* __restrict__ xh, const double2* __restrict__ Rv, const double2* __restrict__ Pold,
              double2* __restrict__ Pnew, Partials sc, const double2* __restrict__ scal,
              double* __restrict__ ppp, int spp, const double2* __restrict__ tw, S2* __restrict__ U2, int J,
              long long X, int first) {
  using T = Team<G>;
  constexpr int R = G / 2, GC = G / 4, NT = R / TWC, NTH = cols_threads<G, TWC>();
  constexpr int MC = (GC / 2 + T::SIZE - 1) / T::SIZE;   // coil-block entries per lane
  __shared__ C lds[TWC * T::LDSC];
  __shared__ double sh[1];
  const bool act = (int)threadIdx.x < TWC * T::SIZE;
  const int col = act ? (int)threadIdx.x % TWC : 0, tl = act ? (int)threadIdx.x / TWC : T::SIZE;
  const int tile = blockIdx.x % NT, bj = blockIdx.x / NT, b = bj / J, j = bj - b * J;
  const int x = tile * TWC + col;
  C* L = lds + col * T::LDSC;
  const size_t xb = (size_t)b * X;

  // Every load of the block is issued before the first wait, so that the
  // pass has one memory round trip ahead of its first transform and none
  // after it (at batch 1 the CG iteration is a chain of such round trips;
  // the registers this takes leave 2 waves per SIMD instead of 3): the
  // partial sums behind beta (first wavefront), the CG scalars, the x-stage
  // rows of r_i and p_{i-1} at this column, the twiddle value, the residual
  // and old direction of the image and coil blocks, and rho and the coil image.
  double ps[BETA_PRE];
  const bool w0 = threadIdx.x < 64;
  const double* pcur = sc.cur + (size_t)b * sc.stride;
  if (!first && w0) {
    sfor<0, BETA_PRE>([&](auto c) {
      constexpr int k = decltype(c)::value;
      const int i = (int)threadIdx.x + 64 * k;
      ps[k] = i < sc.ncur ? pcur[i] : 0.0;
    });
  }
  // rr_{i-1}: the reducing block of the previous iteration's back column pass
  // summed the same partials in the same order
  const double rr_prev = first ? 0.0 : scal[b].y;
  const size_t vo = (size_t)bj * GC * R + x;
  C a[T::G2], vp[T::G2];
  if (tl < T::G1) {
    sfor<0, T::G2>([&](auto c) {
      constexpr int n2 = decltype(c)::value;
      a[n2] = czero<C>();
      vp[n2] = czero<C>();
      if constexpr (cls_n<G, SET_COIL, n2>() != NEVER) {
        const int i = coil_idx<G>(tl + T::G1 * n2);
        if (i >= 0) {
          a[n2] = Vr[vo + (size_t)i * R];
          if (!first) vp[n2] = Vp[vo + (size_t)i * R];
        }
      }
    });
  }
  const double2 tv = twiddle_of<G>(tw, tl);
  // coil block of p_i: column x takes half of coil row x / 2 (R = 2 G_c), and
  // every partial below covers one column, so the sums do not depend on the
  // tile schedule (every schedule gives the same bits)
  const size_t e0 = xb + (size_t)R * R + ((size_t)j * GC + (x >> 1)) * GC + (x & 1) * (GC / 2);
  const float2* rho = xh + xb;
  const float2* cj = co + (size_t)bj * R * R;
  double2 rv[T::G1], po[T::G1], crv[MC], cpo[MC];
  float2 rov[T::G1], cv[T::G1];
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      const int iy = img_idx<G>(T::G2 * k1 + tl);
      if (cls_k<G, SET_IMG, k1>() != NEVER && iy >= 0) {
        const size_t e = xb + (size_t)iy * R + x;
        rv[k1] = Rv[e];
        if (!first) po[k1] = Pold[e];
      }
    });
  }
  if (act) {
    sfor<0, MC>([&](auto c) {
      constexpr int k = decltype(c)::value;
      const int m = tl + T::SIZE * k;
      if (m < GC / 2) {
        crv[k] = Rv[e0 + m];
        if (!first) cpo[k] = Pold[e0 + m];
      }
    });
  }
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      if constexpr (cls_k<G, SET_IMG, k1>() != NEVER) {
        const int iy = img_idx<G>(T::G2 * k1 + tl);
        if (iy >= 0) {
          const size_t e = (size_t)iy * R + x;
          rov[k1] = rho[e];
          cv[k1] = cj[e];
        }
      }
    });
  }
  // beta = rr_i / rr_{i-1}: the first wavefront sums the partials of rr_i in
  // index order (the order of every other reduction of these partials),
  // whatever the block size
  double beta = 0.0;
  if (!first) {
    if (w0) {
      double su = 0.0;
      sfor<0, BETA_PRE>([&](auto c) { su += ps[decltype(c)::value]; });
      for (int i = (int)threadIdx.x + 64 * BETA_PRE; i < sc.ncur; i += 64) su += pcur[i];
      for (int off = 32; off > 0; off >>= 1) su += __shfl_down(su, off, 64);
      if (threadIdx.x == 0) sh[0] = su;
    }
    __syncthreads();
    beta = rr_prev != 0.0 ? sh[0] / rr_prev : 0.0;
  }
  // V_p = V_r + beta V_p: the x-stage of W^-1 p_i, kept for the next iteration
  if (tl < T::G1) {
    sfor<0, T::G2>([&](auto c) {
      constexpr int n2 = decltype(c)::value;
      if constexpr (cls_n<G, SET_COIL, n2>() != NEVER) {
        const int i = coil_idx<G>(tl + T::G1 * n2);
        if (i >= 0) {
          a[n2] = make_double2(a[n2].x + beta * vp[n2].x, a[n2].y + beta * vp[n2].y);
          nt_store(Vp + vo + (size_t)i * R, a[n2]);
        }
      }
    });
  }
  // image block of p_i at this column (written once, by the channel-0 blocks),
  // and its product with the coil image, formed before the transform so that
  // the residual values need not be held through it
  double acc = 0.0;
  C cp[T::G1];
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      const int iy = img_idx<G>(T::G2 * k1 + tl);
      cp[k1] = czero<C>();
      if (cls_k<G, SET_IMG, k1>() != NEVER && iy >= 0) {
        double2 dp = rv[k1];
        if (!first) dp = make_double2(dp.x + beta * po[k1].x, dp.y + beta * po[k1].y);
        if (j == 0) {
          nt_store(Pnew + xb + (size_t)iy * R + x, dp);
          acc += dp.x * dp.x + dp.y * dp.y;
        }
        cp[k1] = cmul(to_d(cv[k1]), dp);
      }
    });
  }
  C v[T::G1];
  fsA_regs<G, +1, SET_IMG>(tl, L, tv, a, v);
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      const int iy = img_idx<G>(T::G2 * k1 + tl);
      C u = czero<C>();
      if (cls_k<G, SET_IMG, k1>() != NEVER && iy >= 0) u = cadd(cp[k1], cmul(to_d(rov[k1]), v[k1]));
      v[k1] = u;
    });
  }
  S2* o = U2 + (size_t)bj * G * R + x;
  fsB<G, -1, SET_IMG, SET_ALL>(tl, L, tv, v, [&](int n, C val) { nt_store(o + (size_t)n * R, store_as<S2>(val)); });
  if (act) {
    sfor<0, MC>([&](auto c) {
      constexpr int k = decltype(c)::value;
      const int m = tl + T::SIZE * k;
      if (m < GC / 2) {
        double2 p = crv[k];
        if (!first) p = make_double2(p.x + beta * cpo[k].x, p.y + beta * cpo[k].y);
        nt_store(Pnew + e0 + m, p);
        acc += p.x * p.x + p.y * p.y;
      }
    });
  }
  // |p_i|^2 partial of each column: its lanes in lane order
  __shared__ double shc[NTH];
  shc[threadIdx.x] = acc;
  __syncthreads();
  if ((int)threadIdx.x < TWC) {
    double sp = 0.0;
    for (int t = 0; t < T::SIZE; ++t) sp += shc[t * TWC + threadIdx.x];
    ppp[(size_t)b * spp + (size_t)j * R + tile * TWC + threadIdx.x] = sp;
  }
}

template <int G>
__global__ void __launch_bounds__(row_threads<G>())
k_cg_coilh(const double2* __restrict__ U4, const float* __restrict__ dinv, const double2* __restrict__ tw,
           const double2* __restrict__ Pn, const float2* __restrict__ PR, double2* __restrict__ H,
           double2* __restrict__ Rv, float2* __restrict__ xh, double2* __restrict__ Vr,
           const double2* __restrict__ scal, double alpha, double* __restrict__ rr_next, int stride, int J,
           long long X, int nb, int nr, int first, int last) {
  using T = Team<G>;
  constexpr int R = G / 2, GC = G / 4, NTH = row_threads<G>(), RT = row_lines<G>();
  static_assert(NTH == 64, "the image-block count assumes one wavefront per block");
  __shared__ C lds[RT * T::LDSN];
  __shared__ double sh[NTH];
  const int b = blockIdx.x / (nb + nr), chunk = blockIdx.x - b * (nb + nr);
  // In both block kinds every load is issued before the first wait (one
  // memory round trip; the CG scalars, which only the arithmetic needs, last).
  if (chunk >= nb) {   // block-uniform: image block, one pixel per lane
    const int e = (chunk - nb) * NTH + (int)threadIdx.x;
    const bool in = e < R * R;
    const size_t ve = (size_t)b * X + e;
    // the first JP channel products are loaded up front (channel indices
    // clamped to J - 1, so that no load waits on a branch; only k < J is
    // summed), the rest after them
    constexpr int JP = 16;
    float2 pr[JP];
    double2 p, h, r;
    float2 xv;
    if (in) {
      sfor<0, JP>([&](auto c) {
        constexpr int k = decltype(c)::value;
        pr[k] = PR[((size_t)b * J + (k < J ? k : J - 1)) * R * R + e];
      });
      p = Pn[ve];
      h = first ? make_double2(0.0, 0.0) : H[ve];
      if (last) xv = xh[ve];
      else r = Rv[ve];
    }
    const double2 sv = scal[b];                        // (Re<p, q>, rr_i)
    const double a = sv.x != 0.0 ? sv.y / sv.x : 0.0;
    double acc = 0.0;
    if (in) {
      double qx = 0.0, qy = 0.0;   // channel sum in channel order
      sfor<0, JP>([&](auto c) {
        constexpr int k = decltype(c)::value;
        if (k < J) {
          qx += pr[k].x;
          qy += pr[k].y;
        }
      });
      for (int j = JP; j < J; ++j) {
        const float2 t = PR[((size_t)b * J + j) * R * R + e];
        qx += t.x;
        qy += t.y;
      }
      qx += alpha * p.x;
      qy += alpha * p.y;
      h = make_double2(h.x + a * p.x, h.y + a * p.y);
      if (last) {
        nt_store(xh + ve, make_float2((float)(xv.x + h.x), (float)(xv.y + h.y)));
      } else {
        nt_store(H + ve, h);
        r = make_double2(r.x - a * qx, r.y - a * qy);
        nt_store(Rv + ve, r);
        acc = r.x * r.x + r.y * r.y;
      }
    }
    if (!last) {
      const double s = block_sum_waves<NTH>(acc, sh);
      if (threadIdx.x == 0) rr_next[(size_t)b * stride + nb + (chunk - nb)] = s;
    }
    return;
  }
  const int rl0 = (int)threadIdx.x / T::SIZE, l0 = chunk * RT + rl0;
  const bool act = rl0 < RT && l0 < J * GC;
  const int tl = act ? (int)threadIdx.x % T::SIZE : T::SIZE, rl = act ? rl0 : 0;
  const int l = act ? l0 : 0;
  const int i = l % GC, j = l / GC, bj = b * J + j;
  const double2* line = U4 + ((size_t)bj * GC + i) * R;
  const size_t base = (size_t)b * X + (size_t)R * R + ((size_t)j * GC + i) * GC;
  const float* dw = dinv + i * GC;
  C ln[T::G2];
  fsA_load<G, SET_IMG>(tl, ln, [&](int n) -> C {
    const int ix = img_idx<G>(n);
    return ix < 0 ? czero<C>() : line[ix];
  });
  const double2 tv = twiddle_of<G>(tw, tl);
  float wv[T::G1];
  double2 pvv[T::G1], hv[T::G1], rvv[T::G1];
  float2 xv[T::G1];
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      if constexpr (cls_k<G, SET_COIL, k1>() != NEVER) {
        const int ic = coil_idx<G>(T::G2 * k1 + tl);
        if (ic >= 0) {
          wv[k1] = dw[ic];
          pvv[k1] = Pn[base + ic];
          hv[k1] = first ? make_double2(0.0, 0.0) : H[base + ic];
          if (last) xv[k1] = xh[base + ic];
          else rvv[k1] = Rv[base + ic];
        }
      }
    });
  }
  const double2 sv = scal[b];                        // (Re<p, q>, rr_i)
  const double a = sv.x != 0.0 ? sv.y / sv.x : 0.0;
  C* L = lds + rl * T::LDSN;
  C v[T::G1];
  fsA_regs<G, -1, SET_COIL>(tl, L, tv, ln, v);
  double acc = 0.0;
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      const int ic = coil_idx<G>(T::G2 * k1 + tl);
      C nv = czero<C>();
      if (cls_k<G, SET_COIL, k1>() != NEVER && ic >= 0) {
        const size_t e = base + ic;
        const double2 w = cscale(v[k1], (double)wv[k1]);
        const double2 p = pvv[k1];
        const double2 q = make_double2(w.x + alpha * p.x, w.y + alpha * p.y);
        const double2 h = make_double2(hv[k1].x + a * p.x, hv[k1].y + a * p.y);
        if (last) {
          nt_store(xh + e, make_float2((float)(xv[k1].x + h.x), (float)(xv[k1].y + h.y)));
        } else {
          nt_store(H + e, h);
          const double2 r = make_double2(rvv[k1].x - a * q.x, rvv[k1].y - a * q.y);
          nt_store(Rv + e, r);
          acc += r.x * r.x + r.y * r.y;
          nv = cscale(r, (double)wv[k1]);   // input of the x-stage of W^-1 r_{i+1}
        }
      }
      v[k1] = nv;
    });
  }
  if (!last) {   // uniform
    double2* o = Vr + ((size_t)bj * GC + i) * R;
    fsB<G, +1, SET_COIL, SET_IMG>(tl, L, tv, v, [&](int n, C val) {
      const int ix = img_idx<G>(n);
      if (ix >= 0) nt_store(o + ix, val);
    });
    const double s = block_sum_waves<NTH>(acc, sh);
    if (threadIdx.x == 0) rr_next[(size_t)b * stride + chunk] = s;
  }
}

// ---------------------------------------------------------------------------
// PSF kernel: full forward 2D FFT of the embedded PSF (float64 scratch)
// ---------------------------------------------------------------------------

// Full G-point FFT along the rows of a G x G array (in place), forward.
template <int G>
__global__ void __launch_bounds__(rows_threads<G>())
k_fft_rows_full(double2* __restrict__ a, const double2* __restrict__ tw) {
  using T = Team<G>;
  __shared__ C lds[ROWS * T::LDSN];
  const bool act = (int)threadIdx.x < ROWS * T::SIZE;
  const int tl = act ? (int)threadIdx.x % T::SIZE : T::SIZE, rl = act ? (int)threadIdx.x / T::SIZE : 0;
  const int row = blockIdx.x * ROWS + rl;
  double2* line = a + (size_t)row * G;
  C v[T::G1];
  fsA<G, -1, SET_ALL, SET_ALL>(tl, lds + rl * T::LDSN, tw, [&](int n) -> C { return line[n]; }, v);
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      line[T::G2 * k1 + tl] = v[k1];
    });
  }
}

// Full forward FFT along the columns; P[ky][kx] = Re(.) * scale (float32).
template <int G>
__global__ void __launch_bounds__(cols_threads<G>())
k_fft_cols_psf(const double2* __restrict__ a, float* __restrict__ P, const double2* __restrict__ tw,
               double scale) {
  using T = Team<G>;
  __shared__ C lds[TW * T::LDSC];
  const bool act = (int)threadIdx.x < TW * T::SIZE;
  const int col = act ? (int)threadIdx.x % TW : 0, tl = act ? (int)threadIdx.x / TW : T::SIZE;
  const int x = blockIdx.x * TW + col;
  C v[T::G1];
  fsA<G, -1, SET_ALL, SET_ALL>(tl, lds + col * T::LDSC, tw, [&](int n) -> C { return a[(size_t)n * G + x]; }, v);
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      P[(size_t)(T::G2 * k1 + tl) * G + x] = (float)(v[k1].x * scale);
    });
  }
}

// ---------------------------------------------------------------------------
// Kaiser-Bessel gridding of the data (z_j = F^H y_j to within the kernel's
// error): gather onto the G x G grid through the per-turn table, inverse FFT
// of the rows (keep R columns), inverse FFT of the columns (keep R rows) with
// the deapodisation 1 / (R c(x) c(y)).
// ---------------------------------------------------------------------------

// g[b][j][p] = sum over table row p of w * y[b][j][s], in table order, FP64.
// Grid points with at most KB_SHORT entries take one thread each (all entry
// loads issued together); the few longer rows near the k-space centre, where
// every spoke passes, take a wavefront each, lanes striding over the entries
// and a fixed shuffle tree summing the lanes.  Both orders are fixed, so the
// result is reproducible.
constexpr int KBJ = 8;

template <int G>
__global__ void __launch_bounds__(VT)
k_kb_gather_short(const int* __restrict__ rp, const int2* __restrict__ ent, const int* __restrict__ pts,
                  const int2* __restrict__ counts, long long rp_stride, long long ent_stride, TurnArgs turns,
                  const float2* __restrict__ y, float2* __restrict__ grid, int J, int S) {
  constexpr int GG = G * G;
  const int b = blockIdx.y, t = turns.t[b];
  const int q = blockIdx.x * VT + threadIdx.x;
  if (q >= counts[t].x) return;
  const int p = pts[(size_t)t * GG + q];
  const int* r = rp + t * rp_stride;
  const int2* e = ent + t * ent_stride;
  const int e0 = r[p], n = r[p + 1] - e0;
  int2 en[KB_SHORT];
#pragma unroll
  for (int k = 0; k < KB_SHORT; ++k) en[k] = k < n ? e[e0 + k] : make_int2(0, 0);
  for (int j0 = 0; j0 < J; j0 += KBJ) {
    const int nj = J - j0 < KBJ ? J - j0 : KBJ;
    double2 acc[KBJ];
#pragma unroll
    for (int c = 0; c < KBJ; ++c) acc[c] = make_double2(0.0, 0.0);
    const float2* yb = y + ((size_t)b * J + j0) * S;
#pragma unroll
    for (int k = 0; k < KB_SHORT; ++k) {
      if (k < n) {
        const double wv = (double)__int_as_float(en[k].y);
#pragma unroll
        for (int c = 0; c < KBJ; ++c) {
          if (c < nj) {
            const float2 v = yb[(size_t)c * S + en[k].x];
            acc[c].x += wv * v.x;
            acc[c].y += wv * v.y;
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < KBJ; ++c)
      if (c < nj) grid[((size_t)b * J + j0 + c) * GG + p] = make_float2((float)acc[c].x, (float)acc[c].y);
  }
}

template <int G>
__global__ void __launch_bounds__(VT)
k_kb_gather_long(const int* __restrict__ rp, const int2* __restrict__ ent, const int* __restrict__ pts,
                 const int2* __restrict__ counts, long long rp_stride, long long ent_stride, TurnArgs turns,
                 const float2* __restrict__ y, float2* __restrict__ grid, int J, int S) {
  constexpr int GG = G * G;
  const int b = blockIdx.y, t = turns.t[b];
  const int lane = threadIdx.x & 63;
  const int nl = counts[t].y, nw = gridDim.x * (VT / 64);
  const int* r = rp + t * rp_stride;
  const int2* e = ent + t * ent_stride;
  for (int q = blockIdx.x * (VT / 64) + (int)(threadIdx.x >> 6); q < nl; q += nw) {   // wave-uniform
    const int p = pts[(size_t)t * GG + GG - 1 - q];     // long points are stored from the end
    const int e0 = r[p], e1 = r[p + 1];
    for (int j0 = 0; j0 < J; j0 += KBJ) {
      const int nj = J - j0 < KBJ ? J - j0 : KBJ;
      double2 acc[KBJ];
#pragma unroll
      for (int c = 0; c < KBJ; ++c) acc[c] = make_double2(0.0, 0.0);
      const float2* yb = y + ((size_t)b * J + j0) * S;
      for (int k = e0 + lane; k < e1; k += 64) {
        const int2 en = e[k];
        const double wv = (double)__int_as_float(en.y);
#pragma unroll
        for (int c = 0; c < KBJ; ++c) {
          if (c < nj) {
            const float2 v = yb[(size_t)c * S + en.x];
            acc[c].x += wv * v.x;
            acc[c].y += wv * v.y;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < KBJ; ++c) {
        double ax = acc[c].x, ay = acc[c].y;
        for (int off = 32; off > 0; off >>= 1) {
          ax += __shfl_down(ax, off, 64);
          ay += __shfl_down(ay, off, 64);
        }
        if (lane == 0 && c < nj) grid[((size_t)b * J + j0 + c) * GG + p] = make_float2((float)ax, (float)ay);
      }
    }
  }
}

// Inverse FFT of grid rows (all G samples) keeping the R image columns.
template <int G, class S2>
__global__ void __launch_bounds__(row_threads<G>())
k_kb_rows(const float2* __restrict__ grid, S2* __restrict__ out, const double2* __restrict__ tw, int nlines) {
  using T = Team<G>;
  constexpr int R = G / 2, RT = row_lines<G>();
  __shared__ C lds[RT * T::LDSN];
  const int rl0 = (int)threadIdx.x / T::SIZE;
  const int row0 = blockIdx.x * RT + rl0;
  const bool act = rl0 < RT && row0 < nlines;
  const int tl = act ? (int)threadIdx.x % T::SIZE : T::SIZE, rl = act ? rl0 : 0;
  const int row = act ? row0 : 0;
  const float2* line = grid + (size_t)row * G;
  C v[T::G1];
  fsA<G, +1, SET_ALL, SET_IMG>(tl, lds + rl * T::LDSN, tw, [&](int n) -> C { return to_d(line[n]); }, v);
  if (tl < T::G2) {
    S2* o = out + (size_t)row * R;
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      if constexpr (cls_k<G, SET_IMG, k1>() != NEVER) {
        const int ix = img_idx<G>(T::G2 * k1 + tl);
        if (ix >= 0) o[ix] = store_as<S2>(v[k1]);
      }
    });
  }
}

// Inverse FFT of the columns of the row output keeping R rows; deapodisation.
template <int G, class S2>
__global__ void __launch_bounds__(cols_threads<G>())
k_kb_cols(const S2* __restrict__ in, const float* __restrict__ cinv, const double2* __restrict__ tw,
          float2* __restrict__ z) {
  using T = Team<G>;
  constexpr int R = G / 2, NT = R / TW;
  __shared__ C lds[TW * T::LDSC];
  const bool act = (int)threadIdx.x < TW * T::SIZE;
  const int col = act ? (int)threadIdx.x % TW : 0, tl = act ? (int)threadIdx.x / TW : T::SIZE;
  const int tile = blockIdx.x % NT, bj = blockIdx.x / NT;
  const int x = tile * TW + col;
  const S2* c0 = in + (size_t)bj * G * R + x;
  C v[T::G1];
  fsA<G, +1, SET_ALL, SET_IMG>(tl, lds + col * T::LDSC, tw, [&](int n) -> C { return to_d(c0[(size_t)n * R]); }, v);
  if (tl < T::G2) {
    const double cx = cinv[x];
    float2* o = z + (size_t)bj * R * R + x;
    sfor<0, T::G1>([&](auto c) {
      constexpr int k1 = decltype(c)::value;
      if constexpr (cls_k<G, SET_IMG, k1>() != NEVER) {
        const int iy = img_idx<G>(T::G2 * k1 + tl);
        if (iy >= 0) o[(size_t)iy * R] = to_f(cscale(v[k1], cx * (double)cinv[iy]));
      }
    });
  }
}

// ---------------------------------------------------------------------------
// per-grid launch table
// ---------------------------------------------------------------------------

template <int G>
struct GLaunch {
  static constexpr int TH_ROWS = rows_threads<G>();
  static constexpr int TH_ROW1 = row_threads<G>();
  static constexpr int TH_COLS = cols_threads<G>();

  static hipError_t coil_rows(const Shape& s, const Bufs& w, hipStream_t st, const float2* src) {
    return launch_timed(w, k_coil_rows<G, float2>, dim3(s.B * s.NX3), dim3(TH_ROW1), 0, st, src,
                        (const double2*)nullptr, (double2*)nullptr, Partials{}, (const float*)w.dinv,
                        (const double2*)w.tw, w.U1, s.J, (long long)s.X, s.NX3, 0);
  }
  static hipError_t coil_rows_cg(const Shape& s, const Bufs& w, hipStream_t st, const double2* src,
                                 const double2* rsrc, double2* pdst, Partials sc) {
    constexpr int PER_BLOCK = TH_ROW1 * RHO_PER_THREAD;
    const int nr = rsrc ? (s.R * s.R + PER_BLOCK - 1) / PER_BLOCK : 0;
    return launch_timed(w, k_coil_rows<G, double2>, dim3(s.B * (s.NX3 + nr)), dim3(TH_ROW1), 0, st, src, rsrc,
                        pdst, sc, (const float*)w.dinv, (const double2*)w.tw, w.U1, s.J, (long long)s.X,
                        s.NX3, nr);
  }
  template <class S2, int TWC>
  static hipError_t cols_fwd_k(const Shape& s, const Bufs& w, hipStream_t st, int mode, float2* co,
                               const float2* xh, const double2* pv, void* out) {
    constexpr int TH = cols_threads<G, TWC>();
    const int blocks = s.B * s.J * (s.R / TWC);
    switch (mode) {
      case 0: return launch_timed(w, k_cols_fwd<G, TWC, 0, S2>, dim3(blocks), dim3(TH), 0, st,
                                   (const double2*)w.U1, co, xh, pv, (const double2*)w.tw, out, s.J, (long long)s.X);
      case 1: return launch_timed(w, k_cols_fwd<G, TWC, 1, S2>, dim3(blocks), dim3(TH), 0, st,
                                   (const double2*)w.U1, co, xh, pv, (const double2*)w.tw, out, s.J, (long long)s.X);
      case 2: return launch_timed(w, k_cols_fwd<G, TWC, 2, S2>, dim3(blocks), dim3(TH), 0, st,
                                   (const double2*)w.U1, co, xh, pv, (const double2*)w.tw, out, s.J, (long long)s.X);
      case 3: return launch_timed(w, k_cols_fwd<G, TWC, 3, S2>, dim3(blocks), dim3(TH), 0, st,
                                   (const double2*)w.U1, co, xh, pv, (const double2*)w.tw, out, s.J, (long long)s.X);
      default: return hipErrorInvalidValue;
    }
  }
  template <class S2>
  static hipError_t cols_fwd_t(const Shape& s, const Bufs& w, hipStream_t st, int mode, float2* co,
                               const float2* xh, const double2* pv, void* out) {
    return col_tile(s, true) == 4 ? cols_fwd_k<S2, 4>(s, w, st, mode, co, xh, pv, out)
                                  : cols_fwd_k<S2, TW>(s, w, st, mode, co, xh, pv, out);
  }
  static hipError_t cols_fwd(const Shape& s, const Bufs& w, hipStream_t st, int mode, float2* co,
                             const float2* xh, const double2* pv, void* out) {
    return cols_fwd_t<double2>(s, w, st, mode, co, xh, pv, out);
  }
  template <class S2, int KEY>
  static hipError_t toep_rows_t(const Shape& s, const Bufs& w, hipStream_t st, const TurnArgs& turns) {
    constexpr int RT = row_lines<KEY>();
    const int nlines = s.B * s.J * s.G;
    const int blocks = (nlines + RT - 1) / RT;
    return launch_timed(w, k_toep_rows<KEY, S2, false>, dim3(blocks), dim3(row_threads<KEY>()), 0, st,
                        static_cast<S2*>(w.U2), (const float*)w.P, turns, (const double2*)w.tw, s.J, nlines,
                        (double*)nullptr, 0, 1);
  }
  static hipError_t toep_rows(const Shape& s, const Bufs& w, hipStream_t st, const TurnArgs& turns) {
    return s.split ? toep_rows_t<double2, G + GKEY>(s, w, st, turns) : toep_rows_t<double2, G>(s, w, st, turns);
  }
  template <class S2, int TWC>
  static hipError_t cols_back_k(const Shape& s, const Bufs& w, hipStream_t st, int mode, const void* in,
                                const float2* co, const float2* xh, const float2* z) {
    constexpr int TH = cols_threads<G, TWC>();
    const int blocks = s.B * s.J * (s.R / TWC);
    switch (mode) {
      case 0: return launch_timed(w, k_cols_back<G, TWC, 0, S2>, dim3(blocks), dim3(TH), 0, st, in, co, xh, z,
                                   (const double2*)w.tw, w.PR, w.U1, s.J, (long long)s.X, CGRed{});
      case 1: return launch_timed(w, k_cols_back<G, TWC, 1, S2>, dim3(blocks), dim3(TH), 0, st, in, co, xh, z,
                                   (const double2*)w.tw, w.PR, w.U1, s.J, (long long)s.X, CGRed{});
      case 2: return launch_timed(w, k_cols_back<G, TWC, 2, S2>, dim3(blocks), dim3(TH), 0, st, in, co, xh, z,
                                   (const double2*)w.tw, w.PR, w.U1, s.J, (long long)s.X, CGRed{});
      case 3: return launch_timed(w, k_cols_back<G, TWC, 3, S2>, dim3(blocks), dim3(TH), 0, st, in, co, xh, z,
                                   (const double2*)w.tw, w.PR, w.U1, s.J, (long long)s.X, CGRed{});
      default: return hipErrorInvalidValue;
    }
  }
  template <class S2>
  static hipError_t cols_back_t(const Shape& s, const Bufs& w, hipStream_t st, int mode, const void* in,
                                const float2* co, const float2* xh, const float2* z) {
    return col_tile(s, false) == 4 ? cols_back_k<S2, 4>(s, w, st, mode, in, co, xh, z)
                                  : cols_back_k<S2, TW>(s, w, st, mode, in, co, xh, z);
  }
  static hipError_t cols_back(const Shape& s, const Bufs& w, hipStream_t st, int mode, const void* in,
                              const float2* co, const float2* xh, const float2* z) {
    return cols_back_t<double2>(s, w, st, mode, in, co, xh, z);
  }
  static hipError_t coilh_rows(const Shape& s, const Bufs& w, hipStream_t st, int mode, const double2* pv,
                               const float2* xh, const float2* xprev, double alpha, double2* out,
                               double2* out2) {
    // modes 0 and 1: NRQ image blocks per item after the line blocks
    const int nr = mode <= 1 ? s.NRQ : 0;
    const int blocks = s.B * (s.NX3 + nr);
    double* part = mode == 1 ? w.rr[0] : w.pq;
    const int off = 0;
    switch (mode) {
      case 0: return launch_timed(w, k_coilh_rows<G, 0>, dim3(blocks), dim3(TH_ROW1), 0, st,
                                   (const double2*)w.U1, (const float*)w.dinv, (const double2*)w.tw, pv, xh, xprev,
                                   (const float2*)w.PR, alpha, out, out2, part, s.stride, off, s.J,
                                   (long long)s.X, s.NX3, nr, (double2*)nullptr);
      case 1: return launch_timed(w, k_coilh_rows<G, 1>, dim3(blocks), dim3(TH_ROW1), 0, st,
                                   (const double2*)w.U1, (const float*)w.dinv, (const double2*)w.tw, pv, xh, xprev,
                                   (const float2*)w.PR, alpha, out, out2, part, s.stride, off, s.J,
                                   (long long)s.X, s.NX3, nr, w.Vr);
      case 2: return launch_timed(w, k_coilh_rows<G, 2>, dim3(blocks), dim3(TH_ROW1), 0, st,
                                   (const double2*)w.U1, (const float*)w.dinv, (const double2*)w.tw, pv, xh, xprev,
                                   (const float2*)w.PR, alpha, out, out2, part, s.stride, off, s.J,
                                   (long long)s.X, s.NX3, nr, (double2*)nullptr);
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  // four-pass CG iteration
  template <class S2, int TWC>
  static hipError_t cg_cols_fwd_k(const Shape& s, const Bufs& w, hipStream_t st, const float2* xh,
                                  const double2* pold, double2* pnew, Partials sc, int first) {
    constexpr int TH = cols_threads<G, TWC>();
    const int blocks = s.B * s.J * (s.R / TWC);
    return launch_timed(w, k_cg_cols_fwd<G, TWC, S2>, dim3(blocks), dim3(TH), 0, st, (const double2*)w.Vr, w.Vp,
                        (const float2*)w.CO, xh,
                        (const double2*)w.Rv, pold, pnew, sc, (const double2*)w.scal, w.ppp, s.NPP,
                        (const double2*)w.tw, static_cast<S2*>(w.U2), s.J, (long long)s.X, first);
  }
  template <class S2>
  static hipError_t cg_cols_fwd_t(const Shape& s, const Bufs& w, hipStream_t st, const float2* xh,
                                  const double2* pold, double2* pnew, Partials sc, int first) {
    return col_tile(s, true) == 4 ? cg_cols_fwd_k<S2, 4>(s, w, st, xh, pold, pnew, sc, first)
                                  : cg_cols_fwd_k<S2, TW>(s, w, st, xh, pold, pnew, sc, first);
  }
  static hipError_t cg_cols_fwd(const Shape& s, const Bufs& w, hipStream_t st, const float2* xh,
                                const double2* pold, double2* pnew, Partials sc, int first) {
    return cg_cols_fwd_t<double2>(s, w, st, xh, pold, pnew, sc, first);
  }
  // s.NTB blocks per item: the plan's derivation sizes it with the row
  // lines of the chosen factorisation (GTable::row_lines_split)
  template <class S2, int KEY>
  static hipError_t cg_toep_rows_t(const Shape& s, const Bufs& w, hipStream_t st, const TurnArgs& turns) {
    return launch_timed(w, k_toep_rows<KEY, S2, true>, dim3(s.B * s.NTB), dim3(row_threads<KEY>()), 0, st,
                        static_cast<S2*>(w.U2), (const float*)w.P, turns, (const double2*)w.tw, s.J,
                        s.B * s.J * s.G, w.pdfp, s.NTB, s.NTB);
  }
  static hipError_t cg_toep_rows(const Shape& s, const Bufs& w, hipStream_t st, const TurnArgs& turns) {
    return s.split ? cg_toep_rows_t<double2, G + GKEY>(s, w, st, turns)
                   : cg_toep_rows_t<double2, G>(s, w, st, turns);
  }
  template <class S2, int TWC>
  static hipError_t cg_cols_back_k(const Shape& s, const Bufs& w, hipStream_t st, const float2* xh,
                                   const CGRed& red) {
    constexpr int TH = cols_threads<G, TWC>();
    const int blocks = s.B * s.J * (s.R / TWC);
    CGRed r = red;
    r.nbase = blocks;   // one reducing block per item after the pass's blocks
    return launch_timed(w, k_cols_back<G, TWC, 0, S2, true>, dim3(blocks + s.B), dim3(TH), 0, st, (const void*)w.U2,
                        (const float2*)w.CO, xh, (const float2*)nullptr, (const double2*)w.tw, w.PR, w.U1, s.J,
                        (long long)s.X, r);
  }
  template <class S2>
  static hipError_t cg_cols_back_t(const Shape& s, const Bufs& w, hipStream_t st, const float2* xh,
                                   const CGRed& red) {
    return col_tile(s, false) == 4 ? cg_cols_back_k<S2, 4>(s, w, st, xh, red) : cg_cols_back_k<S2, TW>(s, w, st, xh, red);
  }
  static hipError_t cg_cols_back(const Shape& s, const Bufs& w, hipStream_t st, const float2* xh, const CGRed& red) {
    return cg_cols_back_t<double2>(s, w, st, xh, red);
  }
  static hipError_t cg_coilh(const Shape& s, const Bufs& w, hipStream_t st, const double2* pnew, float2* xh,
                             double alpha, double* rr_next, int first, int last) {
    const int blocks = s.B * (s.NX3 + s.NRQ);
    return launch_timed(w, k_cg_coilh<G>, dim3(blocks), dim3(TH_ROW1), 0, st, (const double2*)w.U1,
                        (const float*)w.dinv, (const double2*)w.tw, pnew, (const float2*)w.PR, w.H, w.Rv, xh, w.Vr,
                        (const double2*)w.scal, alpha, rr_next, s.stride, s.J, (long long)s.X, s.NX3, s.NRQ, first,
                        last);
  }
  static hipError_t psf_fft(const Shape& s, const Bufs& w, hipStream_t st, float* P, double scale) {
    k_fft_rows_full<G><<<G / ROWS, TH_ROWS, 0, st>>>(w.psf, w.tw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_fft_cols_psf<G><<<G / TW, TH_COLS, 0, st>>>(w.psf, P, w.tw, scale);
    return hipGetLastError();
  }
  template <class S2>
  static hipError_t kb_grid_t(const Shape& s, const Bufs& w, hipStream_t st, const TurnArgs& turns,
                              const float2* y, float2* z) {
    constexpr int RT = row_lines<G>();
    // the point counts live on the device (the tables are built there): the
    // short-row launch covers every grid point, the long-row one strides
    const long long rps = (long long)G * G + 1;
    k_kb_gather_short<G><<<dim3((G * G + VT - 1) / VT, s.B), VT, 0, st>>>(w.kbr, w.kbe, w.kbp, w.kbn, rps,
                                                                        s.kbe_stride, turns, y, w.KG, s.J, s.S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_kb_gather_long<G><<<dim3(KB_LONG_BLOCKS, s.B), VT, 0, st>>>(w.kbr, w.kbe, w.kbp, w.kbn, rps, s.kbe_stride,
                                                                  turns, y, w.KG, s.J, s.S);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nlines = s.B * s.J * G;
    k_kb_rows<G, S2><<<(nlines + RT - 1) / RT, TH_ROW1, 0, st>>>(w.KG, static_cast<S2*>(w.U2), w.tw, nlines);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_kb_cols<G, S2><<<s.B * s.J * s.NT, TH_COLS, 0, st>>>(static_cast<const S2*>(w.U2), w.kbc, w.tw, z);
    return hipGetLastError();
  }
  static hipError_t kb_grid(const Shape& s, const Bufs& w, hipStream_t st, const TurnArgs& turns,
                            const float2* y, float2* z) {
    return kb_grid_t<double2>(s, w, st, turns, y, z);
  }
};

template <int G>
constexpr GTable make_table() {
  return GTable{&GLaunch<G>::coil_rows, &GLaunch<G>::coil_rows_cg, &GLaunch<G>::cols_fwd,
                &GLaunch<G>::toep_rows, &GLaunch<G>::cols_back, &GLaunch<G>::coilh_rows,
                &GLaunch<G>::cg_cols_fwd, &GLaunch<G>::cg_toep_rows, &GLaunch<G>::cg_cols_back,
                &GLaunch<G>::cg_coilh, &GLaunch<G>::psf_fft, &GLaunch<G>::kb_grid, row_lines<G>(),
                row_lines<G + GKEY>()};
}

}  // namespace nlv
