// Grid-size independent kernels of the NLINV hot path (gfx950): the CG vector
// updates and FP64 reductions, output assembly, and the exact non-uniform DFT
// sums (gridding, PSF lags, forward transform); plus the dispatch to the
// per-grid-size launch tables.
#include "nlinv_kernels.h"

namespace nlv {

const GTable* table_g64();
const GTable* table_g128();
const GTable* table_g256();
const GTable* table_g320();
const GTable* table_g384();
const GTable* table_g432();
const GTable* table_g448();
const GTable* table_g480();
const GTable* table_g512();

const GTable* table_for(int G) {
  switch (G) {
    case 64: return table_g64();
    case 128: return table_g128();
    case 256: return table_g256();
    case 320: return table_g320();
    case 384: return table_g384();
    case 432: return table_g432();
    case 448: return table_g448();
    case 480: return table_g480();
    case 512: return table_g512();
    default: return nullptr;
  }
}

__device__ __forceinline__ double2 ldv(const float2* __restrict__ p, size_t i) {
  const float2 v = p[i];
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 tof(double2 v) { return make_float2((float)v.x, (float)v.y); }

// CG step: a = rr / Re<p, q>; h += a p; r -= a q; rr' partials.  q is complete in Q
// (its image block formed by the q_rho blocks of the coil-adjoint rows).
// On the last iteration the Newton update x += h is applied instead of the r update.
// All element loads are issued before the scalar reductions so that their
// latencies overlap.
__global__ void __launch_bounds__(VT)
k_cg_update(const double2* __restrict__ Q, const double2* __restrict__ P, double2* __restrict__ H,
            double2* __restrict__ Rv, float2* __restrict__ xh, Partials rr, const double* __restrict__ pq,
            int npq, double* __restrict__ rr_next, int first, int last, long long X, int nchunk) {
  constexpr int EPT = CHUNK / VT;
  __shared__ double sh[VT];
  const int b = blockIdx.x / nchunk, c = blockIdx.x - b * nchunk;
  const long long e0 = (long long)c * CHUNK;
  double2 pv[EPT], hv[EPT], rv[EPT], qv[EPT];
  float2 xv[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const long long e = e0 + k * VT + threadIdx.x;
    pv[k] = hv[k] = rv[k] = qv[k] = make_double2(0.0, 0.0);
    xv[k] = make_float2(0.f, 0.f);
    if (e >= X) continue;
    const size_t ve = (size_t)b * X + e;
    pv[k] = P[ve];
    if (!first) hv[k] = H[ve];
    if (last) {
      xv[k] = xh[ve];
    } else {
      rv[k] = Rv[ve];
      qv[k] = Q[ve];
    }
  }
  const double2 sums = block_sum2_arrays_waves<VT>(pq + (size_t)b * rr.stride, npq,
                                                   rr.cur + (size_t)b * rr.stride, rr.ncur, sh);
  const double pqs = sums.x, rrs = sums.y;
  const double a = pqs != 0.0 ? rrs / pqs : 0.0;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const long long e = e0 + k * VT + threadIdx.x;
    if (e >= X) continue;
    const size_t ve = (size_t)b * X + e;
    const double hx = hv[k].x + a * pv[k].x, hy = hv[k].y + a * pv[k].y;
    if (last) {
      xh[ve] = make_float2((float)(xv[k].x + hx), (float)(xv[k].y + hy));
    } else {
      const double qx = qv[k].x, qy = qv[k].y;
      H[ve] = make_double2(hx, hy);
      const double2 rn = make_double2(rv[k].x - a * qx, rv[k].y - a * qy);
      Rv[ve] = rn;
      acc += rn.x * rn.x + rn.y * rn.y;
    }
  }
  if (!last) {
    const double s = block_sum_waves<VT>(acc, sh);
    if (threadIdx.x == 0) rr_next[(size_t)b * rr.stride + c] = s;
  }
}

template <class O> __device__ __forceinline__ O out_as(double x, double y);
template <> __device__ __forceinline__ float2 out_as<float2>(double x, double y) {
  return make_float2((float)x, (float)y);
}
template <> __device__ __forceinline__ double2 out_as<double2>(double x, double y) { return make_double2(x, y); }

// Assemble an operator result (complex64 or complex128 storage): image block
// sum_j PR_j + alpha p (p may be null), coil block copied from Q.
template <class O>
__global__ void __launch_bounds__(VT)
k_finalize(const float2* __restrict__ PR, const double2* __restrict__ p, double alpha,
           const double2* __restrict__ Q, O* __restrict__ out, int J, int RR, long long X,
           int nchunk) {
  const int b = blockIdx.x / nchunk, c = blockIdx.x - b * nchunk;
  const long long e0 = (long long)c * CHUNK;
  const long long e1 = e0 + CHUNK < X ? e0 + CHUNK : X;
  for (long long e = e0 + threadIdx.x; e < e1; e += VT) {
    const size_t ve = (size_t)b * X + e;
    if (e < RR) {
      double sx = 0.0, sy = 0.0;
      for (int j = 0; PR && j < J; ++j) {   // PR == nullptr: image block zero
        const float2 pr = PR[((size_t)b * J + j) * RR + e];
        sx += pr.x;
        sy += pr.y;
      }
      if (p) {
        const double2 pp = p[ve];
        sx += alpha * pp.x;
        sy += alpha * pp.y;
      }
      out[ve] = out_as<O>(sx, sy);
    } else {
      out[ve] = out_as<O>(Q[ve].x, Q[ve].y);
    }
  }
}

// dst = (double) src
__global__ void __launch_bounds__(VT)
k_to_double(double2* __restrict__ dst, const float2* __restrict__ src, long long n) {
  const long long e = (long long)blockIdx.x * VT + threadIdx.x;
  if (e < n) dst[e] = ldv(src, e);
}

// x = xprev (copy) for the "start from the previous frame" initialisation.
__global__ void __launch_bounds__(VT)
k_copy(float2* __restrict__ dst, const float2* __restrict__ src, long long n) {
  const long long e = (long long)blockIdx.x * VT + threadIdx.x;
  if (e < n) dst[e] = src[e];
}

// dst[b][k] = src[k] for every item b.
__global__ void __launch_bounds__(VT)
k_bcast(float2* __restrict__ dst, const float2* __restrict__ src, long long X, long long n) {
  const long long e = (long long)blockIdx.x * VT + threadIdx.x;
  if (e < n) dst[e] = src[e % X];
}

// x = (rho = 1, c_hat = 0) for every item.
__global__ void __launch_bounds__(VT)
k_init_unit(float2* __restrict__ xh, int RR, long long X, long long n) {
  const long long e = (long long)blockIdx.x * VT + threadIdx.x;
  if (e >= n) return;
  const long long k = e % X;
  xh[e] = k < RR ? make_float2(1.f, 0.f) : czero<float2>();
}

// img = |rho| sqrt(sum_j |c_j|^2)
__global__ void __launch_bounds__(VT)
k_image(const float2* __restrict__ xh, const float2* __restrict__ co, float* __restrict__ img,
        int J, int RR, long long X, int B) {
  const long long e = (long long)blockIdx.x * VT + threadIdx.x;
  if (e >= (long long)B * RR) return;
  const int b = (int)(e / RR), k = (int)(e - (long long)b * RR);
  double s = 0.0;
  for (int j = 0; j < J; ++j) {
    const float2 c = co[((size_t)b * J + j) * RR + k];
    s += (double)c.x * c.x + (double)c.y * c.y;
  }
  const float2 r = xh[(size_t)b * X + k];
  img[e] = (float)(sqrt((double)r.x * r.x + (double)r.y * r.y) * sqrt(s));
}

// ---------------------------------------------------------------------------
// exact non-uniform DFT: gridding (adjoint), forward, and the PSF lags
// ---------------------------------------------------------------------------

// exp(SIGN i 2 pi k m) for float k (cycles) and integer m, with the product's
// rounding error carried exactly (fma) and the integer cycles removed before
// the sincospi evaluation.
template <int SIGN>
__device__ __forceinline__ float2 cis_cycles(float k, int m) {
  const float fm = (float)m;
  const float p = k * fm;
  const float err = fmaf(k, fm, -p);
  const float f = (p - rintf(p)) + err;
  float s, c;
  sincospif(2.0f * f, &s, &c);
  return make_float2(c, SIGN > 0 ? s : -s);
}

constexpr int GSC = 64;   // samples per LDS stage
constexpr int GT = 16;    // pixel tile side (16 x 16 = 256 threads)

// Gridding, register-blocked: a block owns a 32 x 32 pixel tile and JG channels
// (the last tile row and column are partial when R is not a multiple of 32),
// each thread a 2 x 2 pixel patch; samples are staged in LDS 32 at a time
// (phase factors exp(+i 2 pi k x) and exp(+i 2 pi k y) per sample and tile row /
// column), float32 sums per stage are accumulated in float64.  With nsplit > 1
// the sample range is split over blocks and out receives nsplit partial grids
// [nsplit][B][J][R][R] that k_grid_reduce adds in a fixed order.
constexpr int GS2 = 32;
template <int JG>
__global__ void __launch_bounds__(VT)
k_grid2(const float* __restrict__ traj, const float2* __restrict__ yv, float2* __restrict__ out,
        int J, int S, int R, int B, int nsplit, float scale) {
  __shared__ __align__(16) float2 ex[GS2][32];
  __shared__ __align__(16) float2 ey[GS2][32];
  __shared__ float2 ys[JG][GS2];
  const int nt = (R + 31) / 32;
  const int ty0 = (blockIdx.x / nt) * 32, tx0 = (blockIdx.x % nt) * 32;
  const int jg = blockIdx.y;
  const int b = blockIdx.z / nsplit, sp = blockIdx.z - b * nsplit;
  const int per = (S + nsplit - 1) / nsplit;
  const int s_lo = sp * per, s_hi = min(S, s_lo + per);
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
  const float* tr = traj + (size_t)b * S * 2;
  double2 acc[JG][4];
#pragma unroll
  for (int q = 0; q < JG; ++q)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[q][k] = make_double2(0.0, 0.0);
  for (int s0 = s_lo; s0 < s_hi; s0 += GS2) {
    for (int q = threadIdx.x; q < GS2 * 32; q += VT) {
      const int ss = q / 32, pix = q % 32, s = s0 + ss;
      if (s < s_hi) {
        ex[ss][pix] = cis_cycles<+1>(tr[2 * s], tx0 + pix - R / 2);
        ey[ss][pix] = cis_cycles<+1>(tr[2 * s + 1], ty0 + pix - R / 2);
      } else {
        ex[ss][pix] = czero<float2>();
        ey[ss][pix] = czero<float2>();
      }
    }
    for (int q = threadIdx.x; q < JG * GS2; q += VT) {
      const int jj = q / GS2, ss = q % GS2, s = s0 + ss, j = jg * JG + jj;
      ys[jj][ss] = (s < s_hi && j < J) ? yv[((size_t)b * J + j) * S + s] : czero<float2>();
    }
    __syncthreads();
    float2 part[JG][4];
#pragma unroll
    for (int q = 0; q < JG; ++q)
#pragma unroll
      for (int k = 0; k < 4; ++k) part[q][k] = czero<float2>();
#pragma unroll 2
    for (int ss = 0; ss < GS2; ++ss) {
      const float4 xx = *reinterpret_cast<const float4*>(&ex[ss][2 * tx]);
      const float4 yy = *reinterpret_cast<const float4*>(&ey[ss][2 * ty]);
      const float2 ex0 = make_float2(xx.x, xx.y), ex1 = make_float2(xx.z, xx.w);
      const float2 ey0 = make_float2(yy.x, yy.y), ey1 = make_float2(yy.z, yy.w);
      float2 e[4];
      e[0] = cmul(ey0, ex0);
      e[1] = cmul(ey0, ex1);
      e[2] = cmul(ey1, ex0);
      e[3] = cmul(ey1, ex1);
#pragma unroll
      for (int q = 0; q < JG; ++q) {
        const float2 y = ys[q][ss];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          part[q][k].x += y.x * e[k].x - y.y * e[k].y;
          part[q][k].y += y.x * e[k].y + y.y * e[k].x;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < JG; ++q)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        acc[q][k].x += part[q][k].x;
        acc[q][k].y += part[q][k].y;
      }
    __syncthreads();
  }
  float2* o = out + (nsplit > 1 ? (size_t)sp * B * J * R * R : 0);
#pragma unroll
  for (int q = 0; q < JG; ++q) {
    const int j = jg * JG + q;
    if (j >= J) continue;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int y = ty0 + 2 * ty + (k >> 1), x = tx0 + 2 * tx + (k & 1);
      if (y < R && x < R)
        o[(((size_t)b * J + j) * R + y) * R + x] =
            make_float2((float)(acc[q][k].x * scale), (float)(acc[q][k].y * scale));
    }
  }
}

// z = sum over the nsplit partial grids (fixed order, float64 sum)
__global__ void __launch_bounds__(VT)
k_grid_reduce(const float2* __restrict__ part, float2* __restrict__ z, long long n, int nsplit) {
  const long long e = (long long)blockIdx.x * VT + threadIdx.x;
  if (e >= n) return;
  double sx = 0.0, sy = 0.0;
  for (int k = 0; k < nsplit; ++k) {
    const float2 v = part[(size_t)k * n + e];
    sx += v.x;
    sy += v.y;
  }
  z[e] = make_float2((float)sx, (float)sy);
}

// psf[n_y][n_x] = sum_s exp(+i 2 pi k_s . d), d = n or n - G, kept for |d| <= R-1, else 0.
__global__ void __launch_bounds__(VT)
k_psf_lags(const float* __restrict__ traj, double2* __restrict__ psf, int S, int R, int G) {
  __shared__ float2 ex[GSC][GT], ey[GSC][GT];
  const int nt = G / GT;
  const int ty0 = (blockIdx.x / nt) * GT, tx0 = (blockIdx.x % nt) * GT;
  const int py = threadIdx.x / GT, px = threadIdx.x % GT;
  auto lag = [&](int n) { return n < G / 2 ? n : n - G; };
  double2 acc = make_double2(0.0, 0.0);
  for (int s0 = 0; s0 < S; s0 += GSC) {
    for (int q = threadIdx.x; q < GSC * GT; q += VT) {
      const int ss = q / GT, pix = q % GT, s = s0 + ss;
      if (s < S) {
        ex[ss][pix] = cis_cycles<+1>(traj[2 * s], lag(tx0 + pix));
        ey[ss][pix] = cis_cycles<+1>(traj[2 * s + 1], lag(ty0 + pix));
      } else {
        ex[ss][pix] = czero<float2>();
        ey[ss][pix] = czero<float2>();
      }
    }
    __syncthreads();
    float2 part = czero<float2>();
#pragma unroll 4
    for (int ss = 0; ss < GSC; ++ss) part = cadd(part, cmul(ey[ss][py], ex[ss][px]));
    acc.x += part.x;
    acc.y += part.y;
    __syncthreads();
  }
  const int dy = lag(ty0 + py), dx = lag(tx0 + px);
  const bool keep = dy >= -(R - 1) && dy <= R - 1 && dx >= -(R - 1) && dx <= R - 1;
  psf[(size_t)(ty0 + py) * G + tx0 + px] = keep ? acc : make_double2(0.0, 0.0);
}

// y[b][j][s] = scale sum_{y,x} u[b][j][y][x] exp(-i 2 pi (kx_s x + ky_s y))
constexpr int FXC = 32;           // x chunk
constexpr int NUDFT_MAXR = 256;   // largest field of view (64 KB of LDS per block)
__global__ void __launch_bounds__(VT)
k_nudft_fwd(const float* __restrict__ traj, const float2* __restrict__ u, float2* __restrict__ yv,
            int J, int S, int R, float scale) {
  __shared__ float2 uc[NUDFT_MAXR * FXC];
  const int s = blockIdx.x * VT + threadIdx.x;
  const int j = blockIdx.y, b = blockIdx.z;
  const bool valid = s < S;
  const float kx = valid ? traj[((size_t)b * S + s) * 2] : 0.f;
  const float ky = valid ? traj[((size_t)b * S + s) * 2 + 1] : 0.f;
  const float2* ub = u + ((size_t)b * J + j) * R * R;
  double2 acc = make_double2(0.0, 0.0);
  for (int x0 = 0; x0 < R; x0 += FXC) {
    __syncthreads();
    for (int q = threadIdx.x; q < R * FXC; q += VT) {
      const int yy = q / FXC, xx = q % FXC;   // columns past R (last chunk) are zero
      uc[q] = x0 + xx < R ? ub[(size_t)yy * R + x0 + xx] : czero<float2>();
    }
    __syncthreads();
    float2 exv[FXC];
#pragma unroll
    for (int xx = 0; xx < FXC; ++xx) exv[xx] = cis_cycles<-1>(kx, x0 + xx - R / 2);
    for (int yy = 0; yy < R; ++yy) {
      float2 a = czero<float2>();
#pragma unroll
      for (int xx = 0; xx < FXC; ++xx) {
        const float2 uv = uc[yy * FXC + xx];
        a.x += uv.x * exv[xx].x - uv.y * exv[xx].y;
        a.y += uv.x * exv[xx].y + uv.y * exv[xx].x;
      }
      const float2 t = cmul(cis_cycles<-1>(ky, yy - R / 2), a);
      acc.x += t.x;
      acc.y += t.y;
    }
  }
  if (valid) yv[((size_t)b * J + j) * S + s] = make_float2((float)(acc.x * scale), (float)(acc.y * scale));
}


// flag |= 1 when any of the n complex values is NaN or infinite (a NaN fails
// the comparison, an infinity exceeds the largest float)
__global__ void __launch_bounds__(VT)
k_check_finite(const float2* __restrict__ x, long long n, int* __restrict__ flag) {
  bool bad = false;
  for (long long i = (long long)blockIdx.x * VT + threadIdx.x; i < n; i += (long long)gridDim.x * VT) {
    const float2 v = x[i];
    bad |= !(fabsf(v.x) <= 3.402823466e38f && fabsf(v.y) <= 3.402823466e38f);
  }
  if (bad) atomicOr(flag, 1);
}

// p[0] = v (a one-thread fill kernel instead of hipMemsetAsync, so that the
// clear is an ordinary kernel node wherever the call is enqueued)
__global__ void k_fill_int(int* __restrict__ p, int v) {
  if (threadIdx.x == 0) p[0] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_fill_int(hipStream_t st, int* p, int v) {
  k_fill_int<<<1, 64, 0, st>>>(p, v);
  return hipGetLastError();
}

hipError_t launch_cg_update(const Shape& s, const Bufs& w, hipStream_t st, int iter, int last,
                            const double2* p, Partials rr, float2* xh) {
  double* next = w.rr[(iter + 1) & 1];
  return launch_timed(w, k_cg_update, dim3(s.B * s.NCH), dim3(VT), 0, st, (const double2*)w.Q, p, w.H, w.Rv,
                      xh, rr, (const double*)w.pq, s.NX3 + s.NRQ, next, (int)(iter == 0), last,
                      (long long)s.X, s.NCH);
}

// Channel compression y[b][j][s] = sum_p cc[j][p] yp[b][p][s]: one thread per
// sample, the matrix in LDS, FP64 sums over the receive channels.
constexpr int CJ = 16;   // virtual channels per register pass
__global__ void __launch_bounds__(VT)
k_compress(const float2* __restrict__ cc, const float2* __restrict__ yp, float2* __restrict__ y, int J, int Jp,
           int S) {
  extern __shared__ float2 scc[];                 // [J][Jp]
  for (int i = threadIdx.x; i < J * Jp; i += VT) scc[i] = cc[i];
  __syncthreads();
  const int s = blockIdx.x * VT + threadIdx.x, b = blockIdx.y;
  if (s >= S) return;
  const float2* src = yp + (size_t)b * Jp * S + s;
  for (int j0 = 0; j0 < J; j0 += CJ) {
    const int nj = J - j0 < CJ ? J - j0 : CJ;
    double2 acc[CJ];
#pragma unroll
    for (int c = 0; c < CJ; ++c) acc[c] = make_double2(0.0, 0.0);
    for (int p = 0; p < Jp; ++p) {
      const float2 v = src[(size_t)p * S];
#pragma unroll
      for (int c = 0; c < CJ; ++c) {
        if (c < nj) {
          const float2 m = scc[(j0 + c) * Jp + p];
          acc[c].x += (double)m.x * v.x - (double)m.y * v.y;
          acc[c].y += (double)m.x * v.y + (double)m.y * v.x;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CJ; ++c)
      if (c < nj) y[((size_t)b * J + j0 + c) * S + s] = make_float2((float)acc[c].x, (float)acc[c].y);
  }
}

// Channel covariance cov[p][q] = sum_s y0[p][s] conj(y0[q][s]) (FP64, fixed order).
__global__ void __launch_bounds__(VT)
k_channel_cov(const float2* __restrict__ y0, double2* __restrict__ cov, int Jp, int S) {
  __shared__ double sh[2 * VT];
  const int p = blockIdx.x / Jp, q = blockIdx.x % Jp;
  double sr = 0.0, si = 0.0;
  for (int s = threadIdx.x; s < S; s += VT) {
    const float2 a = y0[(size_t)p * S + s], c = y0[(size_t)q * S + s];
    sr += (double)a.x * c.x + (double)a.y * c.y;
    si += (double)a.y * c.x - (double)a.x * c.y;
  }
  const double2 t = block_sum2_waves<VT>(sr, si, sh);
  if (threadIdx.x == 0) cov[blockIdx.x] = t;
}

hipError_t launch_compress(const Shape& s, hipStream_t st, const float2* cc, int Jp, const float2* yp, float2* y) {
  dim3 grid((s.S + VT - 1) / VT, s.B);
  k_compress<<<grid, VT, (size_t)s.J * Jp * sizeof(float2), st>>>(cc, yp, y, s.J, Jp, s.S);
  return hipGetLastError();
}

hipError_t launch_channel_cov(const Shape& s, hipStream_t st, const float2* y0, int Jp, double2* cov) {
  k_channel_cov<<<Jp * Jp, VT, 0, st>>>(y0, cov, Jp, s.S);
  return hipGetLastError();
}

// Eigen-decomposition of the n x n Hermitian channel covariance by parallel
// cyclic Jacobi rotations in one block (n <= MAX_JP): each element a_pq =
// |a_pq| e^{i phi} is removed by U = diag(1, e^{-i phi}) R(theta), which
// turns the 2 x 2 block real and rotates it diagonal (the classical Jacobi
// method, Golub and Van Loan, Matrix Computations, Sec. 8.5, after the phase
// change).  A sweep visits every pair once in n' - 1 rounds of n'/2 disjoint
// pairs (n' = n rounded up to even; the round-robin order), and the rotations
// of a round, which touch disjoint rows and columns, are applied together.
// Sweeps stop when the off-diagonal mass is below 1e-30 of the diagonal's, or
// after 100.  Then the rows of cc [J][n] are the conjugated eigenvectors of
// the J largest eigenvalues, in descending order (ties: lower index first).
constexpr int EIG_T = 1024;

__global__ void __launch_bounds__(EIG_T)
k_herm_jacobi(double2* __restrict__ A, double2* __restrict__ V, int n, int J, float2* __restrict__ cc) {
  __shared__ double rot[MAX_JP / 2][6];     // per pair: c, s, e^{-i phi} (re, im), p, q
  __shared__ double red[2][EIG_T / 64];
  __shared__ int order[MAX_JP];
  __shared__ int stop;
  const int t = threadIdx.x;
  const int m = n + (n & 1), half = m / 2;
  for (int i = t; i < n * n; i += EIG_T) V[i] = make_double2((i / n) == (i % n) ? 1.0 : 0.0, 0.0);
  __syncthreads();
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, dg = 0.0;
    for (int i = t; i < n * n; i += EIG_T) {
      const int r = i / n, c = i % n;
      const double v = A[i].x * A[i].x + A[i].y * A[i].y;
      if (c > r) off += v;
      if (c == r) dg += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_down(off, o, 64);
      dg += __shfl_down(dg, o, 64);
    }
    if ((t & 63) == 0) {
      red[0][t >> 6] = off;
      red[1][t >> 6] = dg;
    }
    __syncthreads();
    if (t == 0) {
      double so = 0.0, sd = 0.0;
      for (int w = 0; w < EIG_T / 64; ++w) {
        so += red[0][w];
        sd += red[1][w];
      }
      stop = so <= 1e-30 * (sd + 1e-300);
    }
    __syncthreads();
    if (stop) break;
    for (int r = 0; r < m - 1; ++r) {
      if (t < half) {
        int p = t == 0 ? m - 1 : (r + t) % (m - 1);
        int q = t == 0 ? r : (r - t + m - 1) % (m - 1);
        if (p > q) {
          const int u = p;
          p = q;
          q = u;
        }
        double c = 1.0, sn = 0.0, er = 1.0, ei = 0.0;
        bool live = false;                        // a real pair with a nonzero element
        if (q < n) {
          const double2 apq = A[p * n + q];
          const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
          if (mag > 0.0) {
            live = true;
            er = apq.x / mag;                     // e^{-i phi} = conj(a_pq) / |a_pq|
            ei = -apq.y / mag;
            const double app = A[p * n + p].x, aqq = A[q * n + q].x;
            const double tau = (aqq - app) / (2.0 * mag);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            sn = tt * c;
          }
        }
        rot[t][0] = c;
        rot[t][1] = sn;
        rot[t][2] = er;
        rot[t][3] = ei;
        rot[t][4] = p;
        rot[t][5] = live ? q : -1;
      }
      __syncthreads();
      // A <- A U and V <- V U: columns p, q of every row k
      for (int i = t; i < n * half; i += EIG_T) {
        const int k = i / half, j = i % half;
        const int q = (int)rot[j][5];
        if (q < 0) continue;
        const int p = (int)rot[j][4];
        const double c = rot[j][0], sn = rot[j][1], er = rot[j][2], ei = rot[j][3];
        // column p of U: (c, -s e^{-i phi}); column q: (s, c e^{-i phi})
        const double2 upq = make_double2(-sn * er, -sn * ei), uqq = make_double2(c * er, c * ei);
        for (int w = 0; w < 2; ++w) {
          double2* M = w ? V : A;
          const double2 akp = M[k * n + p], akq = M[k * n + q];
          M[k * n + p] = make_double2(akp.x * c + akq.x * upq.x - akq.y * upq.y, akp.y * c + akq.x * upq.y + akq.y * upq.x);
          M[k * n + q] = make_double2(akp.x * sn + akq.x * uqq.x - akq.y * uqq.y, akp.y * sn + akq.x * uqq.y + akq.y * uqq.x);
        }
      }
      __syncthreads();
      // A <- U^H A: rows p, q of every column k
      for (int i = t; i < n * half; i += EIG_T) {
        const int k = i / half, j = i % half;
        const int q = (int)rot[j][5];
        if (q < 0) continue;
        const int p = (int)rot[j][4];
        const double c = rot[j][0], sn = rot[j][1], er = rot[j][2], ei = rot[j][3];
        // conj(U) entries: conj(-s e^{-i phi}), conj(c e^{-i phi})
        const double2 cpq = make_double2(-sn * er, sn * ei), cqq = make_double2(c * er, -c * ei);
        const double2 apk = A[p * n + k], aqk = A[q * n + k];
        A[p * n + k] = make_double2(c * apk.x + cpq.x * aqk.x - cpq.y * aqk.y, c * apk.y + cpq.x * aqk.y + cpq.y * aqk.x);
        A[q * n + k] = make_double2(sn * apk.x + cqq.x * aqk.x - cqq.y * aqk.y, sn * apk.y + cqq.x * aqk.y + cqq.y * aqk.x);
      }
      __syncthreads();
      if (t < half) {
        const int q = (int)rot[t][5];
        if (q >= 0) {
          const int p = (int)rot[t][4];
          A[p * n + q] = make_double2(0.0, 0.0);
          A[q * n + p] = make_double2(0.0, 0.0);
        }
      }
      __syncthreads();
    }
  }
  if (t == 0) {
    // the J largest eigenvalues, descending; ties keep the lower index first
    unsigned long long used[(MAX_JP + 63) / 64] = {};
    for (int j = 0; j < J; ++j) {
      int best = -1;
      for (int i = 0; i < n; ++i) {
        if ((used[i >> 6] >> (i & 63)) & 1ull) continue;
        if (best < 0 || A[i * n + i].x > A[best * n + best].x) best = i;
      }
      used[best >> 6] |= 1ull << (best & 63);
      order[j] = best;
    }
  }
  __syncthreads();
  for (int i = t; i < J * n; i += EIG_T) {
    const int j = i / n, p = i % n;
    const double2 v = V[p * n + order[j]];
    cc[i] = make_float2((float)v.x, (float)-v.y);
  }
}

hipError_t launch_compression_eig(hipStream_t st, double2* A, double2* V, int n, int J, float2* cc) {
  if (n < 1 || n > MAX_JP || J < 1 || J > n) return hipErrorInvalidValue;
  k_herm_jacobi<<<1, EIG_T, 0, st>>>(A, V, n, J, cc);
  return hipGetLastError();
}

hipError_t launch_finalize(const Shape& s, const Bufs& w, hipStream_t st, const double2* p,
                           double alpha, float2* out, bool image_block) {
  k_finalize<float2><<<s.B * s.NCH, VT, 0, st>>>(image_block ? w.PR : nullptr, p, alpha, w.Q, out, s.J,
                                                 s.R * s.R, s.X, s.NCH);
  return hipGetLastError();
}

hipError_t launch_finalize(const Shape& s, const Bufs& w, hipStream_t st, const double2* p,
                           double alpha, double2* out, bool image_block) {
  k_finalize<double2><<<s.B * s.NCH, VT, 0, st>>>(image_block ? w.PR : nullptr, p, alpha, w.Q, out, s.J,
                                                  s.R * s.R, s.X, s.NCH);
  return hipGetLastError();
}

hipError_t launch_to_double(const Shape& s, hipStream_t st, double2* dst, const float2* src) {
  const long long n = (long long)s.B * s.X;
  k_to_double<<<(int)((n + VT - 1) / VT), VT, 0, st>>>(dst, src, n);
  return hipGetLastError();
}

hipError_t launch_init_x(const Shape& s, hipStream_t st, float2* xh, const float2* xprev, int mode) {
  const long long n = (long long)s.B * s.X;
  const int blocks = (int)((n + VT - 1) / VT);
  if (mode == 2) {
    k_copy<<<blocks, VT, 0, st>>>(xh, xprev, n);
  } else if (mode == 3) {
    k_bcast<<<blocks, VT, 0, st>>>(xh, xprev, s.X, n);
  } else {
    k_init_unit<<<blocks, VT, 0, st>>>(xh, s.R * s.R, s.X, n);
  }
  return hipGetLastError();
}

hipError_t launch_image(const Shape& s, hipStream_t st, const float2* xh, const float2* co, float* img) {
  const long long n = (long long)s.B * s.R * s.R;
  k_image<<<(int)((n + VT - 1) / VT), VT, 0, st>>>(xh, co, img, s.J, s.R * s.R, s.X, s.B);
  return hipGetLastError();
}

int grid_jg(int J) {
  if (J % 5 == 0) return 5;
  if (J % 4 == 0) return 4;
  if (J % 3 == 0) return 3;
  if (J % 2 == 0) return 2;
  return J >= 4 ? 4 : 1;
}

int grid_nsplit(int B, int J, int R) {
  const long long nt = (R + 31) / 32;
  const long long blocks = nt * nt * ((J + grid_jg(J) - 1) / grid_jg(J)) * B;
  int n = 1;
  while (n < 8 && blocks * n < 512) n *= 2;
  return n;
}

hipError_t launch_grid(const Shape& s, const Bufs& w, hipStream_t st, const float* traj, const float2* y,
                       float2* z) {
  const int JG = grid_jg(s.J);
  const int nsplit = s.gsplit;
  float2* out = nsplit > 1 ? w.GS : z;
  const int nt = (s.R + 31) / 32;
  dim3 grid(nt * nt, (s.J + JG - 1) / JG, s.B * nsplit);
  const float scale = 1.0f / s.R;
  switch (JG) {
    case 5: k_grid2<5><<<grid, VT, 0, st>>>(traj, y, out, s.J, s.S, s.R, s.B, nsplit, scale); break;
    case 4: k_grid2<4><<<grid, VT, 0, st>>>(traj, y, out, s.J, s.S, s.R, s.B, nsplit, scale); break;
    case 3: k_grid2<3><<<grid, VT, 0, st>>>(traj, y, out, s.J, s.S, s.R, s.B, nsplit, scale); break;
    case 2: k_grid2<2><<<grid, VT, 0, st>>>(traj, y, out, s.J, s.S, s.R, s.B, nsplit, scale); break;
    default: k_grid2<1><<<grid, VT, 0, st>>>(traj, y, out, s.J, s.S, s.R, s.B, nsplit, scale); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nsplit == 1) return e;
  const long long n = (long long)s.B * s.J * s.R * s.R;
  k_grid_reduce<<<(int)((n + VT - 1) / VT), VT, 0, st>>>(w.GS, z, n, nsplit);
  return hipGetLastError();
}

hipError_t launch_check_finite(hipStream_t st, const float2* x, long long n, int* flag) {
  const long long want = (n + VT - 1) / VT;
  const int blocks = (int)(want < 1024 ? (want < 1 ? 1 : want) : 1024);
  k_check_finite<<<blocks, VT, 0, st>>>(x, n, flag);
  return hipGetLastError();
}

hipError_t launch_nudft_fwd(const Shape& s, hipStream_t st, const float* traj, const float2* u,
                            float2* y) {
  if (s.R > NUDFT_MAXR) return hipErrorInvalidValue;
  dim3 grid((s.S + VT - 1) / VT, s.J, s.B);
  k_nudft_fwd<<<grid, VT, 0, st>>>(traj, u, y, s.J, s.S, s.R, 1.0f / s.R);
  return hipGetLastError();
}

hipError_t launch_psf(const Shape& s, const Bufs& w, hipStream_t st, const float* traj, int S, int turn) {
  const GTable* t = table_for(s.G);
  if (!t || S < 1 || S > s.S) return hipErrorInvalidValue;
  const int nt = (s.G / GT) * (s.G / GT);
  k_psf_lags<<<nt, VT, 0, st>>>(traj, w.psf, S, s.R, s.G);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // F^H F = (1/R^2) psf-convolution; the unnormalised 2D DFT pair contributes 1/G^2
  const double scale = 1.0 / ((double)s.G * s.G * (double)s.R * s.R);
  return t->psf_fft(s, w, st, w.P + (size_t)turn * s.G * s.G, scale);
}

// ---------------------------------------------------------------------------
// Kaiser-Bessel gridding table of one turn, built on the device: for every
// grid point p = uy * G + ux of the G x G grid (DC at 0, periodic) the samples
// s whose kernel reaches it (within half a kernel width on both axes), with
// the weights phi(ux - G kx_s) phi(uy - G ky_s) rounded to float32, in sample
// order; and the grid points split into short rows (at most KB_SHORT
// entries, ascending from the front of the point list) and long rows
// (ascending from its back).  Count, scan, fill, then a sort of every row by
// sample index, so the table does not depend on the order in which the
// fill's atomics land.
// ---------------------------------------------------------------------------

// visit(p, w) for every grid point that sample s reaches.
template <class F>
__device__ inline void kb_taps(const float* __restrict__ traj, int s, int G, double beta, F visit) {
  const double x = (double)G * traj[2 * s], y = (double)G * traj[2 * s + 1];
  const int ux0 = (int)ceil(x - 0.5 * KB_W), uy0 = (int)ceil(y - 0.5 * KB_W);
  double wx[KB_TAPS], wy[KB_TAPS];
#pragma unroll
  for (int a = 0; a < KB_TAPS; ++a) {
    wx[a] = kb_phi(ux0 + a - x, beta);
    wy[a] = kb_phi(uy0 + a - y, beta);
  }
  for (int by = 0; by < KB_TAPS; ++by) {
    if (wy[by] == 0.0) continue;
    const int py = ((uy0 + by) % G + G) % G;
    for (int bx = 0; bx < KB_TAPS; ++bx) {
      if (wx[bx] == 0.0) continue;
      const int px = ((ux0 + bx) % G + G) % G;
      visit(py * G + px, (float)(wy[by] * wx[bx]));
    }
  }
}

__global__ void __launch_bounds__(VT) k_fill_ints(int* __restrict__ p, long long n, int v) {
  for (long long i = (long long)blockIdx.x * VT + threadIdx.x; i < n; i += (long long)gridDim.x * VT) p[i] = v;
}

// entries per grid point: cnt[p] += 1 per tap
__global__ void __launch_bounds__(VT)
k_kb_count(const float* __restrict__ traj, int S, int G, double beta, int* __restrict__ cnt) {
  const int s = blockIdx.x * VT + threadIdx.x;
  if (s >= S) return;
  kb_taps(traj, s, G, beta, [&](int p, float) { atomicAdd(&cnt[p], 1); });
}

// One block: rp[1..GG] counts -> row ends (inclusive sums), the point list and
// the (short, long) point counts.  Thread t owns the points of one contiguous
// chunk; exclusive block scans of the chunk sums give its offsets.
constexpr int KB_SCAN_T = 1024;

__global__ void __launch_bounds__(KB_SCAN_T)
k_kb_scan(int* __restrict__ rp, int* __restrict__ pts, int2* __restrict__ counts, int GG) {
  __shared__ int sh[2][KB_SCAN_T];
  const int t = threadIdx.x;
  const int chunk = (GG + KB_SCAN_T - 1) / KB_SCAN_T;
  const int p0 = min(GG, t * chunk), p1 = min(GG, p0 + chunk);
  int sum = 0, nshort = 0;
  for (int p = p0; p < p1; ++p) {
    const int c = rp[p + 1];
    sum += c;
    nshort += c <= KB_SHORT;
  }
  sh[0][t] = sum;
  sh[1][t] = nshort;
  __syncthreads();
  for (int off = 1; off < KB_SCAN_T; off <<= 1) {
    const int a = t >= off ? sh[0][t - off] : 0, b = t >= off ? sh[1][t - off] : 0;
    __syncthreads();
    sh[0][t] += a;
    sh[1][t] += b;
    __syncthreads();
  }
  int end = sh[0][t] - sum;              // entries before p0
  int qs = sh[1][t] - nshort;            // short points before p0
  int ql = p0 - qs;                      // long points before p0
  for (int p = p0; p < p1; ++p) {
    const int c = rp[p + 1];
    end += c;
    rp[p + 1] = end;
    if (c <= KB_SHORT) pts[qs++] = p;
    else pts[GG - 1 - ql++] = p;
  }
  if (t == 0) {
    const int ns = sh[1][KB_SCAN_T - 1];
    rp[0] = 0;
    counts[0] = make_int2(ns, GG - ns);
  }
}

// entries into their rows, in arrival order
__global__ void __launch_bounds__(VT)
k_kb_fill(const float* __restrict__ traj, int S, int G, double beta, const int* __restrict__ rp,
          int* __restrict__ cur, int2* __restrict__ stage) {
  const int s = blockIdx.x * VT + threadIdx.x;
  if (s >= S) return;
  kb_taps(traj, s, G, beta, [&](int p, float wt) {
    const int k = rp[p] + atomicAdd(&cur[p], 1);
    stage[k] = make_int2(s, __float_as_int(wt));
  });
}

// short rows: one thread each, odd-even transposition sort in registers
__global__ void __launch_bounds__(VT)
k_kb_sort_short(const int* __restrict__ rp, const int2* __restrict__ stage, int2* __restrict__ ent, int GG) {
  const int p = blockIdx.x * VT + threadIdx.x;
  if (p >= GG) return;
  const int e0 = rp[p], n = rp[p + 1] - e0;
  if (n > KB_SHORT) return;
  int2 v[KB_SHORT];
#pragma unroll
  for (int k = 0; k < KB_SHORT; ++k) v[k] = k < n ? stage[e0 + k] : make_int2(0x7fffffff, 0);
#pragma unroll
  for (int r = 0; r < KB_SHORT; ++r) {
#pragma unroll
    for (int k = r & 1; k + 1 < KB_SHORT; k += 2) {
      if (v[k].x > v[k + 1].x) {
        const int2 tmp = v[k];
        v[k] = v[k + 1];
        v[k + 1] = tmp;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < KB_SHORT; ++k)
    if (k < n) ent[e0 + k] = v[k];
}

// long rows: one wavefront each (grid-stride over the long points), every
// entry placed at its rank (sample indices of a row are distinct)
__global__ void __launch_bounds__(VT)
k_kb_sort_long(const int* __restrict__ rp, const int* __restrict__ pts, const int2* __restrict__ counts,
               const int2* __restrict__ stage, int2* __restrict__ ent, int GG) {
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * (VT / 64);
  const int nl = counts[0].y;
  for (int q = blockIdx.x * (VT / 64) + (int)(threadIdx.x >> 6); q < nl; q += nw) {
    const int p = pts[GG - 1 - q];
    const int e0 = rp[p], n = rp[p + 1] - e0;
    for (int i0 = 0; i0 < n; i0 += 64) {
      const int i = i0 + lane;
      const int2 v = i < n ? stage[e0 + i] : make_int2(0, 0);
      int rank = 0;
      for (int j = 0; j < n; ++j) rank += stage[e0 + j].x < v.x;
      if (i < n) ent[e0 + rank] = v;
    }
  }
}

hipError_t launch_kb_table(const Shape& s, const Bufs& w, hipStream_t st, const float* traj, int S, int turn) {
  if (!s.kb || S < 1 || S > s.S || turn < 0 || turn >= s.U) return hipErrorInvalidValue;
  const int G = s.G, GG = G * G;
  int* rp = w.kbr + (size_t)turn * ((size_t)GG + 1);
  int2* ent = w.kbe + (size_t)turn * s.kbe_stride;
  int* pts = w.kbp + (size_t)turn * GG;
  const double beta = kb_beta();
  const int fb = (GG + 1 + VT - 1) / VT < 1024 ? (GG + 1 + VT - 1) / VT : 1024;
  k_fill_ints<<<fb, VT, 0, st>>>(rp, (long long)GG + 1, 0);
  k_fill_ints<<<fb, VT, 0, st>>>(w.kbq, (long long)GG, 0);
  k_kb_count<<<(S + VT - 1) / VT, VT, 0, st>>>(traj, S, G, beta, rp + 1);
  k_kb_scan<<<1, KB_SCAN_T, 0, st>>>(rp, pts, w.kbn + turn, GG);
  k_kb_fill<<<(S + VT - 1) / VT, VT, 0, st>>>(traj, S, G, beta, rp, w.kbq, w.kbs);
  k_kb_sort_short<<<(GG + VT - 1) / VT, VT, 0, st>>>(rp, w.kbs, ent, GG);
  k_kb_sort_long<<<KB_LONG_BLOCKS, VT, 0, st>>>(rp, pts, w.kbn + turn, w.kbs, ent, GG);
  return hipGetLastError();
}

// The ragged Toeplitz row pass over plans of the grid sides 256, 320 and 384
// (slot k holds the plan of grid 256, 320 or 384; nlines = 0 for an absent
// one): one persistent launch over the shapes' tiles.
hipError_t launch_toep_ragged(hipStream_t st, const ToepShape (&shapes)[3]) {
  const int tiles = (shapes[0].nlines + row_lines<256>() - 1) / row_lines<256>() +
                    (shapes[1].nlines + row_lines<320>() - 1) / row_lines<320>() +
                    (shapes[2].nlines + row_lines<384>() - 1) / row_lines<384>();
  if (tiles == 0) return hipSuccess;
  // enough resident blocks to fill the GPU (about 8 per CU at this block's LDS size)
  constexpr int RESIDENT = 2048;
  const int blocks = tiles < RESIDENT ? tiles : RESIDENT;
  k_toep_rows_ragged<256, 320, 384><<<blocks, 64, 0, st>>>(shapes[0], shapes[1], shapes[2]);
  return hipGetLastError();
}

}  // namespace nlv
