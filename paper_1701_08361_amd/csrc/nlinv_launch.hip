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
const GTable* table_g448();

const GTable* table_for(int G) {
  switch (G) {
    case 64: return table_g64();
    case 128: return table_g128();
    case 256: return table_g256();
    case 320: return table_g320();
    case 384: return table_g384();
    case 448: return table_g448();
    default: return nullptr;
  }
}

__device__ __forceinline__ double2 ldv(const float2* __restrict__ p, size_t i) {
  const float2 v = p[i];
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 tof(double2 v) { return make_float2((float)v.x, (float)v.y); }

// Image block of the Newton right-hand side: b_rho = sum_j PR_j - alpha (rho - rho_prev);
// r = p = b_rho; partials |b_rho|^2 -> rr0[b][slot_off + chunk].
__global__ void __launch_bounds__(VT)
k_cg_init(const float2* __restrict__ PR, const float2* __restrict__ xh, const float2* __restrict__ xprev,
          double alpha, double2* __restrict__ Rv, double2* __restrict__ P0, double* __restrict__ rr0,
          int stride, int slot_off, int J, int RR, long long X, int nchunk) {
  __shared__ double sh[VT];
  const int b = blockIdx.x / nchunk, c = blockIdx.x - b * nchunk;
  const int e0 = c * CHUNK, e1 = min(RR, e0 + CHUNK);
  double acc = 0.0;
  for (int e = e0 + threadIdx.x; e < e1; e += VT) {
    double sx = 0.0, sy = 0.0;
    for (int j = 0; j < J; ++j) {
      const float2 pr = PR[((size_t)b * J + j) * RR + e];
      sx += pr.x;
      sy += pr.y;
    }
    const size_t ve = (size_t)b * X + e;
    const float2 rho = xh[ve];
    const float2 rp = xprev ? xprev[ve] : make_float2(1.f, 0.f);
    const double2 bv = make_double2(sx - alpha * ((double)rho.x - rp.x), sy - alpha * ((double)rho.y - rp.y));
    Rv[ve] = bv;
    P0[ve] = bv;
    acc += bv.x * bv.x + bv.y * bv.y;
  }
  const double s = block_sum<VT>(acc, sh);
  if (threadIdx.x == 0) rr0[(size_t)b * stride + slot_off + c] = s;
}

// CG step: a = rr / Re<p, q>; h += a p; r -= a q; rr' partials.  The image block
// of q is formed here from the channel partials: q_rho = sum_j PR_j + alpha p_rho.
// On the last iteration the Newton update x += h is applied instead of the r update.
__global__ void __launch_bounds__(VT)
k_cg_update(const float2* __restrict__ PR, const double2* __restrict__ Q, const double2* __restrict__ P,
            double2* __restrict__ H, double2* __restrict__ Rv, float2* __restrict__ xh,
            Partials rr, const double* __restrict__ pq, int npq, double alpha,
            double* __restrict__ rr_next, int first, int last, int J, int RR, long long X, int nchunk) {
  __shared__ double sh[VT];
  const int b = blockIdx.x / nchunk, c = blockIdx.x - b * nchunk;
  const double pqs = block_sum_array<VT>(pq + (size_t)b * rr.stride, npq, sh);
  const double rrs = block_sum_array<VT>(rr.cur + (size_t)b * rr.stride, rr.ncur, sh);
  const double a = pqs != 0.0 ? rrs / pqs : 0.0;
  const long long e0 = (long long)c * CHUNK;
  const long long e1 = e0 + CHUNK < X ? e0 + CHUNK : X;
  double acc = 0.0;
  for (long long e = e0 + threadIdx.x; e < e1; e += VT) {
    const size_t ve = (size_t)b * X + e;
    const double2 p = P[ve];
    double hx = a * p.x, hy = a * p.y;
    if (!first) {
      const double2 h = H[ve];
      hx += h.x;
      hy += h.y;
    }
    if (last) {
      const float2 x = xh[ve];
      xh[ve] = make_float2((float)(x.x + hx), (float)(x.y + hy));
    } else {
      double qx, qy;
      if (e < RR) {
        qx = alpha * p.x;
        qy = alpha * p.y;
        for (int j = 0; j < J; ++j) {
          const float2 pr = PR[((size_t)b * J + j) * RR + e];
          qx += pr.x;
          qy += pr.y;
        }
      } else {
        const double2 q = Q[ve];
        qx = q.x;
        qy = q.y;
      }
      H[ve] = make_double2(hx, hy);
      const double2 r = Rv[ve];
      const double2 rn = make_double2(r.x - a * qx, r.y - a * qy);
      Rv[ve] = rn;
      acc += rn.x * rn.x + rn.y * rn.y;
    }
  }
  if (!last) {
    const double s = block_sum<VT>(acc, sh);
    if (threadIdx.x == 0) rr_next[(size_t)b * rr.stride + c] = s;
  }
}

// Assemble an operator result in float32 storage: image block sum_j PR_j + alpha p
// (p may be null), coil block copied from Q.
__global__ void __launch_bounds__(VT)
k_finalize(const float2* __restrict__ PR, const double2* __restrict__ p, double alpha,
           const double2* __restrict__ Q, float2* __restrict__ out, int J, int RR, long long X,
           int nchunk) {
  const int b = blockIdx.x / nchunk, c = blockIdx.x - b * nchunk;
  const long long e0 = (long long)c * CHUNK;
  const long long e1 = e0 + CHUNK < X ? e0 + CHUNK : X;
  for (long long e = e0 + threadIdx.x; e < e1; e += VT) {
    const size_t ve = (size_t)b * X + e;
    if (e < RR) {
      double sx = 0.0, sy = 0.0;
      for (int j = 0; j < J; ++j) {
        const float2 pr = PR[((size_t)b * J + j) * RR + e];
        sx += pr.x;
        sy += pr.y;
      }
      if (p) {
        const double2 pp = p[ve];
        sx += alpha * pp.x;
        sy += alpha * pp.y;
      }
      out[ve] = make_float2((float)sx, (float)sy);
    } else {
      out[ve] = tof(Q[ve]);
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

// z[b][j][y][x] = scale sum_s y[b][j][s] exp(+i 2 pi (kx_s x + ky_s y)), x, y in [-R/2, R/2)
template <int JG>
__global__ void __launch_bounds__(VT)
k_grid(const float* __restrict__ traj, const float2* __restrict__ yv, float2* __restrict__ z,
       int J, int S, int R, float scale) {
  __shared__ float2 ex[GSC][GT], ey[GSC][GT], ys[JG][GSC];
  const int nt = R / GT;
  const int ty0 = (blockIdx.x / nt) * GT, tx0 = (blockIdx.x % nt) * GT;
  const int jg = blockIdx.y, b = blockIdx.z;
  const int py = threadIdx.x / GT, px = threadIdx.x % GT;
  const float* tr = traj + (size_t)b * S * 2;
  double2 acc[JG];   // float32 sums over GSC samples, accumulated in float64
#pragma unroll
  for (int q = 0; q < JG; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int s0 = 0; s0 < S; s0 += GSC) {
    for (int q = threadIdx.x; q < GSC * GT; q += VT) {
      const int ss = q / GT, pix = q % GT, s = s0 + ss;
      if (s < S) {
        const float kx = tr[2 * s], ky = tr[2 * s + 1];
        ex[ss][pix] = cis_cycles<+1>(kx, tx0 + pix - R / 2);
        ey[ss][pix] = cis_cycles<+1>(ky, ty0 + pix - R / 2);
      } else {
        ex[ss][pix] = czero<float2>();
        ey[ss][pix] = czero<float2>();
      }
    }
    for (int q = threadIdx.x; q < JG * GSC; q += VT) {
      const int jj = q / GSC, ss = q % GSC, s = s0 + ss, j = jg * JG + jj;
      ys[jj][ss] = (s < S && j < J) ? yv[((size_t)b * J + j) * S + s] : czero<float2>();
    }
    __syncthreads();
    float2 part[JG];
#pragma unroll
    for (int q = 0; q < JG; ++q) part[q] = czero<float2>();
#pragma unroll 4
    for (int ss = 0; ss < GSC; ++ss) {
      const float2 e = cmul(ey[ss][py], ex[ss][px]);
#pragma unroll
      for (int q = 0; q < JG; ++q) {
        const float2 y = ys[q][ss];
        part[q].x += y.x * e.x - y.y * e.y;
        part[q].y += y.x * e.y + y.y * e.x;
      }
    }
#pragma unroll
    for (int q = 0; q < JG; ++q) {
      acc[q].x += part[q].x;
      acc[q].y += part[q].y;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < JG; ++q) {
    const int j = jg * JG + q;
    if (j < J)
      z[(((size_t)b * J + j) * R + ty0 + py) * R + tx0 + px] =
          make_float2((float)(acc[q].x * scale), (float)(acc[q].y * scale));
  }
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
constexpr int FXC = 32;   // x chunk
__global__ void __launch_bounds__(VT)
k_nudft_fwd(const float* __restrict__ traj, const float2* __restrict__ u, float2* __restrict__ yv,
            int J, int S, int R, float scale) {
  __shared__ float2 uc[224 * FXC];
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
      const int yy = q / FXC, xx = q % FXC;
      uc[q] = ub[(size_t)yy * R + x0 + xx];
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


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_cg_init(const Shape& s, const Bufs& w, hipStream_t st, const float2* xh,
                          const float2* xprev, double alpha) {
  k_cg_init<<<s.B * s.NCI, VT, 0, st>>>(w.PR, xh, xprev, alpha, w.Rv, w.Pv[0], w.rr[0], s.stride,
                                        s.NX3, s.J, s.R * s.R, s.X, s.NCI);
  return hipGetLastError();
}

hipError_t launch_cg_update(const Shape& s, const Bufs& w, hipStream_t st, int iter, int last,
                            const double2* p, Partials rr, float2* xh, double alpha) {
  double* next = w.rr[(iter + 1) & 1];
  k_cg_update<<<s.B * s.NCH, VT, 0, st>>>(w.PR, w.Q, p, w.H, w.Rv, xh, rr, w.pq, s.NY2 + s.NX3,
                                          alpha, next, iter == 0, last, s.J, s.R * s.R, s.X, s.NCH);
  return hipGetLastError();
}

hipError_t launch_finalize(const Shape& s, const Bufs& w, hipStream_t st, const double2* p,
                           double alpha, float2* out) {
  k_finalize<<<s.B * s.NCH, VT, 0, st>>>(w.PR, p, alpha, w.Q, out, s.J, s.R * s.R, s.X, s.NCH);
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

hipError_t launch_grid(const Shape& s, hipStream_t st, const float* traj, const float2* y, float2* z) {
  const int nt = (s.R / GT) * (s.R / GT);
  auto go = [&](auto jg) {
    constexpr int JG = decltype(jg)::value;
    dim3 grid(nt, (s.J + JG - 1) / JG, s.B);
    k_grid<JG><<<grid, VT, 0, st>>>(traj, y, z, s.J, s.S, s.R, 1.0f / s.R);
  };
  if (s.J % 8 == 0) go(IC<8>{});
  else if (s.J % 5 == 0) go(IC<5>{});
  else if (s.J % 4 == 0) go(IC<4>{});
  else if (s.J % 3 == 0) go(IC<3>{});
  else if (s.J % 2 == 0) go(IC<2>{});
  else go(IC<1>{});
  return hipGetLastError();
}

hipError_t launch_nudft_fwd(const Shape& s, hipStream_t st, const float* traj, const float2* u,
                            float2* y) {
  if (s.R > 224 || s.R % FXC) return hipErrorInvalidValue;
  dim3 grid((s.S + VT - 1) / VT, s.J, s.B);
  k_nudft_fwd<<<grid, VT, 0, st>>>(traj, u, y, s.J, s.S, s.R, 1.0f / s.R);
  return hipGetLastError();
}

hipError_t launch_psf(const Shape& s, const Bufs& w, hipStream_t st, const float* traj, int turn) {
  const GTable* t = table_for(s.G);
  if (!t) return hipErrorInvalidValue;
  const int nt = (s.G / GT) * (s.G / GT);
  k_psf_lags<<<nt, VT, 0, st>>>(traj, w.psf, s.S, s.R, s.G);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // F^H F = (1/R^2) psf-convolution; the unnormalised 2D DFT pair contributes 1/G^2
  const double scale = 1.0 / ((double)s.G * s.G * (double)s.R * s.R);
  return t->psf_fft(s, w, st, w.P + (size_t)turn * s.G * s.G, scale);
}

}  // namespace nlv
