// Device FFT building blocks for gfx950 (wave64, LDS exchange).
//
// A G-point DFT of one line is computed by a "team" of threads with the
// four-step factorisation G = G1 * G2 (both factors small, built from radices
// 2, 3, 4, 5, 7):
//
//   X[G2 k1 + k2] = sum_n1 w_G1^(n1 k1) w_G^(n1 k2) sum_n2 w_G2^(n2 k2) x[n1 + G1 n2]
//
// Each thread keeps a whole G2- (or G1-) point sub-transform in registers
// (fully unrolled, compile-time twiddles); the two stages exchange data once
// through LDS.  fsA takes inputs in the order n = n1 + G1 n2 (thread n1 holds
// n2 = 0..G2-1) and leaves outputs in the order k = G2 k1 + k2 (thread k2 holds
// k1 = 0..G1-1); fsB is the same transform with the two index maps swapped, so
// fsA followed by a pointwise step and fsB keeps every value in registers
// between the two transforms.  All transforms are unnormalised; the sign of
// the exponent is the template parameter DIR (-1 forward, +1 inverse).
//
// Everything is templated on the complex type C (float2 or double2) used for
// the arithmetic and the LDS exchange; loads and stores go through caller
// functors, which implement zero padding and cropping ("pruning") and the
// conversion from / to the storage precision.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>

namespace nlv {

// ---------------------------------------------------------------------------
// compile-time helpers
// ---------------------------------------------------------------------------

template <int V>
using IC = std::integral_constant<int, V>;

template <int B, int E, class F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(IC<B>{});
    sfor<B + 1, E>(f);
  }
}

constexpr double kPi = 3.14159265358979323846264338327950288;

// Taylor series of sin / cos on [-pi, pi]; 18 terms reach double rounding.
constexpr double ct_reduce(double x) {
  while (x > kPi) x -= 2.0 * kPi;
  while (x < -kPi) x += 2.0 * kPi;
  return x;
}
constexpr double ct_sin(double x) {
  x = ct_reduce(x);
  double term = x, sum = x;
  for (int k = 1; k < 18; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos(double x) {
  x = ct_reduce(x);
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 18; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

// ---------------------------------------------------------------------------
// complex helpers (interleaved re, im) for C = float2 / double2
// ---------------------------------------------------------------------------

template <class C> struct CT;
template <> struct CT<float2> {
  using R = float;
  __device__ __forceinline__ static float2 mk(float a, float b) { return make_float2(a, b); }
};
template <> struct CT<double2> {
  using R = double;
  __device__ __forceinline__ static double2 mk(double a, double b) { return make_double2(a, b); }
};

template <class C> __device__ __forceinline__ C cadd(C a, C b) { return CT<C>::mk(a.x + b.x, a.y + b.y); }
template <class C> __device__ __forceinline__ C csub(C a, C b) { return CT<C>::mk(a.x - b.x, a.y - b.y); }
template <class C> __device__ __forceinline__ C cmul(C a, C b) {
  return CT<C>::mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <class C> __device__ __forceinline__ C cjmul(C a, C b) {
  return CT<C>::mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <class C> __device__ __forceinline__ C cscale(C a, typename CT<C>::R s) { return CT<C>::mk(a.x * s, a.y * s); }
template <class C> __device__ __forceinline__ C czero() { return CT<C>::mk(0, 0); }
// multiply by (DIR * i)
template <int DIR, class C>
__device__ __forceinline__ C mul_di(C a) {
  return DIR > 0 ? CT<C>::mk(-a.y, a.x) : CT<C>::mk(a.y, -a.x);
}

// conversions between storage and arithmetic precision
__device__ __forceinline__ double2 to_d(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 to_d(double2 v) { return v; }
__device__ __forceinline__ float2 to_f(double2 v) { return make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ float2 to_f(float2 v) { return v; }
template <class S> __device__ __forceinline__ S store_as(double2 v);
template <> __device__ __forceinline__ float2 store_as<float2>(double2 v) { return to_f(v); }
template <> __device__ __forceinline__ double2 store_as<double2>(double2 v) { return v; }

// v * exp(DIR * i * 2 pi * M / N), M and N compile-time.
template <int N, int M, int DIR, class C>
__device__ __forceinline__ C twc(C v) {
  using R = typename CT<C>::R;
  constexpr int m = ((M % N) + N) % N;
  if constexpr (m == 0) {
    return v;
  } else if constexpr (2 * m == N) {
    return CT<C>::mk(-v.x, -v.y);
  } else if constexpr (4 * m == N) {
    return mul_di<DIR>(v);
  } else if constexpr (4 * m == 3 * N) {
    return mul_di<-DIR>(v);
  } else if constexpr ((8 * m) % N == 0) {
    // odd multiple of pi/4: |cos| = |sin| = sqrt(1/2)
    constexpr double ang = 2.0 * kPi * m / N;
    constexpr R h = (R)0.70710678118654752440084436210484904;
    constexpr R c = ct_cos(ang) > 0 ? h : -h;
    constexpr R s = DIR * ct_sin(ang) > 0 ? h : -h;
    if constexpr (c == s) {
      return CT<C>::mk((v.x - v.y) * c, (v.x + v.y) * c);
    } else {
      return CT<C>::mk((v.x + v.y) * c, (v.y - v.x) * c);
    }
  } else {
    constexpr double ang = 2.0 * kPi * m / N;
    constexpr R c = (R)ct_cos(ang);
    constexpr R s = (R)(DIR * ct_sin(ang));
    return CT<C>::mk(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// ---------------------------------------------------------------------------
// in-register DFT codelets, natural order in and out
// ---------------------------------------------------------------------------

constexpr int first_factor(int n) {
  if (n % 4 == 0 && n != 4) return 4;
  if (n % 2 == 0 && n != 2) return 2;
  if (n % 3 == 0 && n != 3) return 3;
  if (n % 5 == 0 && n != 5) return 5;
  if (n % 7 == 0 && n != 7) return 7;
  return n;
}

template <int N, int DIR, class C>
struct DFT {
  static constexpr int N1 = first_factor(N);
  static constexpr int N2 = N / N1;
  static_assert(N1 != N, "unsupported prime length");
  __device__ __forceinline__ static void run(C (&x)[N]) {
    C y[N];
    sfor<0, N1>([&](auto i1) {
      constexpr int n1 = decltype(i1)::value;
      C t[N2];
      sfor<0, N2>([&](auto i2) {
        constexpr int n2 = decltype(i2)::value;
        t[n2] = x[n1 + N1 * n2];
      });
      DFT<N2, DIR, C>::run(t);
      sfor<0, N2>([&](auto i2) {
        constexpr int k2 = decltype(i2)::value;
        y[n1 * N2 + k2] = twc<N, n1 * k2, DIR>(t[k2]);
      });
    });
    sfor<0, N2>([&](auto i2) {
      constexpr int k2 = decltype(i2)::value;
      C u[N1];
      sfor<0, N1>([&](auto i1) {
        constexpr int n1 = decltype(i1)::value;
        u[n1] = y[n1 * N2 + k2];
      });
      DFT<N1, DIR, C>::run(u);
      sfor<0, N1>([&](auto i1) {
        constexpr int k1 = decltype(i1)::value;
        x[N2 * k1 + k2] = u[k1];
      });
    });
  }
};

template <int DIR, class C>
struct DFT<1, DIR, C> {
  __device__ __forceinline__ static void run(C (&)[1]) {}
};

template <int DIR, class C>
struct DFT<2, DIR, C> {
  __device__ __forceinline__ static void run(C (&x)[2]) {
    const C a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <int DIR, class C>
struct DFT<4, DIR, C> {
  __device__ __forceinline__ static void run(C (&x)[4]) {
    const C s02 = cadd(x[0], x[2]), d02 = csub(x[0], x[2]);
    const C s13 = cadd(x[1], x[3]), d13 = mul_di<DIR>(csub(x[1], x[3]));
    x[0] = cadd(s02, s13);
    x[2] = csub(s02, s13);
    x[1] = cadd(d02, d13);
    x[3] = csub(d02, d13);
  }
};

// Odd prime P: X[k] = x0 + sum_{n=1}^{(P-1)/2} (x_n + x_{P-n}) cos(2 pi n k / P)
//                    + i DIR sin(2 pi n k / P) (x_n - x_{P-n}),  X[P-k] likewise with -i.
template <int P, int DIR, class C>
struct DFTPrime {
  __device__ __forceinline__ static void run(C (&x)[P]) {
    using R = typename CT<C>::R;
    constexpr int H = (P - 1) / 2;
    C a[H + 1], b[H + 1];
    C sum = x[0];
    sfor<1, H + 1>([&](auto in) {
      constexpr int n = decltype(in)::value;
      a[n] = cadd(x[n], x[P - n]);
      b[n] = csub(x[n], x[P - n]);
      sum = cadd(sum, a[n]);
    });
    C out[P];
    out[0] = sum;
    sfor<1, H + 1>([&](auto ik) {
      constexpr int k = decltype(ik)::value;
      C A = x[0];
      C Bv = czero<C>();
      sfor<1, H + 1>([&](auto in) {
        constexpr int n = decltype(in)::value;
        constexpr double ang = 2.0 * kPi * ((n * k) % P) / P;
        constexpr R c = (R)ct_cos(ang);
        constexpr R s = (R)ct_sin(ang);
        A = CT<C>::mk(A.x + a[n].x * c, A.y + a[n].y * c);
        Bv = CT<C>::mk(Bv.x + b[n].x * s, Bv.y + b[n].y * s);
      });
      const C iB = mul_di<DIR>(Bv);
      out[k] = cadd(A, iB);
      out[P - k] = csub(A, iB);
    });
    sfor<0, P>([&](auto ik) {
      constexpr int k = decltype(ik)::value;
      x[k] = out[k];
    });
  }
};

template <int DIR, class C>
struct DFT<3, DIR, C> {
  __device__ __forceinline__ static void run(C (&x)[3]) { DFTPrime<3, DIR, C>::run(x); }
};
template <int DIR, class C>
struct DFT<5, DIR, C> {
  __device__ __forceinline__ static void run(C (&x)[5]) { DFTPrime<5, DIR, C>::run(x); }
};
template <int DIR, class C>
struct DFT<7, DIR, C> {
  __device__ __forceinline__ static void run(C (&x)[7]) { DFTPrime<7, DIR, C>::run(x); }
};

// ---------------------------------------------------------------------------
// team four-step transforms
// ---------------------------------------------------------------------------

// The factorisation G = G1 G2 of a grid's team transform.  A team key
// names a grid side and one of its factorisations: key = G + split * GKEY,
// split 0 the default below, split 1 an alternative (the swapped order
// G2 G1, or for a square split another one); every kernel that takes a key
// derives the grid side with grid_of.
constexpr int GKEY = 1 << 16;
constexpr int grid_of(int key) { return key % GKEY; }

template <int G>
struct FS0;
template <> struct FS0<64>  { static constexpr int G1 = 8,  G2 = 8,  A1 = 16, A2 = 4;  };
template <> struct FS0<128> { static constexpr int G1 = 16, G2 = 8,  A1 = 8,  A2 = 16; };
template <> struct FS0<256> { static constexpr int G1 = 16, G2 = 16, A1 = 32, A2 = 8;  };
template <> struct FS0<320> { static constexpr int G1 = 16, G2 = 20, A1 = 20, A2 = 16; };
template <> struct FS0<384> { static constexpr int G1 = 16, G2 = 24, A1 = 24, A2 = 16; };
template <> struct FS0<432> { static constexpr int G1 = 16, G2 = 27, A1 = 27, A2 = 16; };
template <> struct FS0<448> { static constexpr int G1 = 16, G2 = 28, A1 = 28, A2 = 16; };
template <> struct FS0<480> { static constexpr int G1 = 16, G2 = 30, A1 = 30, A2 = 16; };
template <> struct FS0<512> { static constexpr int G1 = 16, G2 = 32, A1 = 32, A2 = 16; };

template <int KEY>
struct FS {
  static constexpr int G = grid_of(KEY), split = KEY / GKEY;
  static_assert(split == 0 || split == 1, "bad team key");
  static constexpr int G1 = split ? FS0<G>::A1 : FS0<G>::G1;
  static constexpr int G2 = split ? FS0<G>::A2 : FS0<G>::G2;
};

template <int KEY>
struct Team {
  static constexpr int GRID = grid_of(KEY);
  static constexpr int G1 = FS<KEY>::G1, G2 = FS<KEY>::G2;
  static_assert(G1 * G2 == GRID, "bad factorisation");
  static constexpr int SIZE = G1 > G2 ? G1 : G2;   // threads per line
  static constexpr int LDSN = G1 * (G2 + 1);       // complex LDS slots per line (padded)
  // Line pitch of the column passes, whose neighbouring lanes work on
  // neighbouring lines: LDSN is a multiple of 16 slots (256 B) for G >= 128,
  // which puts those lanes on the same LDS banks; two more slots spread them
  // (measured at G = 320: column passes 15 % faster at batch 16).
  static constexpr int LDSC = LDSN + 2;
};

// Index sets of a G-point line: all G samples, the R = G/2 centred image
// samples, or the G_c = G/4 centred coil-spectrum samples.  For each register
// slot of a team transform the set membership of the slot's index range is
// classified at compile time, so that absent inputs become constant zeros
// (folded away) and unused outputs become dead code.
enum : int { SET_ALL = 0, SET_IMG = 1, SET_COIL = 2 };
enum : int { NEVER = 0, ALWAYS = 1, RUNTIME = 2 };
constexpr int classify(int G, int set, int lo, int len) {
  if (set == SET_ALL) return ALWAYS;
  const int H = set == SET_IMG ? G / 4 : G / 8;
  int nin = 0;
  for (int n = lo; n < lo + len; ++n) nin += (n < H || n >= G - H) ? 1 : 0;
  return nin == 0 ? NEVER : (nin == len ? ALWAYS : RUNTIME);
}
// index n = tl + G1 * N2 (tl in [0, G1)): fsA inputs, fsB outputs
template <int G, int SET, int N2>
constexpr int cls_n() { return classify(Team<G>::GRID, SET, Team<G>::G1 * N2, Team<G>::G1); }
// index k = G2 * K1 + tl (tl in [0, G2)): fsA outputs, fsB inputs
template <int G, int SET, int K1>
constexpr int cls_k() { return classify(Team<G>::GRID, SET, Team<G>::G2 * K1, Team<G>::G2); }

// runtime twiddle exp(DIR i 2 pi m / G) from the value v = tw[m] = (cos, sin)
// of the host-built FP64 table
template <int DIR, class C>
__device__ __forceinline__ C twv(double2 v) {
  using R = typename CT<C>::R;
  return CT<C>::mk((R)v.x, (R)(DIR > 0 ? v.y : -v.y));
}
template <int DIR, class C>
__device__ __forceinline__ C twr(const double2* __restrict__ tw, int m) {
  return twv<DIR, C>(tw[m]);
}

// Gather of the fsA inputs of thread tl < G1: a[n2] = x[tl + G1 n2] from
// load(n), constant zero outside SET_IN.  Split from fsA so that a kernel can
// issue the loads of its next line group before transforming the current one.
template <int G, int SET_IN, class C, class Load>
__device__ __forceinline__ void fsA_load(int tl, C (&a)[Team<G>::G2], Load&& load) {
  using T = Team<G>;
  if (tl < T::G1) {
    sfor<0, T::G2>([&](auto i) {
      constexpr int n2 = decltype(i)::value;
      if constexpr (cls_n<G, SET_IN, n2>() == NEVER) {
        a[n2] = czero<C>();
      } else {
        a[n2] = load(tl + T::G1 * n2);
      }
    });
  }
}

// fsA on gathered inputs a (fsA_load); outputs X[G2 k1 + tl] in out[k1] for
// tl < G2, outputs outside SET_OUT left zero.  Contains one workgroup barrier;
// every thread of the block must call it.  a is overwritten.  tv is the
// thread's twiddle table value tw[tl] (twiddle_of): a kernel that loads it
// together with its data keeps the table load off the transform's critical path.
template <int G, int DIR, int SET_OUT, class C>
__device__ __forceinline__ void fsA_regs(int tl, C* lds, double2 tv, C (&a)[Team<G>::G2],
                                         C (&out)[Team<G>::G1]) {
  using T = Team<G>;
  if (tl < T::G1) {
    DFT<T::G2, DIR, C>::run(a);
    // twiddles w^(tl k2) by recurrence from one table value (FP64: the
    // rounding of the k2-fold product stays near 1e-15, far below float32)
    const C w1 = twv<DIR, C>(tv);
    C wk = w1;
    sfor<0, T::G2>([&](auto i) {
      constexpr int k2 = decltype(i)::value;
      C v = a[k2];
      if constexpr (k2 != 0) {
        v = cmul(v, wk);
        if constexpr (k2 + 1 < T::G2) wk = cmul(wk, w1);
      }
      lds[tl * (T::G2 + 1) + k2] = v;
    });
  }
  __syncthreads();
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto i) {
      constexpr int n1 = decltype(i)::value;
      out[n1] = lds[n1 * (T::G2 + 1) + tl];
    });
    DFT<T::G1, DIR, C>::run(out);
    sfor<0, T::G1>([&](auto i) {
      constexpr int k1 = decltype(i)::value;
      if constexpr (cls_k<G, SET_OUT, k1>() == NEVER) out[k1] = czero<C>();
    });
  }
}

// the twiddle table value of team lane tl (also valid for the idle lanes,
// tl = SIZE < G)
template <int G>
__device__ __forceinline__ double2 twiddle_of(const double2* __restrict__ tw, int tl) {
  return tw[tl];
}

template <int G, int DIR, int SET_OUT, class C>
__device__ __forceinline__ void fsA_regs(int tl, C* lds, const double2* __restrict__ tw,
                                         C (&a)[Team<G>::G2], C (&out)[Team<G>::G1]) {
  fsA_regs<G, DIR, SET_OUT>(tl, lds, twiddle_of<G>(tw, tl), a, out);
}

// fsA: inputs x[n1 + G1 n2] from load(n) (thread tl = n1 < G1); outputs
// X[G2 k1 + tl] in out[k1] for tl < G2.  Inputs outside SET_IN are zero and
// outputs outside SET_OUT are left zero.  Contains one workgroup barrier;
// every thread of the block must call it.
template <int G, int DIR, int SET_IN, int SET_OUT, class C, class Load>
__device__ __forceinline__ void fsA(int tl, C* lds, const double2* __restrict__ tw, Load&& load,
                                    C (&out)[Team<G>::G1]) {
  C a[Team<G>::G2];
  fsA_load<G, SET_IN>(tl, a, load);
  fsA_regs<G, DIR, SET_OUT>(tl, lds, tw, a, out);
}

// fsB: inputs x[G2 k1 + tl] in in[k1] (thread tl < G2), taken as zero outside
// SET_IN; outputs X[n1 + G1 n2] inside SET_OUT are passed to store(n, value) by
// thread tl = n1 < G1.  Starts with a barrier so that the LDS line may be
// reused right after fsA; contains two barriers.
template <int G, int DIR, int SET_IN, int SET_OUT, class C, class Store>
__device__ __forceinline__ void fsB(int tl, C* lds, double2 tv, C (&in)[Team<G>::G1], Store&& store) {
  using T = Team<G>;
  __syncthreads();
  if (tl < T::G2) {
    sfor<0, T::G1>([&](auto i) {
      constexpr int k1 = decltype(i)::value;
      if constexpr (cls_k<G, SET_IN, k1>() == NEVER) in[k1] = czero<C>();
    });
    DFT<T::G1, DIR, C>::run(in);
    const C w1 = twv<DIR, C>(tv);   // w^(n1 tl) by recurrence, as in fsA
    C wk = w1;
    sfor<0, T::G1>([&](auto i) {
      constexpr int n1 = decltype(i)::value;
      C v = in[n1];
      if constexpr (n1 != 0) {
        v = cmul(v, wk);
        if constexpr (n1 + 1 < T::G1) wk = cmul(wk, w1);
      }
      lds[n1 * (T::G2 + 1) + tl] = v;
    });
  }
  __syncthreads();
  if (tl < T::G1) {
    C a[T::G2];
    sfor<0, T::G2>([&](auto i) {
      constexpr int k2 = decltype(i)::value;
      a[k2] = lds[tl * (T::G2 + 1) + k2];
    });
    DFT<T::G2, DIR, C>::run(a);
    sfor<0, T::G2>([&](auto i) {
      constexpr int n2 = decltype(i)::value;
      if constexpr (cls_n<G, SET_OUT, n2>() != NEVER) store(tl + T::G1 * n2, a[n2]);
    });
  }
}

template <int G, int DIR, int SET_IN, int SET_OUT, class C, class Store>
__device__ __forceinline__ void fsB(int tl, C* lds, const double2* __restrict__ tw, C (&in)[Team<G>::G1],
                                    Store&& store) {
  fsB<G, DIR, SET_IN, SET_OUT>(tl, lds, twiddle_of<G>(tw, tl), in, static_cast<Store&&>(store));
}

// ---------------------------------------------------------------------------
// index sets on the G-grid (DFT index n <-> centred coordinate n or n - G)
// ---------------------------------------------------------------------------

// image row/column index of grid index n (R = G/2 centred samples), or -1
template <int G>
__device__ __forceinline__ int img_idx(int n) {
  constexpr int H = G / 4;
  return n < H ? n + H : (n >= G - H ? n - G + H : -1);
}
// coil-spectrum index of grid index n (G_c = G/4 centred samples), or -1
template <int G>
__device__ __forceinline__ int coil_idx(int n) {
  constexpr int H = G / 8;
  return n < H ? n + H : (n >= G - H ? n - G + H : -1);
}

}  // namespace nlv
