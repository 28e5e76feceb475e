// C-ABI of the NLINV hot path: argument validation, workspace layout, FP64
// host tables and the launch sequences of each entry point.
#include "nlinv.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "nlinv_internal.h"

using nlv::Bufs;
using nlv::Partials;
using nlv::Shape;

namespace nlv {
// flag |= 1 if any of the n complex values of x is not finite (nlinv_launch.hip)
hipError_t launch_check_finite(hipStream_t st, const float2* x, long long n, int* flag);
// p[0] = v by a one-thread kernel
hipError_t launch_fill_int(hipStream_t st, int* p, int v);
}  // namespace nlv

struct nlinv_plan_s {
  nlinv_params p;
  Shape s;   // shape of the active batch (s.B <= p.batch)
  Bufs w;
  int* flag = nullptr;   // workspace int set by the finiteness check (NLINV_F_CHECK_FINITE)
  const nlv::GTable* t = nullptr;
  hipStream_t stream = nullptr;
  std::vector<char> psf_valid;
  std::string err;
  int timer_kid = NLINV_KT_NONE;
  std::vector<hipEvent_t> ev;   // start/stop pairs
  size_t ev_used = 0;
  nlv::LaunchTiming lt;         // armed by timed() for single-kernel classes
  // HIP graphs of nlinv_reconstruct, one per distinct argument set
  bool graphs = false;
  hipStream_t cap_stream = nullptr;
  std::map<std::vector<uintptr_t>, hipGraphExec_t> graph_cache;
  float2* xb = nullptr;   // [B][X] source frames of nlinv_reconstruct_frames
  std::vector<hipStream_t> branch;   // streams of the members of a relaxed group run side by side
  std::vector<hipEvent_t> bev;       // their fork and join events
  int device = 0;               // HIP device the plan was created on
  size_t ws_need = 0;           // its workspace size (counted against the device's budget)
  bool is_static = false;       // workspace = the device's static array (nlinv_plan_create_static)
  float* dinv_own = nullptr;    // the plan's own coil-weight table (nlinv_set_coil_weights restores it)
  uint64_t id = 0;              // unique over the process (keys of the multi-plan graphs)
  uint64_t gen = 0;             // bumped when the plan's captured graphs go stale
};

namespace {

thread_local std::string g_err;   // errors not tied to a plan

// Per-device admission budget of plan workspaces (nlinv_set_budget) and the
// owner of each device's static workspace (nlinv_plan_create_static).
constexpr int MAX_DEV = 64;
std::mutex g_dev_mu;
size_t g_budget[MAX_DEV] = {};       // 0: no cap
size_t g_used[MAX_DEV] = {};         // summed workspace sizes of the live plans
nlinv_plan g_static_owner[MAX_DEV] = {};

// Graphs of nlinv_reconstruct_multi, one per argument set of a group of plans
// (keyed by plan ids and generations, so a destroyed plan's address reused by a
// new plan never meets an old graph); dropped with any member plan.
std::atomic<uint64_t> g_next_id{1};
struct MultiGraph {
  hipGraphExec_t exec;
  std::vector<uint64_t> ids;
};
std::mutex g_multi_mu;
std::map<std::vector<uint64_t>, MultiGraph> g_multi;

int fail(nlinv_plan plan, int code, const std::string& msg) {
  if (plan) plan->err = msg; else g_err = msg;
  return code;
}

int fail_hip(nlinv_plan plan, hipError_t e, const char* what) {
  std::string m = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
  return fail(plan, NLINV_E_HIP, m);
}

#define NLV_HIP(plan, expr)                                  \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return fail_hip(plan, e_, #expr);  \
  } while (0)

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

bool supported_grid(int G) {
  return G == 64 || G == 128 || G == 256 || G == 320 || G == 384 || G == 432 || G == 448 || G == 480 ||
         G == 512;
}

using nlv::KB_TAPS;
using nlv::KB_W;

// Fourier transform of the Kaiser-Bessel kernel at u cycles per grid cell
// (|pi W u| < beta): the deapodisation.
double kb_phi_hat(double u, double beta) {
  const double a = std::sqrt(beta * beta - (M_PI * KB_W * u) * (M_PI * KB_W * u));
  return KB_W * std::sinh(a) / a / nlv::kb_bessel_i0(beta);
}

// Validates the parameters, fills the shape and the workspace layout.
struct Layout {
  size_t tw, dinv, P, psf, CO, U1, U2, PR, IMG, GS, H, Rv, Pv0, Pv1, Q, pq, rr0, rr1, XB, KBR, KBE, KBP, KBN, KBS, KBQ, KBC, KG, COV, FLAG,
      VR, VP, PDFP, PPP, SCAL,
      total;
};

int derive(const nlinv_params* p, Shape* s, Layout* L, std::string* err) {
  auto bad = [&](int code, const char* m) { *err = m; return code; };
  if (!p) return bad(NLINV_E_ARG, "params is NULL");
  if (p->N <= 0) return bad(NLINV_E_ARG, "N must be positive");
  // G = 2 gamma N with 1 <= gamma <= 2 (Sec. 3.2): the reconstructed field of
  // view R = G/2 holds the N x N image in its centre
  const int G = p->G == 0 ? 2 * p->N : p->G;
  if (G < 2 * p->N || G > 4 * p->N) return bad(NLINV_E_SIZE, "G must be in [2N, 4N] (G = 2 gamma N, 1 <= gamma <= 2)");
  if (!supported_grid(G)) return bad(NLINV_E_SIZE, "unsupported grid: G must be 64, 128, 256, 320, 384, 432, 448, 480 or 512");
  if (p->J < 1 || p->J > 64) return bad(NLINV_E_ARG, "J must be in [1, 64]");
  if (p->K < 1 || (p->K % 2) == 0) return bad(NLINV_E_ARG, "K must be a positive odd number");
  const int S_r = p->S_r == 0 ? 2 * p->N : p->S_r;
  if (S_r < 1) return bad(NLINV_E_ARG, "S_r must be positive");
  if ((long long)p->K * S_r > (1 << 24)) return bad(NLINV_E_SIZE, "K * S_r too large");
  if (p->U < 1 || p->U > 64) return bad(NLINV_E_ARG, "U must be in [1, 64]");
  if (p->batch < 1 || p->batch > nlv::MAXB) return bad(NLINV_E_ARG, "batch must be in [1, 64]");
  if (p->newton < 0 || p->newton > 1000) return bad(NLINV_E_ARG, "newton must be in [0, 1000]");
  if (p->cg < 1 || p->cg > 100000) return bad(NLINV_E_ARG, "cg must be in [1, 100000]");
  if (p->flags & ~(NLINV_F_EXACT_GRID | NLINV_F_CHECK_FINITE)) return bad(NLINV_E_ARG, "unknown flag bits");
  if (!(p->alpha0 > 0.0) || !std::isfinite(p->alpha0)) return bad(NLINV_E_ARG, "alpha0 must be positive and finite");
  if (!(p->alpha_q > 0.0 && p->alpha_q <= 1.0)) return bad(NLINV_E_ARG, "alpha_q must be in (0, 1]");
  if (!(p->alpha_min >= 0.0) || !std::isfinite(p->alpha_min)) return bad(NLINV_E_ARG, "alpha_min must be >= 0");
  if (!(p->sob_a >= 0.0) || !(p->sob_l >= 0.0) || !std::isfinite(p->sob_a) || !std::isfinite(p->sob_l))
    return bad(NLINV_E_ARG, "Sobolev parameters must be finite and >= 0");
  if (p->col_tile != 0 && p->col_tile != 4 && p->col_tile != 8) return bad(NLINV_E_ARG, "col_tile must be 0, 4 or 8");
  if (p->cg_passes != 0 && p->cg_passes != 4 && p->cg_passes != 6) return bad(NLINV_E_ARG, "cg_passes must be 0, 4 or 6");
  if (p->fft_split != 0 && p->fft_split != 1) return bad(NLINV_E_ARG, "fft_split must be 0 or 1");

  Shape& S = *s;
  S.B = p->batch;
  S.J = p->J;
  S.G = G;
  S.R = G / 2;
  S.GC = G / 4;
  S.S = p->K * S_r;
  S.U = p->U;
  S.X = (long long)S.R * S.R + (long long)S.J * S.GC * S.GC;
  S.NT = S.R / nlv::TW;
  const nlv::GTable* tab = nlv::table_for(G);
  if (!tab) return bad(NLINV_E_SIZE, "no kernels for this grid size");
  S.NX3 = (S.J * S.GC + tab->row_lines - 1) / tab->row_lines;
  S.NRQ = (S.R * S.R + 64 * nlv::RHOQ_E - 1) / (64 * nlv::RHOQ_E);
  S.NCH = (int)((S.X + nlv::CHUNK - 1) / nlv::CHUNK);
  int st = S.NX3 + S.NRQ;
  if (S.NCH > st) st = S.NCH;
  S.stride = st;
  S.coltile = p->col_tile;
  S.gsplit = nlv::grid_nsplit(S.B, S.J, S.R);
  S.split = p->fft_split;
  const int trl = S.split ? tab->row_lines_split : tab->row_lines;   // lines per Toeplitz-pass block
  S.NTB = (S.J * S.G + trl - 1) / trl;
  S.NPP = S.J * S.R;
  // Kaiser-Bessel gridding tables: (W + 1)^2 entries per sample and turn; left
  // out (exact gridding only) when they would take more than 2 GiB
  S.kbe_stride = (long long)S.S * KB_TAPS * KB_TAPS;
  const double kb_bytes = (double)S.U * (2.0 * G * G + 3 + 2.0 * S.kbe_stride) * 4.0 +
                          (double)S.B * S.J * G * G * 8.0 + (double)S.kbe_stride * 8.0 + (double)G * G * 4.0;
  S.kb = (p->flags & NLINV_F_EXACT_GRID) == 0 && kb_bytes <= 2147483648.0;

  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t B = S.B, J = S.J, Gs = S.G, R = S.R, GC = S.GC, X = (size_t)S.X;
  const size_t c8 = 8;    // complex64
  const size_t c16 = 16;  // complex128
  L->tw = take(Gs * c16);
  L->dinv = take(GC * GC * 4);
  L->P = take((size_t)S.U * Gs * Gs * 4);
  L->psf = take(Gs * Gs * c16);
  L->CO = take(B * J * R * R * c8);
  L->U1 = take(B * J * GC * R * c16);
  L->U2 = take(B * J * Gs * R * c16);
  L->PR = take(B * J * R * R * c8);
  L->IMG = take(B * J * R * R * c8);
  // partial gridding sums: enough for the split of every active batch size
  size_t gs_items = 0;
  for (int b = 1; b <= S.B; ++b) {
    const int n = nlv::grid_nsplit(b, S.J, S.R);
    if (n > 1) gs_items = std::max(gs_items, (size_t)n * b);
  }
  L->GS = take(gs_items * J * R * R * c8);
  L->H = take(B * X * c16);
  L->Rv = take(B * X * c16);
  L->Pv0 = take(B * X * c16);
  L->Pv1 = take(B * X * c16);
  L->Q = take(B * X * c16);
  L->pq = take(B * (size_t)S.stride * 8);
  L->rr0 = take(B * (size_t)S.stride * 8);
  L->rr1 = take(B * (size_t)S.stride * 8);
  L->XB = take(B * X * c8);
  L->KBR = take(S.kb ? (size_t)S.U * ((size_t)Gs * Gs + 1) * 4 : 0);
  L->KBE = take(S.kb ? (size_t)S.U * (size_t)S.kbe_stride * 8 : 0);
  L->KBP = take(S.kb ? (size_t)S.U * Gs * Gs * 4 : 0);
  L->KBN = take(S.kb ? (size_t)S.U * 8 : 0);
  L->KBS = take(S.kb ? (size_t)S.kbe_stride * 8 : 0);
  L->KBQ = take(S.kb ? (size_t)Gs * Gs * 4 : 0);
  L->KBC = take(S.kb ? R * 4 : 0);
  L->KG = take(S.kb ? B * J * Gs * Gs * c8 : 0);
  L->COV = take((size_t)2 * nlv::MAX_JP * nlv::MAX_JP * c16);   // covariance, then its eigenvectors
  L->FLAG = take(sizeof(int));
  L->VR = take(B * J * GC * R * c16);
  L->VP = take(B * J * GC * R * c16);
  L->PDFP = take(B * (size_t)S.NTB * 8);
  L->PPP = take(B * (size_t)S.NPP * 8);
  L->SCAL = take(B * c16);
  L->total = off;
  return NLINV_OK;
}

int check_ptr(nlinv_plan plan, const void* ptr, const char* name, bool allow_null = false) {
  if (!ptr) {
    if (allow_null) return NLINV_OK;
    return fail(plan, NLINV_E_ARG, std::string(name) + " is NULL");
  }
  if (!aligned8(ptr)) return fail(plan, NLINV_E_ARG, std::string(name) + " is not 8-byte aligned");
  return NLINV_OK;
}

#define NLV_CHECK(expr)         \
  do {                          \
    int rc_ = (expr);           \
    if (rc_ != NLINV_OK) return rc_; \
  } while (0)

int check_plan(nlinv_plan plan) {
  if (!plan) return fail(nullptr, NLINV_E_ARG, "plan is NULL");
  plan->err.clear();
  return NLINV_OK;
}

// Event-bracketed launch of kernel class `kid` when the timer is enabled for it.
template <class F>
hipError_t timed(nlinv_plan plan, int kid, F&& f) {
  if (plan->timer_kid != kid || kid == NLINV_KT_NONE) return f();
  if (plan->ev_used + 2 > plan->ev.size()) {
    for (int i = 0; i < 256; ++i) {
      hipEvent_t e;
      // timing only: the events are never used to make memory visible, so they
      // skip the system-scope fence (which would write back and invalidate the
      // caches around the timed kernel and make it run colder than untimed)
      hipError_t he = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
      if (he != hipSuccess) return he;
      plan->ev.push_back(e);
    }
  }
  hipEvent_t a = plan->ev[plan->ev_used], b = plan->ev[plan->ev_used + 1];
  if (kid != NLINV_KT_GRID) {
    // one kernel per call: the events ride on its dispatch and time the kernel alone
    plan->lt.start = a;
    plan->lt.stop = b;
    plan->lt.attached = false;
    const hipError_t he = f();
    const bool attached = plan->lt.attached;
    plan->lt.start = plan->lt.stop = nullptr;
    if (he != hipSuccess) return he;
    if (!attached) return hipErrorInvalidValue;   // a launcher of this class bypassed launch_timed
    plan->ev_used += 2;
    return hipSuccess;
  }
  // several kernels per call (gridding): events recorded around the whole call
  hipError_t he = hipEventRecord(a, plan->stream);
  if (he != hipSuccess) return he;
  he = f();
  if (he != hipSuccess) return he;
  he = hipEventRecord(b, plan->stream);
  if (he != hipSuccess) return he;
  plan->ev_used += 2;
  return hipSuccess;
}

int turns_of(nlinv_plan plan, const int32_t* h_turn, nlv::TurnArgs* t) {
  if (!h_turn) return fail(plan, NLINV_E_ARG, "h_turn is NULL");
  std::memset(t, 0, sizeof(*t));
  for (int b = 0; b < plan->s.B; ++b) {
    const int v = h_turn[b];
    if (v < 0 || v >= plan->s.U) return fail(plan, NLINV_E_ARG, "turn out of range [0, U)");
    if (!plan->psf_valid[v])
      return fail(plan, NLINV_E_STATE, "PSF kernel of turn " + std::to_string(v) + " not computed (nlinv_grid / nlinv_psf)");
    t->t[b] = v;
  }
  return NLINV_OK;
}

// c_j = W^-1 c_hat_j of `xh` into `co`.
int coils_into(nlinv_plan plan, const float2* xh, float2* co) {
  const Shape& s = plan->s;
  NLV_HIP(plan, timed(plan, NLINV_KT_COIL_ROWS, [&] { return plan->t->coil_rows(s, plan->w, plan->stream, xh); }));
  NLV_HIP(plan, timed(plan, NLINV_KT_COIL_COLS, [&] {
            return plan->t->cols_fwd(s, plan->w, plan->stream, 0, co, xh, nullptr, nullptr);
          }));
  return NLINV_OK;
}

// PSF kernel and (if enabled) Kaiser-Bessel gridding table of `turn` from the
// first S samples (S <= s.S) of its trajectory (device, [K][S_r][2]); both
// are built by kernels on the plan's stream, so the call does not wait.
int build_turn(nlinv_plan plan, const float* d_traj, int turn, int S) {
  const Shape& s = plan->s;
  NLV_HIP(plan, nlv::launch_psf(s, plan->w, plan->stream, d_traj, S, turn));
  if (s.kb) NLV_HIP(plan, nlv::launch_kb_table(s, plan->w, plan->stream, d_traj, S, turn));
  plan->psf_valid[turn] = 1;
  return NLINV_OK;
}

// Make the first b items of every array the active batch.
void set_active(nlinv_plan plan, int b) {
  plan->s.B = b;
  plan->s.gsplit = nlv::grid_nsplit(b, plan->s.J, plan->s.R);
}

// Restores the active batch size on scope exit.
struct ActiveGuard {
  nlinv_plan plan;
  int b;
  ~ActiveGuard() { set_active(plan, b); }
};

}  // namespace

extern "C" {

int nlinv_params_default(nlinv_params* p) {
  if (!p) return fail(nullptr, NLINV_E_ARG, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->U = 1;
  p->batch = 1;
  p->newton = 7;
  p->cg = 10;
  p->alpha0 = 1.0;
  p->alpha_q = 0.5;
  p->alpha_min = 0.0;
  p->sob_a = 880.0;
  p->sob_l = 16.0;
  return NLINV_OK;
}

int nlinv_workspace_size(const nlinv_params* p, size_t* bytes) {
  if (!bytes) return fail(nullptr, NLINV_E_ARG, "bytes is NULL");
  Shape s;
  Layout L;
  std::string err;
  const int rc = derive(p, &s, &L, &err);
  if (rc != NLINV_OK) return fail(nullptr, rc, err);
  *bytes = L.total;
  return NLINV_OK;
}

int nlinv_sizes(const nlinv_params* p, int32_t* R, int32_t* G, int32_t* Gc, int64_t* S, int64_t* X) {
  Shape s;
  Layout L;
  std::string err;
  const int rc = derive(p, &s, &L, &err);
  if (rc != NLINV_OK) return fail(nullptr, rc, err);
  if (R) *R = s.R;
  if (G) *G = s.G;
  if (Gc) *Gc = s.GC;
  if (S) *S = s.S;
  if (X) *X = s.X;
  return NLINV_OK;
}

// The static workspace of nlinv_plan_create_static: one array per GPU, held
// by the process until it ends.  In host code `scratch` names a host-side
// stand-in, never the device array: its device address is looked up once per
// device (hipGetSymbolAddress, that device current) and only that address is
// used.
static __device__ __align__(256) unsigned char scratch[NLINV_STATIC_WORKSPACE_BYTES];
static void* g_scratch_ptr[MAX_DEV] = {};

// Device address of the current device's static workspace.
static int static_workspace(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(nullptr, e, "hipGetDevice");
  if (dev < 0 || dev >= MAX_DEV) return fail(nullptr, NLINV_E_ARG, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(nullptr, e, "hipGetSymbolAddress(scratch)");
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255u))
      return fail(nullptr, NLINV_E_HIP, "static workspace has no 256-byte aligned device address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return NLINV_OK;
}

// Returns a plan's budget share (and the static workspace) and frees it.
static void release_plan(nlinv_plan plan) {
  {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    g_used[plan->device] -= std::min(g_used[plan->device], plan->ws_need);
    if (plan->is_static && g_static_owner[plan->device] == plan) g_static_owner[plan->device] = nullptr;
  }
  delete plan;
}

static int create_plan(const nlinv_params* p, void* stream, void* d_workspace, size_t ws_bytes,
                       nlinv_plan* out, bool is_static) {
  if (!out) return fail(nullptr, NLINV_E_ARG, "out is NULL");
  *out = nullptr;
  Shape s;
  Layout L;
  std::string err;
  int rc = derive(p, &s, &L, &err);
  if (rc != NLINV_OK) return fail(nullptr, rc, err);
  if (!d_workspace) return fail(nullptr, NLINV_E_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_workspace) & 255u)
    return fail(nullptr, NLINV_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(nullptr, NLINV_E_WORKSPACE,
                "workspace too small: need " + std::to_string(L.total) + " bytes");
  int dev = 0;
  {
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(nullptr, e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEV) return fail(nullptr, NLINV_E_ARG, "device index beyond 63");
  }

  nlinv_plan plan = new (std::nothrow) nlinv_plan_s;
  if (!plan) return fail(nullptr, NLINV_E_ARG, "out of host memory");
  // admission against the device's workspace budget (released by destroy or
  // by a failure below)
  {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (g_budget[dev] != 0 && g_used[dev] + L.total > g_budget[dev]) {
      delete plan;
      return fail(nullptr, NLINV_E_BUDGET,
                  "device budget exceeded: " + std::to_string(g_used[dev]) + " of " +
                      std::to_string(g_budget[dev]) + " bytes in use, the plan needs " + std::to_string(L.total));
    }
    if (is_static && g_static_owner[dev] != nullptr) {
      delete plan;
      return fail(nullptr, NLINV_E_STATE, "the device's static workspace is held by a live plan (destroy it first)");
    }
    g_used[dev] += L.total;
    if (is_static) g_static_owner[dev] = plan;
  }
  plan->device = dev;
  plan->id = g_next_id++;
  plan->ws_need = L.total;
  plan->is_static = is_static;
  plan->p = *p;
  plan->s = s;
  plan->stream = reinterpret_cast<hipStream_t>(stream);
  plan->psf_valid.assign(s.U, 0);
  plan->t = nlv::table_for(s.G);
  if (!plan->t) {
    release_plan(plan);
    return fail(nullptr, NLINV_E_SIZE, "no kernels for this grid size");
  }
  char* base = static_cast<char*>(d_workspace);
  Bufs& w = plan->w;
  w.lt = &plan->lt;
  w.tw = reinterpret_cast<double2*>(base + L.tw);
  w.dinv = reinterpret_cast<float*>(base + L.dinv);
  plan->dinv_own = w.dinv;
  w.P = reinterpret_cast<float*>(base + L.P);
  w.psf = reinterpret_cast<double2*>(base + L.psf);
  w.CO = reinterpret_cast<float2*>(base + L.CO);
  w.U1 = reinterpret_cast<double2*>(base + L.U1);
  w.U2 = static_cast<void*>(base + L.U2);
  w.PR = reinterpret_cast<float2*>(base + L.PR);
  w.IMG = reinterpret_cast<float2*>(base + L.IMG);
  w.GS = reinterpret_cast<float2*>(base + L.GS);
  w.H = reinterpret_cast<double2*>(base + L.H);
  w.Rv = reinterpret_cast<double2*>(base + L.Rv);
  w.Pv[0] = reinterpret_cast<double2*>(base + L.Pv0);
  w.Pv[1] = reinterpret_cast<double2*>(base + L.Pv1);
  w.Q = reinterpret_cast<double2*>(base + L.Q);
  w.pq = reinterpret_cast<double*>(base + L.pq);
  w.rr[0] = reinterpret_cast<double*>(base + L.rr0);
  w.rr[1] = reinterpret_cast<double*>(base + L.rr1);
  plan->xb = reinterpret_cast<float2*>(base + L.XB);
  w.kbr = reinterpret_cast<int*>(base + L.KBR);
  w.kbe = reinterpret_cast<int2*>(base + L.KBE);
  w.kbp = reinterpret_cast<int*>(base + L.KBP);
  w.kbn = reinterpret_cast<int2*>(base + L.KBN);
  w.kbs = reinterpret_cast<int2*>(base + L.KBS);
  w.kbq = reinterpret_cast<int*>(base + L.KBQ);
  w.kbc = reinterpret_cast<float*>(base + L.KBC);
  w.KG = reinterpret_cast<float2*>(base + L.KG);
  w.cov = reinterpret_cast<double2*>(base + L.COV);
  plan->flag = reinterpret_cast<int*>(base + L.FLAG);
  w.Vr = reinterpret_cast<double2*>(base + L.VR);
  w.Vp = reinterpret_cast<double2*>(base + L.VP);
  w.pdfp = reinterpret_cast<double*>(base + L.PDFP);
  w.ppp = reinterpret_cast<double*>(base + L.PPP);
  w.scal = reinterpret_cast<double2*>(base + L.SCAL);

  // FP64 host tables, stored as float32.
  std::vector<double2> tw(s.G);
  for (int m = 0; m < s.G; ++m) {
    const double a = 2.0 * M_PI * m / s.G;
    tw[m] = make_double2(std::cos(a), std::sin(a));
  }
  std::vector<float> dinv((size_t)s.GC * s.GC);
  for (int i = 0; i < s.GC; ++i) {
    for (int ic = 0; ic < s.GC; ++ic) {
      const double ky = (double)(i - s.GC / 2) / s.G, kx = (double)(ic - s.GC / 2) / s.G;
      const double wgt = std::pow(1.0 + p->sob_a * (kx * kx + ky * ky), p->sob_l);
      dinv[(size_t)i * s.GC + ic] = (float)(1.0 / (s.G * wgt));
    }
  }
  // deapodisation of the Kaiser-Bessel gridding, 1 / (sqrt(R) c(r)) per axis
  std::vector<float> kbc(s.R);
  const double beta = nlv::kb_beta();
  for (int i = 0; i < s.R; ++i)
    kbc[i] = (float)(1.0 / (std::sqrt((double)s.R) * kb_phi_hat((double)(i - s.R / 2) / s.G, beta)));
  hipError_t e = hipMemcpyAsync(w.tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice, plan->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(w.dinv, dinv.data(), dinv.size() * sizeof(float), hipMemcpyHostToDevice, plan->stream);
  if (e == hipSuccess && s.kb)
    e = hipMemcpyAsync(w.kbc, kbc.data(), kbc.size() * sizeof(float), hipMemcpyHostToDevice, plan->stream);
  if (e == hipSuccess) e = nlv::launch_fill_int(plan->stream, plan->flag, 0);
  if (e == hipSuccess) e = hipStreamSynchronize(plan->stream);
  if (e != hipSuccess) {
    std::string m = std::string("HIP error uploading tables: ") + hipGetErrorString(e);
    release_plan(plan);
    return fail(nullptr, NLINV_E_HIP, m);
  }
  *out = plan;
  return NLINV_OK;
}

int nlinv_plan_create(const nlinv_params* p, void* stream, void* d_workspace, size_t ws_bytes,
                      nlinv_plan* out) {
  return create_plan(p, stream, d_workspace, ws_bytes, out, false);
}

int nlinv_plan_workspace_size(const nlinv_params* p, size_t* bytes) { return nlinv_workspace_size(p, bytes); }

int nlinv_set_budget(int32_t device, size_t budget_bytes) {
  if (device < 0 || device >= MAX_DEV) return fail(nullptr, NLINV_E_ARG, "device must be in [0, 63]");
  std::lock_guard<std::mutex> lk(g_dev_mu);
  g_budget[device] = budget_bytes;
  return NLINV_OK;
}

int nlinv_budget_used(int32_t device, size_t* used_bytes) {
  if (device < 0 || device >= MAX_DEV) return fail(nullptr, NLINV_E_ARG, "device must be in [0, 63]");
  if (!used_bytes) return fail(nullptr, NLINV_E_ARG, "used_bytes is NULL");
  std::lock_guard<std::mutex> lk(g_dev_mu);
  *used_bytes = g_used[device];
  return NLINV_OK;
}

int nlinv_plan_create_static(const nlinv_params* p, void* stream, nlinv_plan* out) {
  if (!out) return fail(nullptr, NLINV_E_ARG, "out is NULL");
  *out = nullptr;
  Shape s;
  Layout L;
  std::string err;
  const int rc = derive(p, &s, &L, &err);
  if (rc != NLINV_OK) return fail(nullptr, rc, err);
  if (L.total > NLINV_STATIC_WORKSPACE_BYTES)
    return fail(nullptr, NLINV_E_WORKSPACE,
                "the plan needs " + std::to_string(L.total) + " bytes of workspace, more than the static workspace's " +
                    std::to_string((size_t)NLINV_STATIC_WORKSPACE_BYTES) + " (use nlinv_plan_create)");
  void* base = nullptr;
  const int rc2 = static_workspace(&base);
  if (rc2 != NLINV_OK) return rc2;
  return create_plan(p, stream, base, NLINV_STATIC_WORKSPACE_BYTES, out, true);
}

int nlinv_plan_destroy(nlinv_plan plan) {
  if (!plan) return fail(nullptr, NLINV_E_ARG, "plan is NULL");
  for (hipEvent_t e : plan->ev) (void)hipEventDestroy(e);
  for (auto& kv : plan->graph_cache) (void)hipGraphExecDestroy(kv.second);
  {
    std::lock_guard<std::mutex> lk(g_multi_mu);
    for (auto it = g_multi.begin(); it != g_multi.end();) {
      const auto& ids = it->second.ids;
      if (std::find(ids.begin(), ids.end(), plan->id) != ids.end()) {
        (void)hipGraphExecDestroy(it->second.exec);
        it = g_multi.erase(it);
      } else {
        ++it;
      }
    }
  }
  if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
  for (hipStream_t b : plan->branch) (void)hipStreamDestroy(b);
  for (hipEvent_t e : plan->bev) (void)hipEventDestroy(e);
  release_plan(plan);
  return NLINV_OK;
}

int nlinv_set_stream(nlinv_plan plan, void* stream) {
  NLV_CHECK(check_plan(plan));
  plan->stream = reinterpret_cast<hipStream_t>(stream);
  return NLINV_OK;
}

int nlinv_psf(nlinv_plan plan, const float* d_traj, int32_t turn) {
  NLV_CHECK(check_plan(plan));
  return nlinv_psf_spokes(plan, d_traj, plan->p.K, turn);
}

int nlinv_psf_spokes(nlinv_plan plan, const float* d_traj, int32_t spokes, int32_t turn) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_traj, "d_traj"));
  if (turn < 0 || turn >= plan->s.U) return fail(plan, NLINV_E_ARG, "turn out of range [0, U)");
  if (spokes < 1 || spokes > plan->p.K) return fail(plan, NLINV_E_ARG, "spokes must be in [1, K]");
  return build_turn(plan, d_traj, turn, (int)((long long)spokes * (plan->s.S / plan->p.K)));
}

int nlinv_psf_samples(nlinv_plan plan, const float* d_traj, int64_t samples, int32_t turn) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_traj, "d_traj"));
  if (turn < 0 || turn >= plan->s.U) return fail(plan, NLINV_E_ARG, "turn out of range [0, U)");
  if (samples < 1 || samples > plan->s.S) return fail(plan, NLINV_E_ARG, "samples must be in [1, K * S_r]");
  return build_turn(plan, d_traj, turn, (int)samples);
}

int nlinv_grid(nlinv_plan plan, const float* d_traj, const nlinv_c64* d_y, const int32_t* h_turn,
               nlinv_c64* d_z) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_traj, "d_traj"));
  NLV_CHECK(check_ptr(plan, d_y, "d_y"));
  NLV_CHECK(check_ptr(plan, d_z, "d_z"));
  const Shape& s = plan->s;
  if (h_turn) {
    for (int b = 0; b < s.B; ++b)
      if (h_turn[b] < 0 || h_turn[b] >= s.U) return fail(plan, NLINV_E_ARG, "turn out of range [0, U)");
    for (int b = 0; b < s.B; ++b) {
      const int t = h_turn[b];
      if (plan->psf_valid[t]) continue;
      NLV_CHECK(build_turn(plan, d_traj + (size_t)b * s.S * 2, t, (int)s.S));
    }
    if (s.kb) {
      nlv::TurnArgs turns;
      std::memset(&turns, 0, sizeof(turns));
      for (int b = 0; b < s.B; ++b) turns.t[b] = h_turn[b];
      NLV_HIP(plan, timed(plan, NLINV_KT_GRID, [&] {
                return plan->t->kb_grid(s, plan->w, plan->stream, turns, reinterpret_cast<const float2*>(d_y),
                                        reinterpret_cast<float2*>(d_z));
              }));
      return NLINV_OK;
    }
  }
  NLV_HIP(plan, timed(plan, NLINV_KT_GRID, [&] {
            return nlv::launch_grid(s, plan->w, plan->stream, d_traj, reinterpret_cast<const float2*>(d_y),
                                    reinterpret_cast<float2*>(d_z));
          }));
  return NLINV_OK;
}

// CG iteration form: the plan's cg_passes, or six passes (the form that moves
// the fewest bytes; the choice does not depend on the batch size, so that an
// item of a batch reconstructs the same bits as a plan of batch one)
static int cg_passes(nlinv_plan plan) { return plan->p.cg_passes == 4 ? 4 : 6; }

// Enqueue Newton steps m0 <= m < m1 of the reconstruction on plan->stream
// (validated arguments); alpha_m follows the schedule from step 0.
// Enqueue one IRGNM update x_hat <- x_hat + h on plan->stream: the right-hand
// side at x_hat, then C CG iterations from h = 0 (validated arguments).
static int enqueue_newton_step(nlinv_plan plan, const nlv::TurnArgs& turns, const float2* z, const float2* xp,
                               float2* xh, double alpha, int C) {
  const Shape& s = plan->s;
  Bufs& w = plan->w;
  hipStream_t st = plan->stream;
  const Shape& sg = s;
  const int kt_toep = NLINV_KT_TOEPLITZ_ROWS;
  // right-hand side: DF^H (y - F x_n) - alpha (x_n - x_prev), in image space through z
  NLV_HIP(plan, timed(plan, NLINV_KT_COIL_ROWS, [&] { return plan->t->coil_rows(sg, w, st, xh); }));
  NLV_HIP(plan, timed(plan, NLINV_KT_COIL_COLS, [&] {
            return plan->t->cols_fwd(sg, w, st, 0, w.CO, xh, nullptr, w.U2);
          }));
  NLV_HIP(plan, timed(plan, kt_toep, [&] { return plan->t->toep_rows(sg, w, st, turns); }));
  NLV_HIP(plan, timed(plan, NLINV_KT_BACK_COLS, [&] {
            return plan->t->cols_back(sg, w, st, 1, w.U2, w.CO, xh, z);
          }));
  NLV_HIP(plan, timed(plan, NLINV_KT_COILH_ROWS, [&] {
            return plan->t->coilh_rows(sg, w, st, 1, nullptr, xh, xp, alpha, w.Rv, w.Pv[0]);
          }));
  // (the image block of b rides in the coil-adjoint pass's image blocks)
  int ncur = s.NX3 + s.NRQ, nprev = 0;
  if (cg_passes(plan) == 4) {
    // four dependent kernels per CG iteration (see the four-pass section of
    // nlinv_kernels.h): the direction update, the x-stage of W^-1 p and the
    // CG vector updates ride in the operator's passes
    for (int i = 0; i < C; ++i) {
      double2* pn = w.Pv[i & 1];
      const double2* po = w.Pv[(i + 1) & 1];
      const Partials sc{w.rr[i & 1], ncur, w.rr[(i + 1) & 1], nprev, s.stride};
      const int first = i == 0, last = i == C - 1;
      NLV_HIP(plan, timed(plan, NLINV_KT_COIL_COLS, [&] {
                return plan->t->cg_cols_fwd(sg, w, st, xh, po, pn, sc, first);
              }));
      NLV_HIP(plan, timed(plan, kt_toep, [&] { return plan->t->cg_toep_rows(sg, w, st, turns); }));
      const nlv::CGRed red{w.scal, w.pdfp, s.NTB, s.NTB, w.ppp, s.NPP, s.NPP, w.rr[i & 1], ncur, s.stride, alpha, 0};
      NLV_HIP(plan, timed(plan, NLINV_KT_BACK_COLS, [&] { return plan->t->cg_cols_back(sg, w, st, xh, red); }));
      NLV_HIP(plan, timed(plan, NLINV_KT_COILH_ROWS, [&] {
                return plan->t->cg_coilh(sg, w, st, pn, xh, alpha, w.rr[(i + 1) & 1], first, last);
              }));
      nprev = ncur;
      ncur = s.NX3 + s.NRQ;
    }
  } else {
    // six dependent kernels per CG iteration: coil rows with the direction
    // update, the operator's four passes, the CG vector step
    for (int i = 0; i < C; ++i) {
      double2* pc = w.Pv[i & 1];
      double2* pp = w.Pv[(i + 1) & 1];
      const Partials sc{w.rr[i & 1], ncur, w.rr[(i + 1) & 1], nprev, s.stride};
      const bool upd = i > 0;
      NLV_HIP(plan, timed(plan, NLINV_KT_COIL_ROWS, [&] {
                return plan->t->coil_rows_cg(sg, w, st, upd ? pp : pc, upd ? w.Rv : nullptr,
                                             upd ? pc : nullptr, sc);
              }));
      NLV_HIP(plan, timed(plan, NLINV_KT_COIL_COLS, [&] {
                return plan->t->cols_fwd(sg, w, st, 1, w.CO, xh, pc, w.U2);
              }));
      NLV_HIP(plan, timed(plan, kt_toep, [&] { return plan->t->toep_rows(sg, w, st, turns); }));
      NLV_HIP(plan, timed(plan, NLINV_KT_BACK_COLS, [&] {
                return plan->t->cols_back(sg, w, st, 0, w.U2, w.CO, xh, nullptr);
              }));
      NLV_HIP(plan, timed(plan, NLINV_KT_COILH_ROWS, [&] {
                return plan->t->coilh_rows(sg, w, st, 0, pc, xh, nullptr, alpha, w.Q, nullptr);
              }));
      NLV_HIP(plan, timed(plan, NLINV_KT_CG_UPDATE, [&] {
                return nlv::launch_cg_update(s, w, st, i, i == C - 1, pc, sc, xh);
              }));
      nprev = ncur;
      ncur = s.NCH;
    }
  }
  return NLINV_OK;
}

static int enqueue_reconstruct(nlinv_plan plan, const nlv::TurnArgs& turns, const float2* z,
                               const float2* xp, float2* xh, int init, int m0, int m1, float* d_img,
                               float2* d_coils) {
  const Shape& s = plan->s;
  Bufs& w = plan->w;
  hipStream_t st = plan->stream;

  if (init == 1) NLV_HIP(plan, nlv::launch_init_x(s, st, xh, nullptr, 1));
  if (init == 2) NLV_HIP(plan, nlv::launch_init_x(s, st, xh, xp, 2));

  double alpha = plan->p.alpha0;
  for (int n = 0; n < m0; ++n) alpha = std::max(alpha * plan->p.alpha_q, plan->p.alpha_min);
  for (int n = m0; n < m1; ++n) {
    NLV_CHECK(enqueue_newton_step(plan, turns, z, xp, xh, alpha, plan->p.cg));
    alpha = std::max(alpha * plan->p.alpha_q, plan->p.alpha_min);
  }

  if (d_img || d_coils) {
    float2* co = d_coils ? d_coils : w.CO;
    NLV_CHECK(coils_into(plan, xh, co));
    if (d_img) NLV_HIP(plan, nlv::launch_image(s, st, xh, co, d_img));
  }
  return NLINV_OK;
}

// With NLINV_F_CHECK_FINITE: flag non-finite values of a result (outside any
// captured graph; the flag stays set until nlinv_sync reports it).
static int check_finite(nlinv_plan plan, const float2* x, long long n) {
  if (!(plan->p.flags & NLINV_F_CHECK_FINITE)) return NLINV_OK;
  NLV_HIP(plan, nlv::launch_check_finite(plan->stream, x, n, plan->flag));
  return NLINV_OK;
}

// Capture the launch sequence enqueued by `body` once per key and replay it.
static int run_captured(nlinv_plan plan, std::vector<uintptr_t> key, const std::function<int()>& body) {
  key.push_back((uintptr_t)plan->s.B);
  auto it = plan->graph_cache.find(key);
  if (it == plan->graph_cache.end()) {
    if (plan->graph_cache.size() >= 64) {
      for (auto& kv : plan->graph_cache) (void)hipGraphExecDestroy(kv.second);
      plan->graph_cache.clear();
    }
    if (!plan->cap_stream) NLV_HIP(plan, hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking));
    hipStream_t user = plan->stream;
    plan->stream = plan->cap_stream;
    hipError_t e = hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      plan->stream = user;
      return fail_hip(plan, e, "hipStreamBeginCapture");
    }
    const int rc = body();
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(plan->cap_stream, &graph);
    plan->stream = user;
    if (rc != NLINV_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail_hip(plan, e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail_hip(plan, e, "hipGraphInstantiate");
    it = plan->graph_cache.emplace(key, exec).first;
  }
  NLV_HIP(plan, hipGraphLaunch(it->second, plan->stream));
  return NLINV_OK;
}

int nlinv_reconstruct(nlinv_plan plan, const nlinv_c64* d_z, const int32_t* h_turn,
                      const nlinv_c64* d_xprev, nlinv_c64* d_xhat, int32_t init, float* d_img,
                      nlinv_c64* d_coils) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_z, "d_z"));
  NLV_CHECK(check_ptr(plan, d_xhat, "d_xhat"));
  NLV_CHECK(check_ptr(plan, d_xprev, "d_xprev", true));
  NLV_CHECK(check_ptr(plan, d_img, "d_img", true));
  NLV_CHECK(check_ptr(plan, d_coils, "d_coils", true));
  if (init < 0 || init > 2) return fail(plan, NLINV_E_ARG, "init must be 0, 1 or 2");
  if (init == 2 && !d_xprev) return fail(plan, NLINV_E_ARG, "init = 2 needs d_xprev");
  if (d_xprev && (const void*)d_xprev == (const void*)d_xhat)
    return fail(plan, NLINV_E_ARG, "d_xhat must not alias d_xprev");
  nlv::TurnArgs turns;
  NLV_CHECK(turns_of(plan, h_turn, &turns));
  const float2* z = reinterpret_cast<const float2*>(d_z);
  const float2* xp = reinterpret_cast<const float2*>(d_xprev);
  float2* xh = reinterpret_cast<float2*>(d_xhat);
  float2* co = reinterpret_cast<float2*>(d_coils);
  const int M = plan->p.newton;
  auto body = [&] { return enqueue_reconstruct(plan, turns, z, xp, xh, init, 0, M, d_img, co); };
  if (plan->graphs && plan->timer_kid == NLINV_KT_NONE) {
    std::vector<uintptr_t> key = {0, (uintptr_t)z, (uintptr_t)xp, (uintptr_t)xh, (uintptr_t)init,
                                  (uintptr_t)d_img, (uintptr_t)co};
    for (int b = 0; b < plan->s.B; ++b) key.push_back((uintptr_t)turns.t[b]);
    NLV_CHECK(run_captured(plan, std::move(key), body));
  } else {
    NLV_CHECK(body());
  }
  return check_finite(plan, xh, (long long)plan->s.B * plan->s.X);
}

int nlinv_reconstruct_multi(int32_t count, const nlinv_plan* plans, const nlinv_c64* const* d_z,
                            const int32_t* const* h_turn, const nlinv_c64* const* d_xprev,
                            nlinv_c64* const* d_xhat, const int32_t* init, float* const* d_img) {
  if (count < 1 || count > NLINV_MAX_MULTI) return fail(nullptr, NLINV_E_ARG, "count must be in [1, 8]");
  if (!plans || !d_z || !h_turn || !d_xprev || !d_xhat || !init || !d_img)
    return fail(nullptr, NLINV_E_ARG, "NULL array");
  std::vector<nlv::TurnArgs> turns(count);
  std::vector<uint64_t> key = {(uint64_t)count};
  std::vector<uint64_t> ids;
  for (int i = 0; i < count; ++i) {
    nlinv_plan plan = plans[i];
    NLV_CHECK(check_plan(plan));
    for (int k = 0; k < i; ++k)
      if (plans[k] == plan) return fail(plan, NLINV_E_ARG, "a plan appears twice");
    if (plan->device != plans[0]->device) return fail(plan, NLINV_E_ARG, "the plans must live on one device");
    if (plan->timer_kid != NLINV_KT_NONE) return fail(plan, NLINV_E_STATE, "a kernel timer is armed");
    if (plan->is_static) return fail(plan, NLINV_E_STATE, "plans on the static workspace launch eagerly");
    NLV_CHECK(check_ptr(plan, d_z[i], "d_z"));
    NLV_CHECK(check_ptr(plan, d_xhat[i], "d_xhat"));
    NLV_CHECK(check_ptr(plan, d_xprev[i], "d_xprev", true));
    NLV_CHECK(check_ptr(plan, d_img[i], "d_img", true));
    if (init[i] < 0 || init[i] > 2) return fail(plan, NLINV_E_ARG, "init must be 0, 1 or 2");
    if (init[i] == 2 && !d_xprev[i]) return fail(plan, NLINV_E_ARG, "init = 2 needs d_xprev");
    if (d_xprev[i] && (const void*)d_xprev[i] == (const void*)d_xhat[i])
      return fail(plan, NLINV_E_ARG, "d_xhat must not alias d_xprev");
    NLV_CHECK(turns_of(plan, h_turn[i], &turns[i]));
    ids.push_back(plan->id);
    key.insert(key.end(), {plan->id, plan->gen, (uint64_t)plan->s.B, (uint64_t)(uintptr_t)d_z[i],
                           (uint64_t)(uintptr_t)d_xprev[i], (uint64_t)(uintptr_t)d_xhat[i], (uint64_t)init[i],
                           (uint64_t)(uintptr_t)d_img[i]});
    for (int b = 0; b < plan->s.B; ++b) key.push_back((uint64_t)(uint32_t)turns[i].t[b]);
  }
  nlinv_plan lead = plans[0];
  hipGraphExec_t exec = nullptr;
  // the table is process-wide: held from the lookup through the launch, so no
  // other thread's eviction can release the graph in between
  std::unique_lock<std::mutex> lk(g_multi_mu);
  {
    auto it = g_multi.find(key);
    if (it != g_multi.end()) exec = it->second.exec;
  }
  if (!exec) {
    // capture: fork from the lead plan's capture stream into one stream per
    // plan, each plan's launch sequence on its own, join back
    for (int i = 0; i < count; ++i)
      if (!plans[i]->cap_stream)
        NLV_HIP(plans[i], hipStreamCreateWithFlags(&plans[i]->cap_stream, hipStreamNonBlocking));
    std::vector<hipEvent_t> ev(count + 1, nullptr);
    for (auto& e : ev) {
      const hipError_t he = hipEventCreateWithFlags(&e, hipEventDisableTiming);
      if (he != hipSuccess) {
        for (auto& x : ev)
          if (x) (void)hipEventDestroy(x);
        return fail_hip(lead, he, "hipEventCreateWithFlags");
      }
    }
    struct Cleanup {
      std::vector<hipEvent_t>& ev;
      ~Cleanup() {
        for (auto& x : ev) (void)hipEventDestroy(x);
      }
    } cleanup{ev};
    hipStream_t origin = lead->cap_stream;
    hipError_t e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail_hip(lead, e, "hipStreamBeginCapture");
    int rc = NLINV_OK;
    e = hipEventRecord(ev[0], origin);
    for (int i = 0; i < count && rc == NLINV_OK && e == hipSuccess; ++i) {
      nlinv_plan plan = plans[i];
      hipStream_t br = plan->cap_stream;
      if (br != origin) e = hipStreamWaitEvent(br, ev[0], 0);
      if (e != hipSuccess) break;
      hipStream_t user = plan->stream;
      plan->stream = br;
      rc = enqueue_reconstruct(plan, turns[i], reinterpret_cast<const float2*>(d_z[i]),
                               reinterpret_cast<const float2*>(d_xprev[i]), reinterpret_cast<float2*>(d_xhat[i]),
                               init[i], 0, plan->p.newton, d_img[i], nullptr);
      plan->stream = user;
      if (rc == NLINV_OK && br != origin) {
        e = hipEventRecord(ev[i + 1], br);
        if (e == hipSuccess) e = hipStreamWaitEvent(origin, ev[i + 1], 0);
      }
    }
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(origin, &graph);
    if (rc != NLINV_OK || e != hipSuccess || ee != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (rc != NLINV_OK) return rc;
      return fail_hip(lead, e != hipSuccess ? e : ee, "multi-plan capture");
    }
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail_hip(lead, e, "hipGraphInstantiate");
    if (g_multi.size() >= 64) {
      for (auto& kv : g_multi) (void)hipGraphExecDestroy(kv.second.exec);
      g_multi.clear();
    }
    g_multi.emplace(key, MultiGraph{exec, ids});
  }
  NLV_HIP(lead, hipGraphLaunch(exec, lead->stream));
  lk.unlock();
  for (int i = 0; i < count; ++i) {
    nlinv_plan plan = plans[i];
    hipStream_t user = plan->stream;
    plan->stream = lead->stream;
    const int rc = check_finite(plan, reinterpret_cast<float2*>(d_xhat[i]), (long long)plan->s.B * plan->s.X);
    plan->stream = user;
    NLV_CHECK(rc);
  }
  return NLINV_OK;
}

int nlinv_newton_step(nlinv_plan plan, const int32_t* h_turn, const nlinv_c64* d_z, const nlinv_c64* d_xprev,
                      double alpha, int32_t cg, nlinv_c64* d_xhat) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_z, "d_z"));
  NLV_CHECK(check_ptr(plan, d_xhat, "d_xhat"));
  NLV_CHECK(check_ptr(plan, d_xprev, "d_xprev", true));
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(plan, NLINV_E_ARG, "alpha must be finite and >= 0");
  if (cg < 1 || cg > 100000) return fail(plan, NLINV_E_ARG, "cg must be in [1, 100000]");
  if (d_xprev && (const void*)d_xprev == (const void*)d_xhat)
    return fail(plan, NLINV_E_ARG, "d_xhat must not alias d_xprev");
  nlv::TurnArgs turns;
  NLV_CHECK(turns_of(plan, h_turn, &turns));
  NLV_CHECK(enqueue_newton_step(plan, turns, reinterpret_cast<const float2*>(d_z),
                                reinterpret_cast<const float2*>(d_xprev), reinterpret_cast<float2*>(d_xhat), alpha,
                                cg));
  return check_finite(plan, reinterpret_cast<float2*>(d_xhat), (long long)plan->s.B * plan->s.X);
}

int nlinv_set_coil_weights(nlinv_plan plan, const float* d_winv) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_winv, "d_winv", true));
  float* t = d_winv ? const_cast<float*>(d_winv) : plan->dinv_own;
  if (t != plan->w.dinv) {
    // captured graphs hold the table's address: drop them (the multi-plan
    // graphs are keyed by the generation)
    for (auto& kv : plan->graph_cache) (void)hipGraphExecDestroy(kv.second);
    plan->graph_cache.clear();
    ++plan->gen;
    plan->w.dinv = t;
  }
  return NLINV_OK;
}

// The buffers of item k alone, as a batch-1 plan of the same shape holds
// them: every per-item array advanced by k items (the workspace is item
// major), the tables and shared scratch unchanged.
static Bufs item_view(const Bufs& w, const Shape& s, int k) {
  Bufs v = w;
  const size_t K = (size_t)k, J = s.J, R = s.R, G = s.G, GC = s.GC, X = (size_t)s.X;
  v.CO += K * J * R * R;
  v.U1 += K * J * GC * R;
  v.U2 = static_cast<double2*>(w.U2) + K * J * G * R;
  v.PR += K * J * R * R;
  v.IMG += K * J * R * R;
  v.H += K * X;
  v.Rv += K * X;
  v.Pv[0] += K * X;
  v.Pv[1] += K * X;
  v.Q += K * X;
  v.pq += K * s.stride;
  v.rr[0] += K * s.stride;
  v.rr[1] += K * s.stride;
  v.KG += K * J * G * G;
  v.Vr += K * J * GC * R;
  v.Vp += K * J * GC * R;
  v.pdfp += K * s.NTB;
  v.ppp += K * s.NPP;
  v.scal += K;
  return v;
}

// Newton steps 0 .. m1-1 of the members of a relaxed group, each member as a
// batch-1 chain of its own on a stream of its own (forked from and joined
// back into the plan's stream), so that the chains' kernels overlap.  An
// item computes the same bits at any batch size, so this equals the batched
// launch bit for bit; measured at 160 px (three members, four-pass CG form)
// 7.0 against 7.9 ms for the six Newton steps (five members: 13.5 against
// 10.7 ms, six-pass form 9.8 against 7.8, so only small groups of the
// four-pass form take this path).
static bool members_side_by_side(nlinv_plan plan, int count) {
  // not for plans on the static workspace, whose calls create no streams
  return cg_passes(plan) == 4 && count >= 2 && count <= 3 && plan->timer_kid == NLINV_KT_NONE && !plan->is_static;
}

static int enqueue_members(nlinv_plan plan, int count, const nlv::TurnArgs& turns, const float2* z,
                           float2* xh, int m1) {
  while ((int)plan->branch.size() < count) {
    hipStream_t b = nullptr;
    NLV_HIP(plan, hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
    plan->branch.push_back(b);
  }
  while ((int)plan->bev.size() < count + 1) {
    hipEvent_t e = nullptr;
    NLV_HIP(plan, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    plan->bev.push_back(e);
  }
  struct Restore {
    nlinv_plan p;
    Shape s;
    Bufs w;
    hipStream_t st;
    ~Restore() {
      p->s = s;
      p->w = w;
      p->stream = st;
    }
  } restore{plan, plan->s, plan->w, plan->stream};
  const Shape s0 = plan->s;
  const Bufs w0 = plan->w;
  hipStream_t st0 = plan->stream;
  const size_t X = (size_t)s0.X, ZJ = (size_t)s0.J * s0.R * s0.R;
  NLV_HIP(plan, hipEventRecord(plan->bev[0], st0));
  for (int k = 0; k < count; ++k) {
    hipStream_t br = plan->branch[k];
    NLV_HIP(plan, hipStreamWaitEvent(br, plan->bev[0], 0));
    plan->s = s0;
    set_active(plan, 1);
    plan->w = item_view(w0, s0, k);
    plan->stream = br;
    nlv::TurnArgs tk;
    std::memset(&tk, 0, sizeof(tk));
    tk.t[0] = turns.t[k];
    NLV_CHECK(enqueue_reconstruct(plan, tk, z + k * ZJ, plan->xb + k * X, xh + k * X, 2, 0, m1, nullptr, nullptr));
    NLV_HIP(plan, hipEventRecord(plan->bev[k + 1], br));
    NLV_HIP(plan, hipStreamWaitEvent(st0, plan->bev[k + 1], 0));
  }
  return NLINV_OK;
}

// Frames n0 .. n0+count-1 of one series under the relaxed temporal coupling.
static int enqueue_frames(nlinv_plan plan, int count, const nlv::TurnArgs& turns, const float2* z,
                          const float2* xp, float2* xh, float* d_img, float2* d_coils) {
  const int M = plan->p.newton;
  const Shape& s = plan->s;   // active batch = count
  const size_t X = (size_t)s.X, ZJ = (size_t)s.J * s.R * s.R;
  hipStream_t st = plan->stream;
  // source frame of every member: x_{n0-1}, or (rho = 1, c = 0)
  NLV_HIP(plan, xp ? nlv::launch_init_x(s, st, plan->xb, xp, 3) : nlv::launch_init_x(s, st, plan->xb, nullptr, 1));
  if (M <= 1) {
    if (M == 0) NLV_HIP(plan, nlv::launch_init_x(s, st, xh, plan->xb, 2));
  } else {
    // steps 0 .. M-2 of all members together, from and towards the source
    if (members_side_by_side(plan, count)) {
      NLV_CHECK(enqueue_members(plan, count, turns, z, xh, M - 1));
    } else {
      NLV_CHECK(enqueue_reconstruct(plan, turns, z, plan->xb, xh, 2, 0, M - 1, nullptr, nullptr));
    }
  }
  if (M >= 1) {
    // step M-1 of each member, in order, towards the previous frame
    ActiveGuard guard{plan, count};
    set_active(plan, 1);
    for (int k = 0; k < count; ++k) {
      nlv::TurnArgs tk;
      std::memset(&tk, 0, sizeof(tk));
      tk.t[0] = turns.t[k];
      const float2* prev = k == 0 ? plan->xb : xh + (k - 1) * X;
      // with a single step, h(n, 0) = n - 1 gives the starting point as well
      NLV_CHECK(enqueue_reconstruct(plan, tk, z + k * ZJ, prev, xh + k * X, M == 1 ? 2 : 0, M - 1, M,
                                    nullptr, nullptr));
    }
  }
  if (d_img || d_coils) {
    float2* co = d_coils ? d_coils : plan->w.CO;
    NLV_CHECK(coils_into(plan, xh, co));
    if (d_img) NLV_HIP(plan, nlv::launch_image(s, st, xh, co, d_img));
  }
  return NLINV_OK;
}

int nlinv_reconstruct_frames(nlinv_plan plan, int32_t count, const nlinv_c64* d_z, const int32_t* h_turn,
                             const nlinv_c64* d_xprev, nlinv_c64* d_xhat, float* d_img, nlinv_c64* d_coils) {
  NLV_CHECK(check_plan(plan));
  if (count < 1 || count > plan->p.batch) return fail(plan, NLINV_E_ARG, "count must be in [1, batch]");
  NLV_CHECK(check_ptr(plan, d_z, "d_z"));
  NLV_CHECK(check_ptr(plan, d_xhat, "d_xhat"));
  NLV_CHECK(check_ptr(plan, d_xprev, "d_xprev", true));
  NLV_CHECK(check_ptr(plan, d_img, "d_img", true));
  NLV_CHECK(check_ptr(plan, d_coils, "d_coils", true));
  const size_t X = (size_t)plan->s.X;
  if (d_xprev) {
    const char* a = reinterpret_cast<const char*>(d_xprev);
    const char* b = reinterpret_cast<const char*>(d_xhat);
    if (a < b + (size_t)count * X * 8 && b < a + X * 8)
      return fail(plan, NLINV_E_ARG, "d_xhat must not overlap d_xprev");
  }
  ActiveGuard guard{plan, plan->s.B};
  set_active(plan, count);
  nlv::TurnArgs turns;
  NLV_CHECK(turns_of(plan, h_turn, &turns));
  const float2* z = reinterpret_cast<const float2*>(d_z);
  const float2* xp = reinterpret_cast<const float2*>(d_xprev);
  float2* xh = reinterpret_cast<float2*>(d_xhat);
  float2* co = reinterpret_cast<float2*>(d_coils);
  auto body = [&] { return enqueue_frames(plan, count, turns, z, xp, xh, d_img, co); };
  if (plan->graphs && plan->timer_kid == NLINV_KT_NONE) {
    std::vector<uintptr_t> key = {1, (uintptr_t)z, (uintptr_t)xp, (uintptr_t)xh, (uintptr_t)d_img,
                                  (uintptr_t)co};
    for (int b = 0; b < count; ++b) key.push_back((uintptr_t)turns.t[b]);
    NLV_CHECK(run_captured(plan, std::move(key), body));
  } else {
    NLV_CHECK(body());
  }
  return check_finite(plan, xh, (long long)count * plan->s.X);
}

int nlinv_set_batch(nlinv_plan plan, int32_t b) {
  NLV_CHECK(check_plan(plan));
  if (b < 1 || b > plan->p.batch) return fail(plan, NLINV_E_ARG, "batch must be in [1, plan batch]");
  set_active(plan, b);
  return NLINV_OK;
}

int32_t nlinv_get_batch(nlinv_plan plan) { return plan ? plan->s.B : 0; }

int nlinv_apply_F(nlinv_plan plan, const float* d_traj, const nlinv_c64* d_xhat, nlinv_c64* d_y) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_traj, "d_traj"));
  NLV_CHECK(check_ptr(plan, d_xhat, "d_xhat"));
  NLV_CHECK(check_ptr(plan, d_y, "d_y"));
  const Shape& s = plan->s;
  Bufs& w = plan->w;
  const float2* xh = reinterpret_cast<const float2*>(d_xhat);
  NLV_HIP(plan, plan->t->coil_rows(s, w, plan->stream, xh));
  NLV_HIP(plan, plan->t->cols_fwd(s, w, plan->stream, 2, w.CO, xh, nullptr, w.IMG));
  NLV_HIP(plan, nlv::launch_nudft_fwd(s, plan->stream, d_traj, w.IMG, reinterpret_cast<float2*>(d_y)));
  return NLINV_OK;
}

int nlinv_apply_DF(nlinv_plan plan, const float* d_traj, const nlinv_c64* d_xhat, const nlinv_c64* d_dx,
                   nlinv_c64* d_dy) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_traj, "d_traj"));
  NLV_CHECK(check_ptr(plan, d_xhat, "d_xhat"));
  NLV_CHECK(check_ptr(plan, d_dx, "d_dx"));
  NLV_CHECK(check_ptr(plan, d_dy, "d_dy"));
  const Shape& s = plan->s;
  Bufs& w = plan->w;
  const float2* xh = reinterpret_cast<const float2*>(d_xhat);
  const float2* dx = reinterpret_cast<const float2*>(d_dx);
  const Partials none{};
  NLV_CHECK(coils_into(plan, xh, w.CO));
  NLV_HIP(plan, nlv::launch_to_double(s, plan->stream, w.Pv[0], dx));
  NLV_HIP(plan, plan->t->coil_rows_cg(s, w, plan->stream, w.Pv[0], nullptr, nullptr, none));
  NLV_HIP(plan, plan->t->cols_fwd(s, w, plan->stream, 3, w.CO, xh, w.Pv[0], w.IMG));
  NLV_HIP(plan, nlv::launch_nudft_fwd(s, plan->stream, d_traj, w.IMG, reinterpret_cast<float2*>(d_dy)));
  return NLINV_OK;
}

int nlinv_apply_DFH(nlinv_plan plan, const float* d_traj, const nlinv_c64* d_xhat, const nlinv_c64* d_dy,
                    nlinv_c64* d_dx) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_traj, "d_traj"));
  NLV_CHECK(check_ptr(plan, d_xhat, "d_xhat"));
  NLV_CHECK(check_ptr(plan, d_dy, "d_dy"));
  NLV_CHECK(check_ptr(plan, d_dx, "d_dx"));
  const Shape& s = plan->s;
  Bufs& w = plan->w;
  const float2* xh = reinterpret_cast<const float2*>(d_xhat);
  float2* dx = reinterpret_cast<float2*>(d_dx);
  NLV_CHECK(coils_into(plan, xh, w.CO));
  NLV_HIP(plan, nlv::launch_grid(s, w, plan->stream, d_traj, reinterpret_cast<const float2*>(d_dy), w.IMG));
  NLV_HIP(plan, plan->t->cols_back(s, w, plan->stream, 2, w.IMG, w.CO, xh, nullptr));
  NLV_HIP(plan, plan->t->coilh_rows(s, w, plan->stream, 2, nullptr, xh, nullptr, 0.0, w.Q, nullptr));
  NLV_HIP(plan, nlv::launch_finalize(s, w, plan->stream, nullptr, 0.0, dx));
  return NLINV_OK;
}

int nlinv_compress(nlinv_plan plan, const nlinv_c64* d_cc, int32_t J_phys, const nlinv_c64* d_yp,
                   nlinv_c64* d_y) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_cc, "d_cc"));
  NLV_CHECK(check_ptr(plan, d_yp, "d_yp"));
  NLV_CHECK(check_ptr(plan, d_y, "d_y"));
  if (J_phys < 1 || J_phys > nlv::MAX_JP) return fail(plan, NLINV_E_ARG, "J_phys must be in [1, 128]");
  NLV_HIP(plan, nlv::launch_compress(plan->s, plan->stream, reinterpret_cast<const float2*>(d_cc), J_phys,
                                     reinterpret_cast<const float2*>(d_yp), reinterpret_cast<float2*>(d_y)));
  return NLINV_OK;
}

int nlinv_compression_matrix(nlinv_plan plan, const nlinv_c64* d_y0, int32_t J_phys, nlinv_c64* d_cc) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_y0, "d_y0"));
  NLV_CHECK(check_ptr(plan, d_cc, "d_cc"));
  const Shape& s = plan->s;
  if (J_phys < s.J || J_phys > nlv::MAX_JP) return fail(plan, NLINV_E_ARG, "J_phys must be in [J, 128]");
  NLV_HIP(plan, nlv::launch_channel_cov(s, plan->stream, reinterpret_cast<const float2*>(d_y0), J_phys, plan->w.cov));
  NLV_HIP(plan, nlv::launch_compression_eig(plan->stream, plan->w.cov, plan->w.cov + (size_t)nlv::MAX_JP * nlv::MAX_JP,
                                            J_phys, s.J, reinterpret_cast<float2*>(d_cc)));
  return NLINV_OK;
}

int nlinv_apply_WH(nlinv_plan plan, const nlinv_c64* d_coils, nlinv_c64* d_xhat) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_coils, "d_coils"));
  NLV_CHECK(check_ptr(plan, d_xhat, "d_xhat"));
  const Shape& s = plan->s;
  Bufs& w = plan->w;
  const void* c = d_coils;
  NLV_HIP(plan, plan->t->cols_back(s, w, plan->stream, 3, c, nullptr, nullptr, nullptr));
  NLV_HIP(plan, plan->t->coilh_rows(s, w, plan->stream, 2, nullptr, nullptr, nullptr, 0.0, w.Q, nullptr));
  NLV_HIP(plan, nlv::launch_finalize(s, w, plan->stream, nullptr, 0.0, reinterpret_cast<float2*>(d_xhat), false));
  return NLINV_OK;
}

int nlinv_apply_normal(nlinv_plan plan, const int32_t* h_turn, const nlinv_c64* d_xhat, double alpha,
                       const nlinv_c64* d_p, nlinv_c64* d_q) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_xhat, "d_xhat"));
  NLV_CHECK(check_ptr(plan, d_p, "d_p"));
  NLV_CHECK(check_ptr(plan, d_q, "d_q"));
  if (!std::isfinite(alpha)) return fail(plan, NLINV_E_ARG, "alpha must be finite");
  if ((const void*)d_p == (const void*)d_q) return fail(plan, NLINV_E_ARG, "d_q must not alias d_p");
  nlv::TurnArgs turns;
  NLV_CHECK(turns_of(plan, h_turn, &turns));
  const Shape& s = plan->s;
  Bufs& w = plan->w;
  hipStream_t st = plan->stream;
  const float2* xh = reinterpret_cast<const float2*>(d_xhat);
  const float2* p = reinterpret_cast<const float2*>(d_p);
  float2* q = reinterpret_cast<float2*>(d_q);
  const Partials none{};
  NLV_CHECK(coils_into(plan, xh, w.CO));
  double2* pd = w.Pv[0];
  NLV_HIP(plan, nlv::launch_to_double(s, st, pd, p));
  NLV_HIP(plan, plan->t->coil_rows_cg(s, w, st, pd, nullptr, nullptr, none));
  NLV_HIP(plan, plan->t->cols_fwd(s, w, st, 1, w.CO, xh, pd, w.U2));
  NLV_HIP(plan, plan->t->toep_rows(s, w, st, turns));
  NLV_HIP(plan, plan->t->cols_back(s, w, st, 0, w.U2, w.CO, xh, nullptr));
  NLV_HIP(plan, plan->t->coilh_rows(s, w, st, 0, pd, xh, nullptr, alpha, w.Q, nullptr));
  NLV_HIP(plan, nlv::launch_finalize(s, w, st, pd, alpha, q));
  return NLINV_OK;
}

int nlinv_apply_normal_multi(int32_t count, const nlinv_plan* plans, const int32_t* const* h_turns,
                             const nlinv_c64* const* d_xhat, const double* alpha, const nlinv_c64* const* d_p,
                             nlinv_c64* const* d_q) {
  if (count < 1 || count > 3) return fail(nullptr, NLINV_E_ARG, "count must be in [1, 3]");
  if (!plans || !h_turns || !d_xhat || !alpha || !d_p || !d_q) return fail(nullptr, NLINV_E_ARG, "NULL array");
  int slot_of[3] = {-1, -1, -1};   // plan index per ragged slot (grid 256, 320, 384)
  nlv::TurnArgs turns[3];
  for (int i = 0; i < count; ++i) {
    nlinv_plan plan = plans[i];
    NLV_CHECK(check_plan(plan));
    NLV_CHECK(check_ptr(plan, d_xhat[i], "d_xhat"));
    NLV_CHECK(check_ptr(plan, d_p[i], "d_p"));
    NLV_CHECK(check_ptr(plan, d_q[i], "d_q"));
    if (!std::isfinite(alpha[i])) return fail(plan, NLINV_E_ARG, "alpha must be finite");
    if ((const void*)d_p[i] == (const void*)d_q[i]) return fail(plan, NLINV_E_ARG, "d_q must not alias d_p");
    if (plan->device != plans[0]->device) return fail(plan, NLINV_E_ARG, "the plans must live on one device");
    const int G = plan->s.G;
    const int slot = G == 256 ? 0 : (G == 320 ? 1 : (G == 384 ? 2 : -1));
    if (slot < 0) return fail(plan, NLINV_E_SIZE, "the ragged pass takes grids 256, 320 and 384");
    if (slot_of[slot] >= 0) return fail(plan, NLINV_E_ARG, "one plan per grid side");
    if (plan->s.split != 0) return fail(plan, NLINV_E_ARG, "the ragged pass uses the default factorisation");
    slot_of[slot] = i;
    NLV_CHECK(turns_of(plan, h_turns[i], &turns[i]));
  }
  hipStream_t st = plans[0]->stream;
  nlinv_plan first = plans[0];
  const Partials none{};
  // every plan's passes on the first plan's stream
  struct StreamSwap {
    nlinv_plan p;
    hipStream_t keep;
    ~StreamSwap() { p->stream = keep; }
  };
  for (int i = 0; i < count; ++i) {
    nlinv_plan plan = plans[i];
    StreamSwap sw{plan, plan->stream};
    plan->stream = st;
    const Shape& s = plan->s;
    Bufs& w = plan->w;
    const float2* xh = reinterpret_cast<const float2*>(d_xhat[i]);
    NLV_CHECK(coils_into(plan, xh, w.CO));
    NLV_HIP(plan, nlv::launch_to_double(s, st, w.Pv[0], reinterpret_cast<const float2*>(d_p[i])));
    NLV_HIP(plan, plan->t->coil_rows_cg(s, w, st, w.Pv[0], nullptr, nullptr, none));
    NLV_HIP(plan, plan->t->cols_fwd(s, w, st, 1, w.CO, xh, w.Pv[0], w.U2));
  }
  nlv::ToepShape shapes[3];
  for (int k = 0; k < 3; ++k) {
    shapes[k] = nlv::ToepShape{nullptr, nullptr, nullptr, nlv::TurnArgs{}, 1, 0};
    const int i = slot_of[k];
    if (i < 0) continue;
    const Shape& s = plans[i]->s;
    const Bufs& w = plans[i]->w;
    shapes[k] = nlv::ToepShape{static_cast<double2*>(w.U2), w.P, w.tw, turns[i], s.J, s.B * s.J * s.G};
  }
  NLV_HIP(first, nlv::launch_toep_ragged(st, shapes));
  for (int i = 0; i < count; ++i) {
    nlinv_plan plan = plans[i];
    const Shape& s = plan->s;
    Bufs& w = plan->w;
    const float2* xh = reinterpret_cast<const float2*>(d_xhat[i]);
    NLV_HIP(plan, plan->t->cols_back(s, w, st, 0, w.U2, w.CO, xh, nullptr));
    NLV_HIP(plan, plan->t->coilh_rows(s, w, st, 0, w.Pv[0], xh, nullptr, alpha[i], w.Q, nullptr));
    NLV_HIP(plan, nlv::launch_finalize(s, w, st, w.Pv[0], alpha[i], reinterpret_cast<float2*>(d_q[i])));
  }
  return NLINV_OK;
}

int nlinv_apply_normal2(nlinv_plan plan, const int32_t* h_turn, const nlinv_c64* d_xa, const nlinv_c64* d_xb,
                        double alpha, const double* d_p, double* d_q) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_xa, "d_xa"));
  NLV_CHECK(check_ptr(plan, d_xb, "d_xb"));
  NLV_CHECK(check_ptr(plan, d_p, "d_p"));
  NLV_CHECK(check_ptr(plan, d_q, "d_q"));
  if (!std::isfinite(alpha)) return fail(plan, NLINV_E_ARG, "alpha must be finite");
  if ((const void*)d_p == (const void*)d_q) return fail(plan, NLINV_E_ARG, "d_q must not alias d_p");
  nlv::TurnArgs turns;
  NLV_CHECK(turns_of(plan, h_turn, &turns));
  const Shape& s = plan->s;
  Bufs& w = plan->w;
  hipStream_t st = plan->stream;
  const float2* xa = reinterpret_cast<const float2*>(d_xa);
  const float2* xb = reinterpret_cast<const float2*>(d_xb);
  const double2* p = reinterpret_cast<const double2*>(d_p);
  const Partials none{};
  // coil images of the forward point (cols_fwd) and of the adjoint point (cols_back)
  NLV_CHECK(coils_into(plan, xb, w.CO));
  NLV_CHECK(coils_into(plan, xa, w.IMG));
  NLV_HIP(plan, plan->t->coil_rows_cg(s, w, st, p, nullptr, nullptr, none));
  NLV_HIP(plan, plan->t->cols_fwd(s, w, st, 1, w.CO, xb, p, w.U2));
  NLV_HIP(plan, plan->t->toep_rows(s, w, st, turns));
  NLV_HIP(plan, plan->t->cols_back(s, w, st, 0, w.U2, w.IMG, xa, nullptr));
  NLV_HIP(plan, plan->t->coilh_rows(s, w, st, 0, p, xa, nullptr, alpha, w.Q, nullptr));
  NLV_HIP(plan, nlv::launch_finalize(s, w, st, p, alpha, reinterpret_cast<double2*>(d_q)));
  return NLINV_OK;
}

int nlinv_apply_E(nlinv_plan plan, const nlinv_c64* d_xhat, const double* d_p, nlinv_c64* d_img) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_xhat, "d_xhat"));
  NLV_CHECK(check_ptr(plan, d_p, "d_p"));
  NLV_CHECK(check_ptr(plan, d_img, "d_img"));
  const Shape& s = plan->s;
  Bufs& w = plan->w;
  const float2* xh = reinterpret_cast<const float2*>(d_xhat);
  const double2* p = reinterpret_cast<const double2*>(d_p);
  const Partials none{};
  NLV_CHECK(coils_into(plan, xh, w.CO));
  NLV_HIP(plan, plan->t->coil_rows_cg(s, w, plan->stream, p, nullptr, nullptr, none));
  NLV_HIP(plan, plan->t->cols_fwd(s, w, plan->stream, 3, w.CO, xh, p, d_img));
  return NLINV_OK;
}

int nlinv_apply_EH(nlinv_plan plan, const nlinv_c64* d_xhat, const nlinv_c64* d_img, double* d_out) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_xhat, "d_xhat"));
  NLV_CHECK(check_ptr(plan, d_img, "d_img"));
  NLV_CHECK(check_ptr(plan, d_out, "d_out"));
  const Shape& s = plan->s;
  Bufs& w = plan->w;
  const float2* xh = reinterpret_cast<const float2*>(d_xhat);
  NLV_CHECK(coils_into(plan, xh, w.CO));
  NLV_HIP(plan, plan->t->cols_back(s, w, plan->stream, 2, d_img, w.CO, xh, nullptr));
  NLV_HIP(plan, plan->t->coilh_rows(s, w, plan->stream, 2, nullptr, xh, nullptr, 0.0, w.Q, nullptr));
  NLV_HIP(plan, nlv::launch_finalize(s, w, plan->stream, nullptr, 0.0, reinterpret_cast<double2*>(d_out)));
  return NLINV_OK;
}

int nlinv_nudft(nlinv_plan plan, const float* d_traj, const nlinv_c64* d_img, nlinv_c64* d_y) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_traj, "d_traj"));
  NLV_CHECK(check_ptr(plan, d_img, "d_img"));
  NLV_CHECK(check_ptr(plan, d_y, "d_y"));
  if (plan->s.R > 256) return fail(plan, NLINV_E_SIZE, "the exact forward transform supports R <= 256");
  NLV_HIP(plan, nlv::launch_nudft_fwd(plan->s, plan->stream, d_traj, reinterpret_cast<const float2*>(d_img),
                                      reinterpret_cast<float2*>(d_y)));
  return NLINV_OK;
}

int nlinv_coils(nlinv_plan plan, const nlinv_c64* d_xhat, nlinv_c64* d_coils, float* d_img) {
  NLV_CHECK(check_plan(plan));
  NLV_CHECK(check_ptr(plan, d_xhat, "d_xhat"));
  NLV_CHECK(check_ptr(plan, d_coils, "d_coils", true));
  NLV_CHECK(check_ptr(plan, d_img, "d_img", true));
  const float2* xh = reinterpret_cast<const float2*>(d_xhat);
  float2* co = d_coils ? reinterpret_cast<float2*>(d_coils) : plan->w.CO;
  NLV_CHECK(coils_into(plan, xh, co));
  if (d_img) NLV_HIP(plan, nlv::launch_image(plan->s, plan->stream, xh, co, d_img));
  return NLINV_OK;
}

int nlinv_sync(nlinv_plan plan) {
  NLV_CHECK(check_plan(plan));
  NLV_HIP(plan, hipStreamSynchronize(plan->stream));
  NLV_HIP(plan, hipGetLastError());
  if (plan->p.flags & NLINV_F_CHECK_FINITE) {
    int flag = 0;
    NLV_HIP(plan, hipMemcpyAsync(&flag, plan->flag, sizeof(int), hipMemcpyDeviceToHost, plan->stream));
    NLV_HIP(plan, hipStreamSynchronize(plan->stream));
    if (flag) {
      NLV_HIP(plan, nlv::launch_fill_int(plan->stream, plan->flag, 0));
      NLV_HIP(plan, hipStreamSynchronize(plan->stream));
      return fail(plan, NLINV_E_NONFINITE, "a reconstruction since the last nlinv_sync produced non-finite values");
    }
  }
  return NLINV_OK;
}

const char* nlinv_last_error(nlinv_plan plan) {
  return plan ? plan->err.c_str() : g_err.c_str();
}

int nlinv_set_graphs(nlinv_plan plan, int32_t enable) {
  NLV_CHECK(check_plan(plan));
  if (enable && plan->is_static)
    return fail(plan, NLINV_E_STATE, "plans on the static workspace launch eagerly (a graph would allocate)");
  plan->graphs = enable != 0;
  return NLINV_OK;
}

int nlinv_timer_enable(nlinv_plan plan, int32_t kernel_id) {
  NLV_CHECK(check_plan(plan));
  if (kernel_id != NLINV_KT_NONE && plan->is_static)
    return fail(plan, NLINV_E_STATE, "plans on the static workspace do not time kernels (events would allocate)");
  if (kernel_id < NLINV_KT_NONE || kernel_id > NLINV_KT_GRID) return fail(plan, NLINV_E_ARG, "unknown kernel id");
  plan->timer_kid = kernel_id;
  plan->ev_used = 0;
  return NLINV_OK;
}

int nlinv_timer_read(nlinv_plan plan, double* ms, int64_t* launches) {
  NLV_CHECK(check_plan(plan));
  if (!ms || !launches) return fail(plan, NLINV_E_ARG, "output pointer is NULL");
  NLV_HIP(plan, hipStreamSynchronize(plan->stream));
  double total = 0.0;
  for (size_t i = 0; i + 1 < plan->ev_used; i += 2) {
    float t = 0.f;
    NLV_HIP(plan, hipEventElapsedTime(&t, plan->ev[i], plan->ev[i + 1]));
    total += t;
  }
  *ms = total;
  *launches = (int64_t)(plan->ev_used / 2);
  plan->ev_used = 0;
  return NLINV_OK;
}

}  // extern "C"
