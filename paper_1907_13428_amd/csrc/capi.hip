// C ABI of the FDE-constrained ADMM hot path (declared in include/fde.h).
//
// Host control, device work: every step of the Krylov and ADMM iterations
// runs in the kernels of k_toeplitz.hip, k_precond.hip and k_vector.hip.
// Scalars of the iteration (alpha, beta, residual norms, the convergence
// flag) stay in device memory; the host enqueues PCG iterations in chunks
// whose kernels exit at once after the device-side convergence flag is set,
// and reads the flag back once per chunk.
#include <hip/hip_runtime.h>

#include <array>
#include <chrono>
#include <climits>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <initializer_list>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "fde_internal.hpp"
#include "host_setup.hpp"

using fde::host::cd;

namespace fde {
thread_local PassEventQueue t_pass_events;
thread_local std::vector<RecordedPass>* t_record = nullptr;
}

namespace {
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return (fde_status)fail(FDE_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// device fields are read and written in 16-byte pairs
bool misaligned(std::initializer_list<const void*> ps) {
  for (const void* p : ps)
    if (p && (reinterpret_cast<uintptr_t>(p) & 15u)) return true;
  return false;
}

#define CHECK_ALIGNED(fn, ...)                                                                \
  do {                                                                                        \
    if (misaligned({__VA_ARGS__}))                                                            \
      return (fde_status)fail(FDE_EINVAL, fn ": device fields must be 16-byte aligned");    \
  } while (0)

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

// Workspace of fde_apply_A_noalloc: a fixed device array, one copy per GPU
// that loads the library, held until the process ends; the library never
// allocates or frees it.  Host code must not pass `scratch` itself to a
// kernel (in host code the name is a stand-in, not a device address): it uses
// the per-device address obtained once with hipGetSymbolAddress.
constexpr size_t kScratchDoubles = size_t(1) << 22;  // 32 MiB per GPU
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, looked up on the first call
// made with that device current.
int scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FDE_EINVAL, "device index out of range for the static workspace");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(FDE_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return FDE_OK;
}
}  // namespace

struct fde_ctx {
  fde_problem prob{};
  fde_admm_params prm{};
  fde::host::Setup su;
  hipStream_t stream = nullptr;
  int device = 0;  // the HIP device current at fde_create
  int nx = 0, ny = 0, nt = 0, H = 0;
  int64_t N = 0;
  bool var = false, fp32 = false;

  // device tables
  double2 *lxA = nullptr, *lxB = nullptr, *lxTA = nullptr, *lxTB = nullptr;  // x: fwd (A,B), trans (A,B)
  double2 *lyA = nullptr, *lyB = nullptr, *lyTA = nullptr, *lyTB = nullptr;
  double2 *twx_emb = nullptr, *twy_emb = nullptr;
  void *twx = nullptr, *twy = nullptr, *twt = nullptr;
  double2 *tcx = nullptr, *tcy = nullptr, *tct = nullptr;
  double2 *ltA = nullptr, *ltTA = nullptr, *twt_emb = nullptr;  // fractional time: 2nt embedding
  bool frac_t = false;
  bool ycol = false;  // coefficient fields constant along y: per-column y-pass multipliers
  double *dplus = nullptr, *dminus = nullptr;
  double *invMp = nullptr, *My = nullptr, *Mu = nullptr, *Mp = nullptr, *wts = nullptr, *ones = nullptr;
  // precond_kind 2: the tables of the diagonal scaling and each slice's table
  // (allocated when that kind is first used, regrown when it needs more tables)
  double* ds_tab = nullptr;
  int* ds_class = nullptr;
  size_t ds_tab_n = 0;
  double2 *dxA = nullptr, *dxB = nullptr, *dyA = nullptr, *dyB = nullptr;  // dL/dalpha, dL/dbeta

  // workspace fields
  double *fa = nullptr, *fw = nullptr, *fb = nullptr;  // line-pass intermediates
  double *q = nullptr, *r = nullptr, *z = nullptr, *pk = nullptr, *bvec = nullptr;
  double *ar = nullptr, *Ru = nullptr, *av = nullptr, *ac = nullptr, *By = nullptr;
  void* spec = nullptr;
  double *part_pq = nullptr, *part_rr = nullptr, *part_rz = nullptr, *part_max = nullptr, *part_dots = nullptr;
  // adjoint time stepping: the 1-point "time" tables of a single-slice problem
  double2* adj_lt = nullptr;
  void* adj_twt = nullptr;
  int maxpart = 0;
  double* scal = nullptr;
  int* ints = nullptr;
  double* h_scal = nullptr;  // pinned
  int* h_ints = nullptr;
  hipEvent_t ev = nullptr;   // marks completion of the last posted readback
  // phase boundaries of an ADMM iteration (timing events): RHS start, Krylov
  // start, Krylov end, update end
  hipEvent_t ph_ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<void*> allocs;

  // one PCG iteration captured as a HIP graph (re-captured when the
  // solution pointer changes); launched on `stream`
  hipStream_t cap_stream = nullptr;
  // PCG iterations captured once: [0] one iteration, [1] kGraphIters in a row
  hipGraph_t pcg_graph[2] = {nullptr, nullptr};
  hipGraphExec_t pcg_exec[2] = {nullptr, nullptr};
  const double* pcg_graph_x = nullptr;
  bool use_graph = true;
  // in-solve pass timing (fde_pass_timing): plain PCG launches with a pair of
  // events bound to each of the nine passes, harvested after every readback
  bool ptime = false;
  std::vector<hipEvent_t> pt_ev;  // pool of event pairs
  int pt_used = 0;                // pairs enqueued since the last harvest
  double pt_us[fde::kNumPasses] = {};
  int64_t pt_n[fde::kNumPasses] = {};
  // column-tile variants (0 widest, 1 half, 2 quarter) chosen by fde_autotune
  int tile_line_y = 0, tile_pre_y = 0, tile_pre_t = 0;
  int conv_sep = -1;  // PCG convergence test: -1 by grid size, 0 fused in the y-forward pass, 1 on its own
  // per-point box bounds set by fde_set_bounds (context copies; null: the scalar bound)
  double *bya = nullptr, *byb = nullptr, *bua = nullptr, *bub = nullptr;
  double *bya_mem = nullptr, *byb_mem = nullptr, *bua_mem = nullptr, *bub_mem = nullptr;

  // MINRES workspace (allocated on first use): Lanczos vectors, preconditioned
  // vectors and directions, two of each, K z, a scratch field, the p block of
  // the ADMM right-hand side, five partial-sum arrays and the device scalars
  bool mr_ready = false;
  fde::Triple mrV[2]{}, mrZ[2]{}, mrW[2]{}, mrQ{};
  double *mr_tmp = nullptr, *mr_rhs = nullptr, *mr_part[5] = {}, *ms = nullptr, *h_ms = nullptr;

  template <typename T>
  hipError_t alloc(T** p, size_t count) {
    void* v = nullptr;
    hipError_t e = hipMalloc(&v, count * sizeof(T));
    if (e == hipSuccess) {
      allocs.push_back(v);
      *p = static_cast<T*>(v);
    }
    return e;
  }
};

namespace {

template <typename T>
hipError_t upload(fde_ctx* c, T** dst, const std::vector<T>& src) {
  hipError_t e = c->alloc(dst, src.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

hipError_t upload_c(fde_ctx* c, double2** dst, const std::vector<cd>& src) {
  std::vector<double2> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = double2{src[i].real(), src[i].imag()};
  return upload(c, dst, tmp);
}

hipError_t upload_tw(fde_ctx* c, void** dst, const std::vector<cd>& src, bool fp32) {
  if (fp32) {
    std::vector<float2> tmp(src.size());
    for (size_t i = 0; i < src.size(); ++i) tmp[i] = float2{(float)src[i].real(), (float)src[i].imag()};
    float2* d = nullptr;
    hipError_t e = upload(c, &d, tmp);
    *dst = d;
    return e;
  }
  double2* d = nullptr;
  hipError_t e = upload_c(c, &d, src);
  *dst = d;
  return e;
}

// maximum number of blocks any reducing launch uses (partial-sum capacity)
int max_partials(int nx, int ny, int nt, bool frac_t) {
  const long long N = (long long)nx * ny * nt;
  long long m = 2048;  // vector kernels
  // t-pass: tiles of at least 2 columns of the nx*ny plane
  if (frac_t) m = std::max(m, ((long long)nx * ny + 1) / 2);
  // y-pass: tiles * nt with at least 2 columns per tile
  m = std::max(m, (long long)((nx + 1) / 2) * nt);
  // x-inverse of the preconditioner: pairs of lines, at least one pair per block
  m = std::max(m, (long long)(ny * nt + 1) / 2);
  (void)N;
  return (int)m;
}

fde::LinePassArgs line_args(fde_ctx* c) {
  fde::LinePassArgs a{};
  a.nx = c->nx;
  a.ny = c->ny;
  a.nt = c->nt;
  a.dplus = c->dplus;
  a.dminus = c->dminus;
  return a;
}

// x-pass: out = s_time * (E or E^T) in + s_sp * L_x(^T) in
hipError_t xpass(fde_ctx* c, const double* in, double* out, bool tr, double s_time, double s_sp,
                 const int* done) {
  fde::LinePassArgs a = line_args(c);
  a.in = in;
  a.out = out;
  a.L = c->su.x.L;
  a.tw = c->twx_emb;
  if (c->var) {
    a.lamA = tr ? c->lxTA : c->lxA;
    a.lamB = tr ? c->lxTB : c->lxB;
  } else {
    a.lamA = tr ? c->lxTA : c->lxA;
  }
  a.s_time = s_time;
  a.s_sp = s_sp;
  a.done = done;
  return fde::launch_xpass(a, tr, c->var, c->stream, nullptr);
}

// y-pass: out_t = osc[t] (acc + s_sp L_y(^T) in) + esc[t] extra
hipError_t ypass(fde_ctx* c, const double* in, const double* acc, double* out, bool tr, double s_sp,
                 const double* osc, const double* extra, const double* esc, const double* dotv,
                 double* partial, const int* done, int* nb) {
  fde::LinePassArgs a = line_args(c);
  a.in = in;
  a.out = out;
  a.L = c->su.y.L;
  a.tw = c->twy_emb;
  a.lamA = tr ? c->lyTA : c->lyA;
  a.lamB = tr ? c->lyTB : c->lyB;
  a.s_sp = s_sp;
  a.tile = c->tile_line_y;
  a.col_coef = c->ycol ? 1 : 0;
  a.acc = acc;
  a.oscale = osc;
  a.extra = extra;
  a.escale = esc;
  a.dotv = dotv;
  a.partial = partial;
  a.done = done;
  return fde::launch_ypass(a, tr, c->var, c->stream, nb);
}

// t-pass of a fractional time order: out_t = osc[t] (acc + s C_t(^T) in) + esc[t] extra, the
// t-lines of the field viewed as [nt][nx*ny] run through the y-pass kernel (rows = time levels)
hipError_t tpass(fde_ctx* c, const double* in, const double* acc, double* out, bool tr, double s,
                 const double* osc, const double* extra, const double* esc, const double* dotv,
                 double* partial, const int* done, int* nb) {
  fde::LinePassArgs a{};
  a.nx = c->nx * c->ny;
  a.ny = c->nt;
  a.nt = 1;
  a.L = c->su.Lt;
  a.in = in;
  a.out = out;
  a.acc = acc;
  a.tw = c->twt_emb;
  a.lamA = tr ? c->ltTA : c->ltA;
  a.s_sp = s;
  a.tile = 0;
  a.row_scale = 1;
  a.oscale = osc;
  a.extra = extra;
  a.escale = esc;
  a.dotv = dotv;
  a.partial = partial;
  a.done = done;
  return fde::launch_ypass(a, tr, false, c->stream, nb);
}

// out = osc[t] (scale D(^T) in) + esc[t] extra, with optional partial sums of (dotv, out);
// tmp1 and tmp2 are workspace fields distinct from in and out.  Implicit Euler: the time
// difference rides in the x-pass and the epilogue in the y-pass; a fractional time order
// adds the t-pass, which then carries the epilogue.
hipError_t apply_op(fde_ctx* c, const double* in, double* out, bool tr, double scale, double* tmp1, double* tmp2,
                    const double* osc, const double* extra, const double* esc, const double* dotv, double* partial,
                    const int* done, int* nb) {
  hipError_t e;
  if (!c->frac_t) {
    if ((e = xpass(c, in, tmp1, tr, scale / c->su.ht, -scale, done)) != hipSuccess) return e;
    return ypass(c, in, tmp1, out, tr, -scale, osc, extra, esc, dotv, partial, done, nb);
  }
  if ((e = xpass(c, in, tmp1, tr, 0.0, -scale, done)) != hipSuccess) return e;
  if ((e = ypass(c, in, tmp1, tmp2, tr, -scale, nullptr, nullptr, nullptr, nullptr, nullptr, done, nullptr)) !=
      hipSuccess)
    return e;
  return tpass(c, in, tmp2, out, tr, scale, osc, extra, esc, dotv, partial, done, nb);
}

// y = S x = M_y x + B^T M_p^{-1} B x, optional partial sums of (x, y)
hipError_t apply_S(fde_ctx* c, const double* x, double* y, double* partial, const int* done, int* nb) {
  const double psi = c->su.psi;
  hipError_t e;
  if ((e = apply_op(c, x, c->fw, false, psi, c->fa, c->fb, c->invMp, nullptr, nullptr, nullptr, nullptr, done,
                    nullptr)) != hipSuccess)
    return e;
  return apply_op(c, c->fw, y, true, psi, c->fa, c->fb, nullptr, x, c->My, partial ? x : nullptr, partial, done, nb);
}

fde::PrecondArgs pre_args(fde_ctx* c, double* r, double* z) {
  fde::PrecondArgs a{};
  a.nx = c->nx;
  a.ny = c->ny;
  a.nt = c->nt;
  a.H = c->H;
  a.r = r;
  a.z = z;
  a.spec = c->spec;
  a.twx = c->twx;
  a.twy = c->twy;
  a.twt = c->twt;
  a.lam_x = c->tcx;
  a.lam_y = c->tcy;
  a.lam_t = c->tct;
  a.psi = c->su.psi;
  a.a = c->su.a;
  a.inv_mbar = c->su.inv_mbar;
  a.match2 = c->su.match2;
  a.inv_n = 1.0 / (double)c->N;
  a.scal = c->scal;
  a.tile_y = c->tile_pre_y;
  a.tile_t = c->tile_pre_t;
  if (c->prm.precond_kind == 2) {
    a.ds_tab = c->ds_tab;
    a.ds_class = c->ds_class;
  }
  return a;
}

fde_status check_ctx(fde_ctx* c) {
  if (!c) return (fde_status)fail(FDE_EINVAL, "context is NULL");
  return FDE_OK;
}

// Device scalars -> pinned host copies, then an event; the host learns the
// outcome of enqueued work without blocking the stream.
fde_status post_readback(fde_ctx* c) {
  HIP_TRY(hipMemcpyAsync(c->h_scal, c->scal, sizeof(double) * fde::kNumScalars, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(c->h_ints, c->ints, sizeof(int) * fde::kNumInts, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipEventRecord(c->ev, c->stream));
  return FDE_OK;
}

fde_status wait_readback(fde_ctx* c) {
  HIP_TRY(hipEventSynchronize(c->ev));
  return FDE_OK;
}

// 1: ready, 0: pending, <0: error
int readback_ready(fde_ctx* c) {
  const hipError_t e = hipEventQuery(c->ev);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  return fail(FDE_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(e));
}

fde_status sync_scalars(fde_ctx* c) {
  fde_status st = post_readback(c);
  if (st != FDE_OK) return st;
  return wait_readback(c);
}

// One PCG iteration (10 launches): q = S p with (p, q) partials ; alpha inside
// the next pass, which also does x += alpha p, r -= alpha q and (r, r) ; the
// convergence test inside the following pass ; z = S~^{-1} r with (r, z)
// partials ; beta inside p = z + beta p.
// Every kernel returns at once when the device flag says the solve is done.
hipError_t enqueue_pcg_iteration_passes(fde_ctx* c, double* x);

// With pass timing on, the nine pass launches of the iteration take the next
// nine event pairs of the context's pool (grown on demand).
hipError_t enqueue_pcg_iteration(fde_ctx* c, double* x) {
  using namespace fde;
  if (!c->ptime) return enqueue_pcg_iteration_passes(c, x);
  const size_t need = 2 * (size_t)(c->pt_used + kNumPasses);
  while (c->pt_ev.size() < need) {
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    c->pt_ev.push_back(ev);
  }
  t_pass_events = PassEventQueue{c->pt_ev.data() + 2 * (size_t)c->pt_used, kNumPasses, 0};
  const hipError_t e = enqueue_pcg_iteration_passes(c, x);
  const int taken = t_pass_events.next;
  t_pass_events = PassEventQueue{};
  if (e != hipSuccess) return e;
  if (taken != kNumPasses) return hipErrorUnknown;  // the pass list changed
  c->pt_used += kNumPasses;
  return hipSuccess;
}

// Kernel durations of the pass launches enqueued since the last harvest (all
// complete: called after a readback of the stream)
hipError_t harvest_pass_times(fde_ctx* c) {
  for (int k = 0; k < c->pt_used; ++k) {
    float ms = 0;
    const hipError_t e = hipEventElapsedTime(&ms, c->pt_ev[2 * (size_t)k], c->pt_ev[2 * (size_t)k + 1]);
    if (e != hipSuccess) return e;
    c->pt_us[k % fde::kNumPasses] += 1000.0 * ms;
    c->pt_n[k % fde::kNumPasses] += 1;
  }
  c->pt_used = 0;
  return hipSuccess;
}

hipError_t enqueue_pcg_iteration_passes(fde_ctx* c, double* x) {
  using namespace fde;
  const int* done = c->ints + kDone;
  int nbS = 0, nb1 = 0, nb5 = 0;
  hipError_t e;
  if ((e = apply_S(c, c->pk, c->q, c->part_pq, done, &nbS)) != hipSuccess) return e;
  // the preconditioner's output is the next direction p = S~^{-1} r + beta p,
  // with (r, z) and beta from the spectrum
  PrecondArgs a = pre_args(c, c->r, c->pk);
  a.q = c->q;
  a.xvec = x;
  a.pvec = c->pk;
  a.partial = c->part_rr;
  a.rzs_partial = c->part_rz;
  a.pdir = 1;
  a.done = done;
  a.pq_partial = c->part_pq;  // alpha computed inside the x-forward pass
  a.pq_n = nbS;
  a.scal_w = c->scal;
  a.ints = c->ints;
  if ((e = launch_precond_stage(a, c->fp32, 1, c->stream, &nb1, &nb5)) != hipSuccess) return e;
  // The convergence test runs inside the y-forward pass, every block summing
  // the (r, r) partials; when those redundant sums would read more than a
  // small launch costs (about 2^21 partial reads, large grids), one block does
  // the test on its own between the passes.
  const bool big = (size_t)nb1 * (size_t)c->H * (size_t)c->nt > ((size_t)1 << 25);
  if (c->conv_sep == 1 || (c->conv_sep < 0 && big)) {
    if ((e = launch_pcg_scalar(FIN_CONV, c->part_rr, nb1, c->scal, c->ints, c->stream)) != hipSuccess) return e;
  } else {
    a.rr_partial = c->part_rr;
    a.rr_n = nb1;
  }
  return launch_precond_stage(a, c->fp32, 2, c->stream, &nb1, &nb5);
}

// Iterations per launch of the larger PCG graph.  Consecutive graph launches
// on a stream are separated by a few microseconds of idle GPU (none between
// the kernels inside a graph), so chunks of iterations are enqueued mostly
// as launches of kGraphIters iterations.
constexpr int kGraphIters = 4;

void drop_pcg_graph(fde_ctx* c) {
  for (int k = 0; k < 2; ++k) {
    if (c->pcg_exec[k]) (void)hipGraphExecDestroy(c->pcg_exec[k]);
    if (c->pcg_graph[k]) (void)hipGraphDestroy(c->pcg_graph[k]);
    c->pcg_exec[k] = nullptr;
    c->pcg_graph[k] = nullptr;
  }
  c->pcg_graph_x = nullptr;
}

// capture iters PCG iterations in a row on the private capture stream
fde_status capture_pcg_iterations(fde_ctx* c, double* x, int iters, hipGraph_t* gout, hipGraphExec_t* xout) {
  hipStream_t user = c->stream;
  c->stream = c->cap_stream;
  HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int k = 0; k < iters && e == hipSuccess; ++k) e = enqueue_pcg_iteration(c, x);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
  c->stream = user;
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return (fde_status)fail(FDE_EHIP, std::string("PCG graph capture: ") +
                                          hipGetErrorString(e != hipSuccess ? e : e2));
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e3 != hipSuccess) {
    (void)hipGraphDestroy(g);
    return (fde_status)fail(FDE_EHIP, std::string("PCG graph instantiate: ") + hipGetErrorString(e3));
  }
  *gout = g;
  *xout = ex;
  return FDE_OK;
}

fde_status ensure_pcg_graph(fde_ctx* c, double* x) {
  if (c->pcg_exec[0] && c->pcg_exec[1] && c->pcg_graph_x == x) return FDE_OK;
  drop_pcg_graph(c);
  if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  const int iters[2] = {1, kGraphIters};
  for (int k = 0; k < 2; ++k) {
    const fde_status st = capture_pcg_iterations(c, x, iters[k], &c->pcg_graph[k], &c->pcg_exec[k]);
    if (st != FDE_OK) {
      drop_pcg_graph(c);
      return st;
    }
  }
  c->pcg_graph_x = x;
  return FDE_OK;
}

// enqueue n PCG iterations (graph launches of kGraphIters and of one)
hipError_t launch_pcg_iterations(fde_ctx* c, double* x, int n) {
  hipError_t e = hipSuccess;
  if (!c->use_graph || c->ptime) {
    for (int k = 0; k < n && e == hipSuccess; ++k) e = enqueue_pcg_iteration(c, x);
    return e;
  }
  for (; n >= kGraphIters && e == hipSuccess; n -= kGraphIters) e = hipGraphLaunch(c->pcg_exec[1], c->stream);
  for (; n > 0 && e == hipSuccess; --n) e = hipGraphLaunch(c->pcg_exec[0], c->stream);
  return e;
}

// PCG on S x = b (x: initial guess in, solution out), in two phases so that
// several contexts can be driven from one host thread:
//   krylov_begin     enqueue r = b - S x, the convergence test, z = S~^{-1} r,
//                    p = z and a first chunk of iterations; post a readback
//   krylov_continue  after the readback: finished, or enqueue two more
//                    iterations and post another readback
struct KrylovRun {
  double* x = nullptr;
  int maxit = 0;
  int enqueued = 0;
  int iters = 0;
  double relres = 0;
  fde_status status = FDE_OK;
  bool defer = false;  // batched solves: the set-up only; the iterations come from the batch
};

// How krylov_begin forms S x for the initial residual: a full apply (SX_APPLY);
// x known to be zero (SX_ZERO: S x = 0); or M_p^{-1} B x already in c->fw from the
// previous ADMM step's recovery pass (SX_BYP: S x = B^T fw + M_y x, half the passes).
enum SxMode { SX_APPLY = 0, SX_ZERO, SX_BYP };

fde_status krylov_begin(fde_ctx* c, const double* b, double* x, double tol, int maxit, int predict, KrylovRun* kr,
                        int sx = SX_APPLY) {
  using namespace fde;
  const int* done = c->ints + kDone;
  const double tol2 = tol * tol;
  int nbv = 0, nb1 = 0, nb5 = 0;
  kr->x = x;
  kr->maxit = maxit;
  kr->enqueued = 0;
  // r = b - S x ; (r, r), (b, b) ; tolerance and iteration limit into the device slots
  if (sx == SX_ZERO) {
    HIP_TRY(launch_lincomb(c->N, 0.0, nullptr, 0.0, nullptr, 0.0, nullptr, c->q, c->stream));
  } else if (sx == SX_BYP) {
    HIP_TRY(apply_op(c, c->fw, c->q, true, c->su.psi, c->fa, c->fb, nullptr, x, c->My, nullptr, nullptr, nullptr,
                     nullptr));
  } else {
    HIP_TRY(apply_S(c, x, c->q, nullptr, nullptr, nullptr));
  }
  HIP_TRY(launch_axpy_dot(VEC_RESID, c->N, b, c->q, c->r, c->scal, c->part_pq, nullptr, c->stream, &nbv));
  HIP_TRY(launch_pcg_scalar(FIN_INIT, c->part_pq, nbv, c->scal, c->ints, c->stream, tol2, maxit));
  HIP_TRY(launch_axpy_dot(VEC_ZERO_IF_BB0, c->N, nullptr, nullptr, x, c->scal, nullptr, nullptr, c->stream,
                          nullptr));
  // p = z = S~^{-1} r ; rz = (r, z) from the spectrum
  PrecondArgs a = pre_args(c, c->r, c->pk);
  a.rzs_partial = c->part_rz;
  a.pdir = 2;
  a.done = done;
  a.scal_w = c->scal;
  a.ints = c->ints;
  HIP_TRY(launch_precond(a, c->fp32, c->stream, &nb1, &nb5));
  if (kr->defer) return FDE_OK;
  if (c->use_graph && !c->ptime) {
    const fde_status st = ensure_pcg_graph(c, x);
    if (st != FDE_OK) return st;
  }
  const int chunk = std::min(predict > 1 ? predict : 2, maxit);
  HIP_TRY(launch_pcg_iterations(c, x, chunk));
  kr->enqueued = chunk;
  return post_readback(c);
}

// returns 1 when finished (kr->status, iters, relres set), 0 when more work was enqueued
int krylov_continue(fde_ctx* c, KrylovRun* kr) {
  using namespace fde;
  if (c->ptime) {
    const hipError_t he = harvest_pass_times(c);
    if (he != hipSuccess) {
      kr->status = (fde_status)fail(FDE_EHIP, std::string("pass timing: ") + hipGetErrorString(he));
      return 1;
    }
  }
  if (!(c->h_ints[kDone] || kr->enqueued >= kr->maxit)) {
    const int more = std::min(2, kr->maxit - kr->enqueued);
    const hipError_t e = launch_pcg_iterations(c, kr->x, more);
    kr->enqueued += more;
    if (e != hipSuccess) {
      kr->status = (fde_status)fail(FDE_EHIP, std::string("PCG launch: ") + hipGetErrorString(e));
      return 1;
    }
    const fde_status st = post_readback(c);
    if (st != FDE_OK) {
      kr->status = st;
      return 1;
    }
    return 0;
  }
  kr->iters = c->h_ints[kIter];
  const double bb = c->h_scal[kBB];
  kr->relres = bb > 0 ? std::sqrt(c->h_scal[kRR] / bb) : 0.0;
  if (c->h_ints[kConv] < 0) kr->status = (fde_status)fail(FDE_ENONFINITE, "non-finite residual in PCG");
  else if (c->h_ints[kConv] == 0) kr->status = FDE_ENOTCONV;
  else kr->status = FDE_OK;
  return 1;
}

fde_status krylov(fde_ctx* c, const double* b, double* x, double tol, int maxit, int* iters, double* relres,
                  int predict) {
  KrylovRun kr;
  fde_status st = krylov_begin(c, b, x, tol, maxit, predict, &kr);
  if (st != FDE_OK) return st;
  while (true) {
    if ((st = wait_readback(c)) != FDE_OK) return st;
    if (krylov_continue(c, &kr)) break;
  }
  *iters = kr.iters;
  *relres = kr.relres;
  return kr.status;
}

// ---------------------------------------------------------------------------
// MINRES on the merged x-step system (3.8) with K~ of eq. (3.12) (kernels in
// k_minres.hip).  Same two-phase driving as PCG: minres_begin enqueues the
// set-up and a first chunk of iterations, minres_continue consumes a readback.
// The vectors rotate between two buffers each (parity bit), so the launches of
// an iteration depend on its parity; they are not captured in a graph.
// ---------------------------------------------------------------------------
fde_status ensure_minres(fde_ctx* c) {
  if (c->mr_ready) return FDE_OK;
  const size_t n = (size_t)c->N;
  auto tri = [&](fde::Triple* t) -> hipError_t {
    hipError_t e = c->alloc(&t->y, n);
    if (e == hipSuccess) e = c->alloc(&t->u, n);
    if (e == hipSuccess) e = c->alloc(&t->p, n);
    return e;
  };
  for (int i = 0; i < 2; ++i) {
    HIP_TRY(tri(&c->mrV[i]));
    HIP_TRY(tri(&c->mrZ[i]));
    HIP_TRY(tri(&c->mrW[i]));
  }
  HIP_TRY(tri(&c->mrQ));
  HIP_TRY(c->alloc(&c->mr_tmp, n));
  HIP_TRY(c->alloc(&c->mr_rhs, n));
  for (auto& p : c->mr_part) HIP_TRY(c->alloc(&p, (size_t)c->maxpart));
  HIP_TRY(c->alloc(&c->ms, (size_t)fde::kNumMinres));
  HIP_TRY(hipHostMalloc((void**)&c->h_ms, sizeof(double) * fde::kNumMinres, hipHostMallocDefault));
  c->mr_ready = true;
  return FDE_OK;
}

fde::MinresConsts minres_consts(fde_ctx* c) {
  fde::MinresConsts k{};
  k.n = c->N;
  k.plane = c->nx * c->ny;
  k.k_u = c->su.k_u;
  k.dr = c->prm.delta / c->prm.rho;
  k.My = c->My;
  k.Mu = c->Mu;
  return k;
}

// q = K z with partial sums (z.u, q.u), (z.p, q.p), (z.y, q.y) in mr_part[0..2]
hipError_t minres_apply_K(fde_ctx* c, fde::Triple z, fde::Triple q, const int* stop, int* nb) {
  const double psi = c->su.psi;
  hipError_t e;
  if ((e = fde::launch_minres_pre(minres_consts(c), z, c->mr_tmp, q.u, c->mr_part[0], c->ints, c->stream, &nb[0])) !=
      hipSuccess)
    return e;
  // q.p = B z.y + (k_u z.u - (delta/rho) z.p)
  if ((e = apply_op(c, z.y, q.p, false, psi, c->fa, c->fb, nullptr, c->mr_tmp, c->ones, z.p, c->mr_part[1], stop,
                    &nb[1])) != hipSuccess)
    return e;
  // q.y = B^T z.p + M_y z.y
  return apply_op(c, z.p, q.y, true, psi, c->fa, c->fb, nullptr, z.y, c->My, z.y, c->mr_part[2], stop, &nb[2]);
}

// z = (a / mbar) S~^{-1} r (the third block of K~^{-1}) with (r, z) partials
hipError_t minres_precond(fde_ctx* c, double* r, double* z, double* partial, const int* done, int* nb) {
  fde::PrecondArgs a = pre_args(c, r, z);
  a.inv_n *= c->su.a * c->su.inv_mbar;
  a.partial2 = partial;
  a.done = done;
  int nb1 = 0;
  return fde::launch_precond(a, c->fp32, c->stream, &nb1, nb);
}

struct MinresRun {
  fde::Triple x{};
  int maxit = 0;
  int enqueued = 0;
  int parity = 0;
  int iters = 0;
  double relres = 0;
  fde_status status = FDE_OK;
};

hipError_t enqueue_minres_iteration(fde_ctx* c, MinresRun* m) {
  using namespace fde;
  const int P = m->parity, O = 1 - P;
  const int* stop = c->ints + kStop;
  const MinresConsts k = minres_consts(c);
  int nb[5] = {0, 0, 0, 0, 0};
  hipError_t e;
  if ((e = minres_apply_K(c, c->mrZ[P], c->mrQ, stop, nb)) != hipSuccess) return e;
  if ((e = launch_minres_scalar(MR_DELTA, c->mr_part[0], nb[0], c->mr_part[1], nb[1], c->mr_part[2], nb[2], c->ms,
                                c->ints, 0.0, 0, c->stream)) != hipSuccess)
    return e;
  // v~_{j+1} over v~_{j-1}; z~_{j+1} = K~^{-1} v~_{j+1}
  if ((e = launch_minres_vec(MR_LANCZOS, k, c->mrQ, c->mrV[P], c->mrV[O], c->mrZ[O], c->ms, c->mr_part[3], stop,
                             c->stream, &nb[3])) != hipSuccess)
    return e;
  if ((e = minres_precond(c, c->mrV[O].p, c->mrZ[O].p, c->mr_part[4], stop, &nb[4])) != hipSuccess) return e;
  if ((e = launch_minres_scalar(MR_GIVENS, c->mr_part[3], nb[3], c->mr_part[4], nb[4], nullptr, 0, c->ms, c->ints,
                                0.0, 0, c->stream)) != hipSuccess)
    return e;
  // w_{j+1} over w_{j-1}; x += c_{j+1} eta_j w_{j+1} (runs in the iteration that raises the stop request)
  if ((e = launch_minres_update(k, c->mrZ[P], c->mrW[P], c->mrW[O], m->x, c->ms, c->ints + kDone, c->stream)) !=
      hipSuccess)
    return e;
  m->parity = O;
  return hipSuccess;
}

fde_status minres_post(fde_ctx* c) {
  HIP_TRY(hipMemcpyAsync(c->h_ms, c->ms, sizeof(double) * fde::kNumMinres, hipMemcpyDeviceToHost, c->stream));
  return post_readback(c);
}

fde_status minres_begin(fde_ctx* c, fde::Triple b, fde::Triple x, double tol, int maxit, bool cold, int predict,
                        MinresRun* m) {
  using namespace fde;
  fde_status st = ensure_minres(c);
  if (st != FDE_OK) return st;
  const MinresConsts k = minres_consts(c);
  *m = MinresRun{};
  m->x = x;
  m->maxit = maxit;
  int nb[5] = {0, 0, 0, 0, 0};
  // |b| in the K~^{-1} norm; also clears the stop/done flags
  HIP_TRY(launch_minres_vec(MR_RHS, k, Triple{}, b, Triple{}, c->mrZ[0], nullptr, c->mr_part[3], nullptr, c->stream,
                            &nb[3]));
  HIP_TRY(minres_precond(c, b.p, c->mrZ[0].p, c->mr_part[4], nullptr, &nb[4]));
  HIP_TRY(launch_minres_scalar(MR_NB, c->mr_part[3], nb[3], c->mr_part[4], nb[4], nullptr, 0, c->ms, c->ints, tol,
                               maxit, c->stream));
  if (cold)
    HIP_TRY(launch_minres_vec(MR_ZERO, k, Triple{}, Triple{}, x, Triple{}, nullptr, nullptr, nullptr, c->stream,
                              nullptr));
  // v~_1 = b - K x, z~_1 = K~^{-1} v~_1, gamma_1
  HIP_TRY(minres_apply_K(c, x, c->mrQ, nullptr, nb));
  HIP_TRY(launch_minres_vec(MR_RESID, k, c->mrQ, b, c->mrV[0], c->mrZ[0], nullptr, c->mr_part[3], nullptr,
                            c->stream, &nb[3]));
  HIP_TRY(minres_precond(c, c->mrV[0].p, c->mrZ[0].p, c->mr_part[4], nullptr, &nb[4]));
  HIP_TRY(launch_minres_scalar(MR_INIT, c->mr_part[3], nb[3], c->mr_part[4], nb[4], nullptr, 0, c->ms, c->ints, tol,
                               maxit, c->stream));
  for (Triple* t : {&c->mrV[1], &c->mrW[0], &c->mrW[1]})
    HIP_TRY(launch_minres_vec(MR_ZERO, k, Triple{}, Triple{}, *t, Triple{}, nullptr, nullptr, nullptr, c->stream,
                              nullptr));
  // b = 0: the solution is x = 0
  HIP_TRY(launch_minres_vec(MR_ZERO, k, Triple{}, Triple{}, x, Triple{}, c->ms, nullptr, nullptr, c->stream, nullptr));
  const int chunk = predict > 1 ? predict : 2;
  for (int i = 0; i < chunk && m->enqueued < maxit; ++i, ++m->enqueued) HIP_TRY(enqueue_minres_iteration(c, m));
  return minres_post(c);
}

// returns 1 when finished (m->status, iters, relres set), 0 when more work was enqueued
int minres_continue(fde_ctx* c, MinresRun* m) {
  using namespace fde;
  if (!(c->h_ints[kStop] || m->enqueued >= m->maxit)) {
    for (int i = 0; i < 2 && m->enqueued < m->maxit; ++i, ++m->enqueued) {
      const hipError_t e = enqueue_minres_iteration(c, m);
      if (e != hipSuccess) {
        m->status = (fde_status)fail(FDE_EHIP, std::string("MINRES launch: ") + hipGetErrorString(e));
        return 1;
      }
    }
    const fde_status st = minres_post(c);
    if (st != FDE_OK) {
      m->status = st;
      return 1;
    }
    return 0;
  }
  m->iters = c->h_ints[kIter];
  const double nb = c->h_ms[kMNb];
  m->relres = nb > 0 ? c->h_ms[kMRes] / nb : 0.0;
  if (c->h_ints[kConv] < 0) m->status = (fde_status)fail(FDE_ENONFINITE, "non-finite value or breakdown in MINRES");
  else if (c->h_ints[kConv] == 0) m->status = FDE_ENOTCONV;
  else m->status = FDE_OK;
  return 1;
}

// ---------------------------------------------------------------------------
// Algorithm 1 as a resumable state machine.  admm_begin enqueues the first
// iteration; each admm_advance call (made once the posted readback is
// complete) consumes it and enqueues the next phase:
//   PH_PCG  Krylov chunks of the x-step
//   PH_RES  recovery, projection, dual update, residual maxima
//   PH_OBJ  objective of the final iterate
// ---------------------------------------------------------------------------
enum AdmmPhase { PH_PCG = 0, PH_RES, PH_OBJ, PH_DONE };

struct AdmmRun {
  fde::AdmmConsts k{};
  fde::AdmmFields f{};
  int j = 0;
  int phase = PH_DONE;
  int predict = 0;
  bool have_byp = false;  // c->fw holds M_p^{-1} B y for the current y
  bool have_rhs = false;  // the update pass already wrote this iteration's Ru, r, v, c
  bool batched = false;   // lockstep batch: Krylov iterations come from batched launches
  double prev_min = 0.0;
  double t0 = 0, tp = 0, t_pcg = 0;
  KrylovRun kr;
  MinresRun mr;
  fde_admm_stats st{};
  fde_status status = FDE_ENOTCONV;
};

fde_status admm_enqueue_iteration(fde_ctx* c, AdmmRun* R) {
  const auto& s = c->su;
  const fde_admm_params& q = c->prm;
  const double psi = s.psi;
  HIP_TRY(hipEventRecord(c->ph_ev[0], c->stream));
  // 1. b = B^T((1-rho) p - M_p^{-1} r) + rho(J1 yhat - e_y wy + e_y^2 zy/delta)
  if (!R->have_rhs) HIP_TRY(fde::launch_admm_rhs(R->k, R->f, psi, c->stream));
  R->have_rhs = false;
  if (q.krylov_solver == 1) {
    // MINRES on the merged system (3.8): right-hand side (R_y, R_u, psi g - (delta/rho) p),
    // R_y = c + (1 - rho) B^T p; warm start from the previous (y, u, p).  The workspace
    // (mr_rhs among it) exists before the first launch that writes it.
    const fde_status ws = ensure_minres(c);
    if (ws != FDE_OK) return ws;
    HIP_TRY(apply_op(c, R->f.p, c->bvec, true, (1.0 - q.rho) * psi, c->fb, c->fa, nullptr, c->ac, c->ones, nullptr,
                     nullptr, nullptr, nullptr));
    HIP_TRY(fde::launch_lincomb(c->N, -q.delta / q.rho, R->f.p, psi, R->f.g, 0.0, nullptr, c->mr_rhs, c->stream));
    const double tol = q.tol_mode == 1 ? 0.05 * std::fmax(R->prev_min, 1e-4) : q.krylov_tol;
    R->tp = now();
    R->phase = PH_PCG;
    HIP_TRY(hipEventRecord(c->ph_ev[1], c->stream));
    return minres_begin(c, fde::Triple{c->bvec, R->f.Ru, c->mr_rhs}, fde::Triple{R->f.y, R->f.u, R->f.p}, tol,
                        q.krylov_maxit, q.pcg_cold_start != 0, R->predict, &R->mr);
  }
  HIP_TRY(apply_op(c, c->av, c->bvec, true, psi, c->fb, c->fa, nullptr, c->ac, c->ones, nullptr, nullptr, nullptr,
                   nullptr));
  // 2. S y = b by PCG, warm-started from the previous y (or from zero); the initial
  //    residual reuses M_p^{-1} B y from the previous recovery pass when y is unchanged
  if (q.pcg_cold_start) HIP_TRY(fde::launch_lincomb(c->N, 0.0, nullptr, 0.0, nullptr, 0.0, nullptr, R->f.y, c->stream));
  const double tol = q.tol_mode == 1 ? 0.05 * std::fmax(R->prev_min, 1e-4) : q.krylov_tol;
  const int sx = q.pcg_cold_start ? SX_ZERO : (R->have_byp ? SX_BYP : SX_APPLY);
  R->have_byp = false;
  R->tp = now();
  R->phase = PH_PCG;
  HIP_TRY(hipEventRecord(c->ph_ev[1], c->stream));
  R->kr.defer = R->batched;
  return krylov_begin(c, c->bvec, R->f.y, tol, q.krylov_maxit, R->predict, &R->kr, sx);
}

fde_status admm_begin(fde_ctx* c, AdmmRun* R, const double* yhat, const double* g, double* y, double* u, double* zy,
                      double* zu, double* p, double* wy, double* wu, bool batched = false) {
  CHECK_ALIGNED("fde_admm_solve", yhat, g, y, u, zy, zu, p, wy, wu);
  const auto& s = c->su;
  const fde_admm_params& q = c->prm;
  *R = AdmmRun{};
  R->batched = batched;
  R->t0 = now();
  fde::AdmmConsts& k = R->k;
  k.n = c->N;
  k.plane = c->nx * c->ny;
  k.nt = c->nt;
  k.rho = q.rho;
  k.delta = q.delta;
  k.e_y = s.e_y;
  k.e_u = s.e_u;
  k.k_u = s.k_u;
  k.ya = q.ya;
  k.yb = q.yb;
  k.ua = q.ua;
  k.ub = q.ub;
  k.prox = q.prox;
  k.cy = s.cy;
  k.cu = s.cu;
  k.gamma = q.gamma;
  k.wts = c->wts;
  k.Mu = c->Mu;
  k.Mp = c->Mp;
  k.invMp = c->invMp;
  k.lya = c->bya;
  k.lyb = c->byb;
  k.lua = c->bua;
  k.lub = c->bub;
  fde::AdmmFields& f = R->f;
  f.yhat = yhat;
  f.g = g;
  f.y = y;
  f.u = u;
  f.zy = zy;
  f.zu = zu;
  f.p = p;
  f.wy = wy;
  f.wu = wu;
  f.r = c->ar;
  f.Ru = c->Ru;
  f.v = c->av;
  f.c = c->ac;
  f.By = c->By;
  f.partial = c->part_max;
  R->j = 1;
  return admm_enqueue_iteration(c, R);
}

// Consume the completed readback and enqueue the next phase.  A negative
// return is an error (the run is over); R->phase == PH_DONE marks the end.
fde_status admm_advance(fde_ctx* c, AdmmRun* R) {
  const auto& s = c->su;
  const fde_admm_params& q = c->prm;
  const double psi = s.psi;
  switch (R->phase) {
    case PH_PCG: {
      const bool mr = q.krylov_solver == 1;
      if (!(mr ? minres_continue(c, &R->mr) : krylov_continue(c, &R->kr))) return FDE_OK;
      R->t_pcg += now() - R->tp;
      const fde_status kst = mr ? R->mr.status : R->kr.status;
      if (kst < 0) {
        R->phase = PH_DONE;
        return kst;
      }
      const int it = mr ? R->mr.iters : R->kr.iters;
      R->predict = it > 2 ? it : 2;  // the next x-step usually needs about as many
      R->st.pcg_total += it;
      R->st.pcg_last = it;
      if (it > R->st.pcg_max) R->st.pcg_max = it;
      // 3-5. By ; p, u recovery ; projection ; dual updates ; residual maxima
      HIP_TRY(hipEventRecord(c->ph_ev[2], c->stream));
      HIP_TRY(apply_op(c, R->f.y, c->By, false, psi, c->fa, c->fb, nullptr, nullptr, nullptr, nullptr, nullptr,
                       nullptr, nullptr));
      int nb = 0;
      // PCG runs keep M_p^{-1} B y in fw for the next x-step's initial residual
      R->f.byp = mr ? nullptr : c->fw;
      // (with the next iteration's right-hand side pieces, computed from the
      // new iterate while it is in registers)
      HIP_TRY(fde::launch_admm_update(R->k, R->f, psi, c->stream, &nb, true));
      R->have_byp = !mr;
      R->have_rhs = true;
      HIP_TRY(fde::launch_max3_finalize(c->part_max, nb, c->scal, c->stream));
      HIP_TRY(hipEventRecord(c->ph_ev[3], c->stream));
      R->phase = PH_RES;
      return post_readback(c);
    }
    case PH_RES: {
      fde_admm_stats& st = R->st;
      {
        // this iteration's phases (complete: the readback behind them has finished)
        float ms[3] = {0, 0, 0};
        for (int k = 0; k < 3; ++k) HIP_TRY(hipEventElapsedTime(&ms[k], c->ph_ev[k], c->ph_ev[k + 1]));
        st.t_rhs += 1e-3 * ms[0];
        st.t_krylov += 1e-3 * ms[1];
        st.t_update += 1e-3 * ms[2];
      }
      st.admm_iters = R->j;
      st.r_p = c->h_scal[fde::kResP];
      st.r_y = c->h_scal[fde::kResY];
      st.r_u = c->h_scal[fde::kResU];
      if (std::isnan(st.r_p) || std::isnan(st.r_y) || std::isnan(st.r_u)) {
        R->phase = PH_DONE;
        return (fde_status)fail(FDE_ENONFINITE, "non-finite ADMM residual");
      }
      R->prev_min = std::fmin(st.r_p, std::fmin(st.r_y, st.r_u));
      // 6. termination (Sec. 6.1)
      const bool conv = q.admm_tol > 0 && std::fmax(st.r_p, std::fmax(st.r_y, st.r_u)) <= q.admm_tol;
      if (conv) R->status = FDE_OK;
      if (conv || R->j >= q.admm_maxit) {
        int nb = 0;
        HIP_TRY(fde::launch_objective(c->N, c->nx * c->ny, c->wts, q.gamma, R->f.y, R->f.yhat, R->f.u, c->part_pq,
                                      c->stream, &nb));
        HIP_TRY(fde::launch_pcg_scalar(fde::FIN_DOT, c->part_pq, nb, c->scal, c->ints, c->stream));
        // dual infeasibility (Sec. 6.1 reports it): B^T p = D^T lambda, lambda = psi p
        HIP_TRY(apply_op(c, R->f.p, c->fw, true, psi, c->fa, c->fb, nullptr, nullptr, nullptr, nullptr, nullptr,
                         nullptr, nullptr));
        HIP_TRY(fde::launch_dual_inf(R->k, R->f, q.gamma, c->fw, c->part_max, c->scal, c->stream));
        R->phase = PH_OBJ;
        return post_readback(c);
      }
      R->j += 1;
      return admm_enqueue_iteration(c, R);
    }
    case PH_OBJ: {
      R->st.J = c->h_scal[fde::kDot];
      R->st.dual_inf = c->h_scal[fde::kDual];
      R->st.t_total = now() - R->t0;
      R->st.t_pcg = R->t_pcg;
      R->phase = PH_DONE;
      return FDE_OK;
    }
    default:
      return FDE_OK;
  }
}

fde_status free_all(fde_ctx* c) {
  drop_pcg_graph(c);
  for (hipEvent_t ev : c->pt_ev) (void)hipEventDestroy(ev);
  c->pt_ev.clear();
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  c->cap_stream = nullptr;
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  if (c->ev) (void)hipEventDestroy(c->ev);
  c->ev = nullptr;
  for (hipEvent_t& pe : c->ph_ev) {
    if (pe) (void)hipEventDestroy(pe);
    pe = nullptr;
  }
  if (c->h_ms) (void)hipHostFree(c->h_ms);
  c->h_ms = nullptr;
  c->mr_ready = false;
  if (c->h_scal) (void)hipHostFree(c->h_scal);
  if (c->h_ints) (void)hipHostFree(c->h_ints);
  c->h_scal = nullptr;
  c->h_ints = nullptr;
  return FDE_OK;
}

fde_status upload_admm_tables(fde_ctx* c) {
  const auto& s = c->su;
  const size_t bytes = sizeof(double) * c->nt;
  HIP_TRY(hipMemcpy(c->invMp, s.invMp.data(), bytes, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->My, s.My.data(), bytes, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->Mu, s.Mu.data(), bytes, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->Mp, s.Mp.data(), bytes, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->wts, s.wts.data(), bytes, hipMemcpyHostToDevice));
  if (c->prm.precond_kind == 2) {
    if (s.ds_tab.size() > c->ds_tab_n) {
      // (a superseded smaller table stays in the context's allocations until it is destroyed)
      HIP_TRY(c->alloc(&c->ds_tab, s.ds_tab.size()));
      c->ds_tab_n = s.ds_tab.size();
    }
    if (!c->ds_class) HIP_TRY(c->alloc(&c->ds_class, (size_t)c->nt));
    HIP_TRY(hipMemcpy(c->ds_tab, s.ds_tab.data(), sizeof(double) * s.ds_tab.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->ds_class, s.ds_class.data(), sizeof(int) * s.ds_class.size(), hipMemcpyHostToDevice));
  }
  return FDE_OK;
}

// ---------------------------------------------------------------------------
// Adjoint state equation D^T lambda = f, f = -J1 (y - yhat) - wy.
// D^T = C_t^T (x) I - L_x^T - L_y^T with C_t lower-triangular Toeplitz in time
// (first column c: implicit Euler (1, -1)/h_t, or the Caputo weights of
// eq. (4.5) over h_t^alpha_t), so lambda is found by backward time stepping:
// for k = nt-1 .. 0
//     A^T lambda_k = f_k - sum_{j > k} c_{j-k} lambda_j,   A = c_0 I - L_x - L_y,
// a 2-D problem whose transposed Toeplitz products run the weights reversed
// (G^T for G).  Each step: BiCGSTAB, right-preconditioned by the inverse of
// the transposed 2-D T. Chan circulant (eigenvalues conj(c_0 - lx - ly)),
// warm-started from lambda_{k+1}.
// ---------------------------------------------------------------------------
struct SliceOps {
  fde_ctx* c;
  int64_t plane;
  // y = A^T x on one slice
  hipError_t applyAT(const double* x, double* y) {
    fde::LinePassArgs a = line_args(c);
    a.nt = 1;
    a.in = x;
    a.out = c->fa;
    a.L = c->su.x.L;
    a.tw = c->twx_emb;
    a.lamA = c->lxTA;
    a.lamB = c->lxTB;
    a.s_time = c->su.ct[0];  // diagonal of the time matrix (1/h_t for implicit Euler)
    a.s_sp = -1.0;
    hipError_t e = fde::launch_xpass(a, true, c->var, c->stream, nullptr);
    if (e != hipSuccess) return e;
    fde::LinePassArgs b = line_args(c);
    b.nt = 1;
    b.in = x;
    b.acc = c->fa;
    b.out = y;
    b.L = c->su.y.L;
    b.tw = c->twy_emb;
    b.lamA = c->lyTA;
    b.lamB = c->lyTB;
    b.s_sp = -1.0;
    b.tile = c->tile_line_y;
    return fde::launch_ypass(b, true, c->var, c->stream, nullptr);
  }
  // z = C(A)^{-T} r on one slice
  hipError_t precond(double* r, double* z) {
    fde::PrecondArgs a = pre_args(c, r, z);
    a.nt = 1;
    a.twt = c->adj_twt;
    a.lam_t = c->adj_lt;
    a.psi = 1.0;
    a.inv_n = 1.0 / (double)plane;
    a.div_mode = 1;
    a.ds_tab = nullptr;  // the transposed slice operator's own circulant, no scaling of S
    a.ds_class = nullptr;
    return fde::launch_precond(a, c->fp32, c->stream, nullptr, nullptr);
  }
  hipError_t dots(int count, const double* const* a, const double* const* b) {
    return fde::launch_dots(plane, count, a, b, c->part_dots, c->scal, c->stream);
  }
};

fde_status read_dots(fde_ctx* c, double* out, int count) {
  const fde_status st = sync_scalars(c);
  if (st != FDE_OK) return st;
  for (int j = 0; j < count; ++j) out[j] = c->h_scal[fde::kD0 + j];
  return FDE_OK;
}

fde_status adjoint_solve_impl(fde_ctx* c, const double* yhat, const double* y, const double* wy, double* lam) {
  using namespace fde;
  const int64_t plane = (int64_t)c->nx * c->ny;
  SliceOps op{c, plane};
  const double tol = 1e-13;
  const int maxit = 500;
  const std::vector<double>& ct = c->su.ct;
  double* f = c->bvec;
  HIP_TRY(launch_adjoint_rhs(c->N, (int)plane, c->wts, y, yhat, wy, f, c->stream));
  double *bk = c->By, *r = c->r, *rh = c->q, *p = c->pk, *v = c->fw, *sv = c->ar, *tv = c->Ru, *ph = c->av,
         *sh = c->ac;
  for (int k = c->nt - 1; k >= 0; --k) {
    double* x = lam + (size_t)k * plane;
    const double* fk = f + (size_t)k * plane;
    const double* xn = (k + 1 < c->nt) ? lam + (size_t)(k + 1) * plane : nullptr;
    // b_k = f_k - sum_{j > k} c_{j-k} lambda_j (two history terms per launch; zero weights skipped) ;
    // x0 = lambda_{k+1}
    HIP_TRY(launch_lincomb(plane, 1.0, fk, xn ? -ct[1] : 0.0, xn, 0.0, nullptr, bk, c->stream));
    for (int j = k + 2; j < c->nt; j += 2) {
      const double c0 = -ct[j - k], c1 = (j + 1 < c->nt) ? -ct[j + 1 - k] : 0.0;
      if (c0 == 0.0 && c1 == 0.0) continue;
      HIP_TRY(launch_lincomb(plane, 1.0, bk, c0, lam + (size_t)j * plane, c1,
                             c1 != 0.0 ? lam + (size_t)(j + 1) * plane : nullptr, bk, c->stream));
    }
    HIP_TRY(launch_lincomb(plane, 1.0, xn, 0.0, nullptr, 0.0, nullptr, x, c->stream));
    HIP_TRY(op.applyAT(x, v));
    HIP_TRY(launch_lincomb(plane, 1.0, bk, -1.0, v, 0.0, nullptr, r, c->stream));
    HIP_TRY(launch_lincomb(plane, 1.0, r, 0.0, nullptr, 0.0, nullptr, rh, c->stream));
    HIP_TRY(launch_lincomb(plane, 0.0, nullptr, 0.0, nullptr, 0.0, nullptr, p, c->stream));
    HIP_TRY(launch_lincomb(plane, 0.0, nullptr, 0.0, nullptr, 0.0, nullptr, v, c->stream));
    double d[4];
    {
      const double* a2[2] = {bk, r};
      const double* b2[2] = {bk, r};
      HIP_TRY(op.dots(2, a2, b2));
      fde_status st = read_dots(c, d, 2);
      if (st != FDE_OK) return st;
    }
    const double bnorm = std::sqrt(d[0]);
    double rr = d[1];
    if (bnorm == 0.0 || std::sqrt(rr) <= tol * bnorm) continue;
    double rho = 1.0, alpha = 1.0, omega = 1.0, rho1 = rr;  // (rhat, r) = (r, r) at the start
    bool ok = false;
    for (int it = 0; it < maxit; ++it) {
      const double beta = (rho1 / rho) * (alpha / omega);
      // p = r + beta (p - omega v)
      HIP_TRY(launch_lincomb(plane, 1.0, r, beta, p, -beta * omega, v, p, c->stream));
      HIP_TRY(op.precond(p, ph));
      HIP_TRY(op.applyAT(ph, v));
      {
        const double* a1[1] = {rh};
        const double* b1[1] = {v};
        HIP_TRY(op.dots(1, a1, b1));
        fde_status st = read_dots(c, d, 1);
        if (st != FDE_OK) return st;
      }
      alpha = rho1 / d[0];
      HIP_TRY(launch_lincomb(plane, 1.0, r, -alpha, v, 0.0, nullptr, sv, c->stream));
      HIP_TRY(op.precond(sv, sh));
      HIP_TRY(op.applyAT(sh, tv));
      {
        const double* a3[3] = {sv, tv, tv};
        const double* b3[3] = {sv, sv, tv};
        HIP_TRY(op.dots(3, a3, b3));
        fde_status st = read_dots(c, d, 3);
        if (st != FDE_OK) return st;
      }
      if (std::sqrt(d[0]) <= tol * bnorm) {
        HIP_TRY(launch_lincomb(plane, 1.0, x, alpha, ph, 0.0, nullptr, x, c->stream));
        ok = true;
        break;
      }
      omega = d[1] / d[2];
      HIP_TRY(launch_lincomb(plane, 1.0, x, alpha, ph, omega, sh, x, c->stream));
      HIP_TRY(launch_lincomb(plane, 1.0, sv, -omega, tv, 0.0, nullptr, r, c->stream));
      {
        const double* a2[2] = {r, rh};
        const double* b2[2] = {r, r};
        HIP_TRY(op.dots(2, a2, b2));
        fde_status st = read_dots(c, d, 2);
        if (st != FDE_OK) return st;
      }
      if (!std::isfinite(d[0])) return (fde_status)fail(FDE_ENONFINITE, "non-finite residual in the adjoint solve");
      if (std::sqrt(d[0]) <= tol * bnorm) {
        ok = true;
        break;
      }
      rho = rho1;
      rho1 = d[1];
    }
    if (!ok) return (fde_status)fail(FDE_ENOTCONV, "adjoint solve: BiCGSTAB did not converge in a time step");
  }
  return FDE_OK;
}

fde_status create_impl(const fde_problem* prob, const fde_admm_params* prm, void* stream, fde_ctx** out) {
  if (!out) return (fde_status)fail(FDE_EINVAL, "out is NULL");
  *out = nullptr;
  auto* c = new fde_ctx();
  std::string msg;
  int st = fde::host::build_setup(prob, prm, &c->su, &msg);
  if (st != FDE_OK) {
    delete c;
    return (fde_status)fail(st, msg);
  }
  c->prob = *prob;
  c->prob.dplus = nullptr;
  c->prob.dminus = nullptr;
  c->prm = *prm;
  c->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return (fde_status)fail(FDE_EHIP, "fde_create: no current HIP device");
  }
  c->nx = prob->nx;
  c->ny = prob->ny;
  c->nt = prob->nt;
  c->H = prob->nx / 2 + 1;
  c->N = (int64_t)prob->nx * prob->ny * prob->nt;
  c->var = c->su.var;
  c->fp32 = prob->precond_fp32 != 0;
  // FDE_NO_GRAPH=1 launches the PCG iteration kernel by kernel (no HIP graph)
  // FDE_CONV_SEPARATE=1 / =0 forces the stand-alone / fused PCG convergence test
  if (const char* cs = std::getenv("FDE_CONV_SEPARATE")) c->conv_sep = (cs[0] == '1') ? 1 : (cs[0] == '0' ? 0 : -1);
  const char* ng = std::getenv("FDE_NO_GRAPH");
  c->use_graph = !(ng && ng[0] == '1');
  // FDE_TILES=a,b,c fixes the column-tile variants (0..2) instead of the default widest tiles
  if (const char* tv = std::getenv("FDE_TILES")) {
    int a = 0, b = 0, d = 0;
    if (std::sscanf(tv, "%d,%d,%d", &a, &b, &d) == 3) {
      auto clampv = [](int v) { return v < 0 ? 0 : (v > 2 ? 2 : v); };
      c->tile_line_y = clampv(a);
      c->tile_pre_y = clampv(b);
      c->tile_pre_t = clampv(d);
    }
  }
  auto& s = c->su;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (e == hipSuccess && x != hipSuccess) e = x;
  };
  // operator tables (x: length 2nx, y: 2ny)
  if (c->var) {
    chk(upload_c(c, &c->lxA, s.x.lamG));
    chk(upload_c(c, &c->lxB, s.x.lamGT));
    chk(upload_c(c, &c->lxTA, s.x.lamGT));  // transpose: G^T (d+ v) + G (d- v)
    chk(upload_c(c, &c->lxTB, s.x.lamG));
    chk(upload_c(c, &c->lyA, s.y.lamG));
    chk(upload_c(c, &c->lyB, s.y.lamGT));
    chk(upload_c(c, &c->lyTA, s.y.lamGT));
    chk(upload_c(c, &c->lyTB, s.y.lamG));
    chk(upload(c, &c->dplus, s.dplus));
    chk(upload(c, &c->dminus, s.dminus));
  } else {
    chk(upload_c(c, &c->lxA, s.x.lamFwd));
    chk(upload_c(c, &c->lxTA, s.x.lamTr));
    chk(upload_c(c, &c->lyA, s.y.lamFwd));
    chk(upload_c(c, &c->lyTA, s.y.lamTr));
  }
  chk(upload_c(c, &c->dxA, s.x.dopA));
  chk(upload_c(c, &c->dxB, s.x.dopB));
  chk(upload_c(c, &c->dyA, s.y.dopA));
  chk(upload_c(c, &c->dyB, s.y.dopB));
  chk(upload_c(c, &c->twx_emb, s.x.tw_emb));
  chk(upload_c(c, &c->twy_emb, s.y.tw_emb));
  chk(upload_tw(c, &c->twx, s.x.tw, c->fp32));
  chk(upload_tw(c, &c->twy, s.y.tw, c->fp32));
  chk(upload_tw(c, &c->twt, s.tw_t, c->fp32));
  chk(upload_c(c, &c->tcx, s.x.tchan));
  chk(upload_c(c, &c->tcy, s.y.tchan));
  chk(upload_c(c, &c->tct, s.tchan_t));
  c->frac_t = s.frac_t;
  // coefficient fields that vary along x only make every y-line constant-coefficient
  // (FDE_YCOL=0 keeps the general variable-coefficient y-pass)
  if (c->var) {
    bool col = true;
    for (const std::vector<double>* f : {&s.dplus, &s.dminus})
      for (int j = 1; j < c->ny && col; ++j)
        for (int i = 0; i < c->nx; ++i)
          if ((*f)[(size_t)j * c->nx + i] != (*f)[i]) {
            col = false;
            break;
          }
    const char* ev = std::getenv("FDE_YCOL");
    c->ycol = col && !(ev && ev[0] == '0');
  }
  if (s.frac_t) {
    chk(upload_c(c, &c->ltA, s.lam_t));
    chk(upload_c(c, &c->ltTA, s.lam_tT));
    chk(upload_c(c, &c->twt_emb, s.tw_t_emb));
  }
  chk(c->alloc(&c->invMp, c->nt));
  chk(c->alloc(&c->My, c->nt));
  chk(c->alloc(&c->Mu, c->nt));
  chk(c->alloc(&c->Mp, c->nt));
  chk(c->alloc(&c->wts, c->nt));
  chk(upload(c, &c->ones, std::vector<double>(c->nt, 1.0)));
  // workspace
  const size_t N = (size_t)c->N;
  double** fields[] = {&c->fa, &c->fw, &c->fb, &c->q, &c->r, &c->z, &c->pk, &c->bvec,
                       &c->ar, &c->Ru, &c->av, &c->ac, &c->By};
  for (double** f : fields) chk(c->alloc(f, N));
  const size_t specn = (size_t)c->H * c->ny * c->nt;
  if (c->fp32) {
    float2* sp = nullptr;
    chk(c->alloc(&sp, specn));
    c->spec = sp;
  } else {
    double2* sp = nullptr;
    chk(c->alloc(&sp, specn));
    c->spec = sp;
  }
  c->maxpart = max_partials(c->nx, c->ny, c->nt, s.frac_t);
  chk(c->alloc(&c->part_pq, 2 * (size_t)c->maxpart));
  chk(c->alloc(&c->part_rr, (size_t)c->maxpart));
  // (r, z) partials: one per block of the preconditioner's t-pass (at most H * ny)
  chk(c->alloc(&c->part_rz, std::max((size_t)c->maxpart, (size_t)c->H * (size_t)c->ny)));
  chk(c->alloc(&c->part_max, 3 * (size_t)c->maxpart));
  chk(c->alloc(&c->part_dots, 4 * (size_t)2048));
  chk(upload_c(c, &c->adj_lt, std::vector<cd>{cd(s.ct[0], 0.0)}));
  chk(upload_tw(c, &c->adj_twt, std::vector<cd>{cd(1.0, 0.0)}, c->fp32));
  chk(c->alloc(&c->scal, fde::kNumScalars));
  chk(c->alloc(&c->ints, fde::kNumInts));
  if (e == hipSuccess) chk(hipHostMalloc((void**)&c->h_scal, sizeof(double) * fde::kNumScalars, hipHostMallocDefault));
  if (e == hipSuccess) chk(hipHostMalloc((void**)&c->h_ints, sizeof(int) * fde::kNumInts, hipHostMallocDefault));
  if (e == hipSuccess) chk(hipEventCreateWithFlags(&c->ev, hipEventDisableTiming));
  for (hipEvent_t& pe : c->ph_ev)
    if (e == hipSuccess) chk(hipEventCreate(&pe));
  if (e == hipSuccess) chk(hipMemset(c->scal, 0, sizeof(double) * fde::kNumScalars));
  if (e == hipSuccess) chk(hipMemset(c->ints, 0, sizeof(int) * fde::kNumInts));
  if (e != hipSuccess) {
    const int code = (e == hipErrorOutOfMemory) ? FDE_ENOMEM : FDE_EHIP;
    free_all(c);
    delete c;
    return (fde_status)fail(code, std::string("fde_create: ") + hipGetErrorString(e));
  }
  fde_status us = upload_admm_tables(c);
  // the MINRES x-step's workspace is allocated here, not inside the solve
  if (us == FDE_OK && c->prm.krylov_solver == 1) us = ensure_minres(c);
  if (us != FDE_OK) {
    free_all(c);
    delete c;
    return us;
  }
  *out = c;
  return FDE_OK;
}

// lower <= upper at every point (arrays where given, the scalar bounds elsewhere), no NaN
fde_status check_bounds(fde_ctx* c, const double* ya, const double* yb, const double* ua, const double* ub,
                        const fde_admm_params& q, const char* who) {
  int nb = 0;
  HIP_TRY(fde::launch_bounds_check(c->N, ya, yb, ua, ub, q.ya, q.yb, q.ua, q.ub, c->part_max, c->stream, &nb));
  HIP_TRY(fde::launch_max3_finalize(c->part_max, nb, c->scal, c->stream));
  const fde_status st = sync_scalars(c);
  if (st != FDE_OK) return st;
  if (c->h_scal[fde::kResP] != 0.0 || c->h_scal[fde::kResY] != 0.0)
    return (fde_status)fail(FDE_EINVAL, std::string(who) + ": a lower bound exceeds its upper bound (or is NaN)");
  return FDE_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* fde_last_error(void) { return g_err.c_str(); }

const char* fde_version(void) { return "fde-mi355x 0.1 (gfx950)"; }

fde_status fde_validate(const fde_problem* prob, const fde_admm_params* prm) {
  std::string msg;
  const int st = fde::host::validate(prob, prm, &msg);
  if (st != FDE_OK) return (fde_status)fail(st, msg);
  g_err.clear();
  return FDE_OK;
}

fde_status fde_host_tables(const fde_problem* prob, const fde_admm_params* prm, double* scal, double* lam_x,
                           double* lam_y, double* lam_t, double* gx, double* gy) {
  fde::host::Setup s;
  std::string msg;
  const int st = fde::host::build_setup(prob, prm, &s, &msg);
  if (st != FDE_OK) return (fde_status)fail(st, msg);
  if (scal) {
    const double v[8] = {s.psi, s.x.h, s.y.h, s.ht, s.a, s.inv_mbar, s.e_u, s.k_u};
    std::memcpy(scal, v, sizeof v);
  }
  auto put = [](double* dst, const std::vector<cd>& src) {
    if (!dst) return;
    for (size_t i = 0; i < src.size(); ++i) {
      dst[2 * i] = src[i].real();
      dst[2 * i + 1] = src[i].imag();
    }
  };
  put(lam_x, s.x.tchan);
  put(lam_y, s.y.tchan);
  put(lam_t, s.tchan_t);
  if (gx) std::memcpy(gx, s.x.g.data(), sizeof(double) * s.x.g.size());
  if (gy) std::memcpy(gy, s.y.g.data(), sizeof(double) * s.y.g.size());
  return FDE_OK;
}

fde_status fde_host_diag_scaling(const fde_problem* prob, const fde_admm_params* prm, double* delta) {
  if (!prm || !delta) return (fde_status)fail(FDE_EINVAL, "fde_host_diag_scaling: null argument");
  fde_admm_params q = *prm;
  q.precond_kind = 2;
  q.krylov_solver = 0;
  fde::host::Setup s;
  std::string msg;
  const int st = fde::host::build_setup(prob, &q, &s, &msg);
  if (st != FDE_OK) return (fde_status)fail(st, msg);
  const size_t plane = (size_t)s.nx * s.ny;
  for (int t = 0; t < s.nt; ++t)
    for (size_t k = 0; k < plane; ++k)
      delta[(size_t)t * plane + k] = s.ds_tab[(size_t)s.ds_class[t] * plane + k];
  return FDE_OK;
}

fde_status fde_create(const fde_problem* prob, const fde_admm_params* prm, void* stream, fde_ctx** out) {
  return create_impl(prob, prm, stream, out);
}

fde_status fde_destroy(fde_ctx* ctx) {
  if (!ctx) return FDE_OK;
  (void)hipStreamSynchronize(ctx->stream);
  free_all(ctx);
  delete ctx;
  return FDE_OK;
}

fde_status fde_set_params(fde_ctx* ctx, const fde_admm_params* prm) {
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  std::string msg;
  const int st = fde::host::validate_params(prm, &msg);
  if (st != FDE_OK) return (fde_status)fail(st, msg);
  if (ctx->bya || ctx->byb || ctx->bua || ctx->bub) {
    // per-point bounds stay; the new scalar bounds must agree with them
    const fde_status bs = check_bounds(ctx, ctx->bya, ctx->byb, ctx->bua, ctx->bub, *prm, "fde_set_params");
    if (bs != FDE_OK) return bs;
  }
  ctx->prm = *prm;
  fde::host::set_admm_scalings(prm, &ctx->su);
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  // the captured PCG iterations hold the preconditioner's scalars (a, 1/mbar_p,
  // the matching term) by value: recapture on the next solve
  drop_pcg_graph(ctx);
  const fde_status us = upload_admm_tables(ctx);
  if (us != FDE_OK || prm->krylov_solver != 1) return us;
  return ensure_minres(ctx);
}

fde_status fde_apply_A(fde_ctx* ctx, const double* x, double* y, int transpose) {
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  if (!x || !y || x == y) return (fde_status)fail(FDE_EINVAL, "fde_apply_A: null or aliased fields");
  CHECK_ALIGNED("fde_apply_A", x, y);
  const bool tr = transpose != 0;
  HIP_TRY(apply_op(ctx, x, y, tr, 1.0, ctx->fa, ctx->fb, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                   nullptr));
  return FDE_OK;
}

fde_status fde_apply_A_noalloc(fde_ctx* ctx, const double* x, double* y, int transpose) {
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  if (!x || !y || x == y) return (fde_status)fail(FDE_EINVAL, "fde_apply_A_noalloc: null or aliased fields");
  CHECK_ALIGNED("fde_apply_A_noalloc", x, y);
  // intermediate fields: one (implicit Euler) or two (fractional time order) of N points
  const size_t need = (ctx->frac_t ? 2 : 1) * (size_t)ctx->N;
  if (need > kScratchDoubles)
    return (fde_status)fail(FDE_EINVAL, "fde_apply_A_noalloc: the grid needs " + std::to_string(need) +
                                            " doubles of workspace; the static workspace holds " +
                                            std::to_string(kScratchDoubles));
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != ctx->device)
    return (fde_status)fail(FDE_EINVAL, "fde_apply_A_noalloc: the context's device must be current");
  double* ws = nullptr;
  const int st = scratch_address(dev, &ws);
  if (st != FDE_OK) return (fde_status)st;
  // N is even (nx is), so ws + N keeps the 16-byte alignment of the pair accesses
  HIP_TRY(apply_op(ctx, x, y, transpose != 0, 1.0, ws, ws + ctx->N, nullptr, nullptr, nullptr, nullptr, nullptr,
                   nullptr, nullptr));
  return FDE_OK;
}

fde_status fde_apply_S(fde_ctx* ctx, const double* x, double* y) {
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  if (!x || !y || x == y) return (fde_status)fail(FDE_EINVAL, "fde_apply_S: null or aliased fields");
  CHECK_ALIGNED("fde_apply_S", x, y);
  HIP_TRY(apply_S(ctx, x, y, nullptr, nullptr, nullptr));
  return FDE_OK;
}

fde_status fde_precond(fde_ctx* ctx, const double* r, double* z) {
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  if (!r || !z) return (fde_status)fail(FDE_EINVAL, "fde_precond: null field");
  CHECK_ALIGNED("fde_precond", r, z);
  fde::PrecondArgs a = pre_args(ctx, const_cast<double*>(r), z);  // r is only read (no fused update)
  HIP_TRY(fde::launch_precond(a, ctx->fp32, ctx->stream, nullptr, nullptr));
  return FDE_OK;
}

fde_status fde_krylov(fde_ctx* ctx, const double* b, double* x, int* iters, double* relres) {
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  if (!b || !x || b == x) return (fde_status)fail(FDE_EINVAL, "fde_krylov: null or aliased fields");
  CHECK_ALIGNED("fde_krylov", b, x);
  int it = 0;
  double rr = 0;
  // a first chunk of two 4-iteration graph launches; iterations past
  // convergence return at once (device done flag)
  const fde_status st = krylov(ctx, b, x, ctx->prm.krylov_tol, ctx->prm.krylov_maxit, &it, &rr, 8);
  if (iters) *iters = it;
  if (relres) *relres = rr;
  return st;
}

fde_status fde_set_bounds(fde_ctx* ctx, const double* ya, const double* yb, const double* ua, const double* ub) {
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  CHECK_ALIGNED("fde_set_bounds", ya, yb, ua, ub);
  fde_ctx* c = ctx;
  fde_status st = check_bounds(c, ya, yb, ua, ub, c->prm, "fde_set_bounds");
  if (st != FDE_OK) return st;
  const size_t bytes = sizeof(double) * (size_t)c->N;
  const double* src[4] = {ya, yb, ua, ub};
  double** mem[4] = {&c->bya_mem, &c->byb_mem, &c->bua_mem, &c->bub_mem};
  double** use[4] = {&c->bya, &c->byb, &c->bua, &c->bub};
  for (int k = 0; k < 4; ++k) {
    if (!src[k]) {
      *use[k] = nullptr;
      continue;
    }
    if (!*mem[k]) {
      const hipError_t e = c->alloc(mem[k], (size_t)c->N);
      if (e != hipSuccess)
        return (fde_status)fail(e == hipErrorOutOfMemory ? FDE_ENOMEM : FDE_EHIP, "fde_set_bounds: allocation");
    }
    HIP_TRY(hipMemcpyAsync(*mem[k], src[k], bytes, hipMemcpyDeviceToDevice, c->stream));
    *use[k] = *mem[k];
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return FDE_OK;
}

fde_status fde_minres(fde_ctx* ctx, const double* b_y, const double* b_u, const double* b_p, double* y, double* u,
                      double* p, int* iters, double* relres) {
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  if (!b_y || !b_u || !b_p || !y || !u || !p) return (fde_status)fail(FDE_EINVAL, "fde_minres: null field");
  const void* in[3] = {b_y, b_u, b_p};
  const void* xs[3] = {y, u, p};
  for (const void* a : in)
    for (const void* b : xs)
      if (a == b) return (fde_status)fail(FDE_EINVAL, "fde_minres: right-hand side aliases an unknown");
  if (y == u || y == p || u == p) return (fde_status)fail(FDE_EINVAL, "fde_minres: aliased unknowns");
  CHECK_ALIGNED("fde_minres", b_y, b_u, b_p, y, u, p);
  MinresRun m;
  fde_status st = minres_begin(ctx, fde::Triple{const_cast<double*>(b_y), const_cast<double*>(b_u),
                                                const_cast<double*>(b_p)},
                               fde::Triple{y, u, p}, ctx->prm.krylov_tol, ctx->prm.krylov_maxit, false, 0, &m);
  if (st != FDE_OK) return st;
  while (true) {
    if ((st = wait_readback(ctx)) != FDE_OK) return st;
    if (minres_continue(ctx, &m)) break;
  }
  if (iters) *iters = m.iters;
  if (relres) *relres = m.relres;
  return m.status;
}

fde_status fde_admm_solve(fde_ctx* ctx, const double* yhat, const double* g, double* y, double* u, double* zy,
                          double* zu, double* p, double* wy, double* wu, fde_admm_stats* stats) {
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  if (!yhat || !y || !u || !zy || !zu || !p || !wy || !wu)
    return (fde_status)fail(FDE_EINVAL, "fde_admm_solve: null field");
  AdmmRun R;
  fde_status st = admm_begin(ctx, &R, yhat, g, y, u, zy, zu, p, wy, wu);
  while (st >= 0 && R.phase != PH_DONE) {
    if ((st = wait_readback(ctx)) != FDE_OK) break;
    st = admm_advance(ctx, &R);
  }
  if (stats) *stats = R.st;
  if (st < 0) return st;
  return R.status;
}

}  // extern "C"

struct fde_batch {
  std::vector<fde_ctx*> ctx;
  std::vector<hipStream_t> streams;
  hipStream_t lockstep = nullptr;  // the one stream of the lockstep mode
};

namespace {
void batch_free(fde_batch* b) {
  for (fde_ctx* c : b->ctx) fde_destroy(c);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  if (b->lockstep) (void)hipStreamDestroy(b->lockstep);
  delete b;
}

// ---------------------------------------------------------------------------
// Lockstep batch: the PCG iterations of all instances as batched pass
// launches.  Each instance's PCG iteration is recorded once (its pass
// launches captured, not issued); the passes at each position are grouped by
// kernel and issued as one launch per group over a table of the instances'
// arguments (BatchArgs), each instance keeping its own block decomposition.
// Iterations after an instance's convergence return at once (its device done
// flag), as in the single solve.
// ---------------------------------------------------------------------------
struct PassGroup {
  const void* kern = nullptr;
  int threads = 0, blocks = 0, count = 0;
  const void* args = nullptr;  // device table of the members' arguments
  const int* first = nullptr;  // device prefix sums of their block counts
};

// The launches of one batch iteration over a set of members, and the device
// tables they read (one region: argument and prefix tables per group, the
// members' int-slot pointers, their gathered done flags).
struct BatchPlan {
  std::vector<std::vector<PassGroup>> pos;  // per pass position, its kernel groups
  std::vector<int> members;                 // instance indices
  const int* const* ints = nullptr;
  int* flags = nullptr;
};

struct BatchPcg {
  std::vector<std::vector<fde::RecordedPass>> rec;  // per instance, its recorded PCG iteration
  size_t region = 0;               // bytes of one plan region
  void* dev = nullptr;             // region 0: the full plan (graph); region 1: subset plans
  unsigned char* stage = nullptr;  // pinned staging of region 1
  int* h_flags = nullptr;          // pinned
  hipEvent_t ev = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BatchPlan full, sub;
  int count = 0;
};

void batch_pcg_free(BatchPcg* bp) {
  if (bp->exec) (void)hipGraphExecDestroy(bp->exec);
  if (bp->graph) (void)hipGraphDestroy(bp->graph);
  if (bp->cap) (void)hipStreamDestroy(bp->cap);
  if (bp->ev) (void)hipEventDestroy(bp->ev);
  if (bp->h_flags) (void)hipHostFree(bp->h_flags);
  if (bp->stage) (void)hipHostFree(bp->stage);
  if (bp->dev) (void)hipFree(bp->dev);
  *bp = BatchPcg{};
}

hipError_t batch_pcg_iteration(const BatchPlan& pl, hipStream_t s) {
  for (const auto& groups : pl.pos)
    for (const PassGroup& g : groups) {
      fde::BatchArgs<fde::LinePassArgs> ba{static_cast<const fde::LinePassArgs*>(g.args), g.first, g.count};
      void* kargs[] = {&ba};
      const hipError_t e = hipLaunchKernel(g.kern, dim3(g.blocks), dim3(g.threads), kargs, 0, s);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

// Group the recorded passes of `members` by kernel at each position and lay
// out their tables in `host` (region bytes, zeroed by the caller), with device
// addresses relative to `base`.  Returns the bytes used, 0 when they exceed
// `cap` (never for a subset of the members the region was sized for).
size_t batch_plan(const BatchPcg& bp, const std::vector<fde_ctx*>& cs, const std::vector<int>& members,
                  unsigned char* host, unsigned char* base, size_t cap, BatchPlan* pl) {
  using fde::RecordedPass;
  const size_t npos = bp.rec[members[0]].size();
  struct GroupHost {
    size_t pos;
    const void* kern;
    int threads, kind;
    std::vector<int> members;
  };
  std::vector<GroupHost> groups;
  for (size_t p = 0; p < npos; ++p) {
    const size_t g0 = groups.size();
    for (int i : members) {
      const RecordedPass& r = bp.rec[i][p];
      size_t g = g0;
      while (g < groups.size() && groups[g].kern != r.batch_kernel) ++g;
      if (g == groups.size()) groups.push_back(GroupHost{p, r.batch_kernel, r.threads, r.kind, {}});
      groups[g].members.push_back(i);
    }
  }
  auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t m = members.size();
  size_t total = 0;
  std::vector<size_t> off_args(groups.size()), off_first(groups.size());
  for (size_t g = 0; g < groups.size(); ++g) {
    const size_t asz = groups[g].kind == 0 ? sizeof(fde::LinePassArgs) : sizeof(fde::PrecondArgs);
    off_args[g] = total;
    total = align(total + asz * groups[g].members.size());
    off_first[g] = total;
    total = align(total + sizeof(int) * (groups[g].members.size() + 1));
  }
  const size_t off_ints = total;
  total = align(total + sizeof(int*) * m);
  const size_t off_flags = total;
  total = align(total + sizeof(int) * m);
  if (!host) return total;  // sizing pass
  if (total > cap) return 0;
  pl->pos.assign(npos, {});
  pl->members = members;
  for (size_t g = 0; g < groups.size(); ++g) {
    const GroupHost& G = groups[g];
    const size_t asz = G.kind == 0 ? sizeof(fde::LinePassArgs) : sizeof(fde::PrecondArgs);
    int* first = reinterpret_cast<int*>(host + off_first[g]);
    int blocks = 0;
    for (size_t k = 0; k < G.members.size(); ++k) {
      const RecordedPass& r = bp.rec[G.members[k]][G.pos];
      std::memcpy(host + off_args[g] + asz * k, r.args, asz);
      first[k] = blocks;
      blocks += r.blocks;
    }
    first[G.members.size()] = blocks;
    PassGroup pg;
    pg.kern = G.kern;
    pg.threads = G.threads;
    pg.blocks = blocks;
    pg.count = (int)G.members.size();
    pg.args = base + off_args[g];
    pg.first = reinterpret_cast<const int*>(base + off_first[g]);
    pl->pos[G.pos].push_back(pg);
  }
  const int** ints_host = reinterpret_cast<const int**>(host + off_ints);
  for (size_t k = 0; k < m; ++k) ints_host[k] = cs[members[k]]->ints;
  pl->ints = reinterpret_cast<const int* const*>(base + off_ints);
  pl->flags = reinterpret_cast<int*>(base + off_flags);
  return total;
}

// Record the PCG iterations of the instances cs (solution fields xs), build the
// plan over all of them and capture kGraphIters of its iterations in a graph;
// FDE_EINVAL when a pass has no batched form (the caller runs another mode).
fde_status batch_pcg_build(const std::vector<fde_ctx*>& cs, const std::vector<double*>& xs, BatchPcg* bp) {
  using fde::RecordedPass;
  const int n = (int)cs.size();
  bp->rec.assign(n, {});
  for (int i = 0; i < n; ++i) {
    fde::t_record = &bp->rec[i];
    const hipError_t e = enqueue_pcg_iteration_passes(cs[i], xs[i]);
    fde::t_record = nullptr;
    if (e != hipSuccess) return (fde_status)fail(FDE_EHIP, std::string("batch record: ") + hipGetErrorString(e));
  }
  const size_t npos = bp->rec[0].size();
  for (int i = 0; i < n; ++i) {
    if (bp->rec[i].size() != npos) return (fde_status)fail(FDE_EINVAL, "batch: instances with different pass lists");
    for (const RecordedPass& r : bp->rec[i])
      if (!r.batch_kernel) return (fde_status)fail(FDE_EINVAL, "batch: a pass without a batched form");
  }
  std::vector<int> all(n);
  for (int i = 0; i < n; ++i) all[i] = i;
  bp->region = batch_plan(*bp, cs, all, nullptr, nullptr, 0, nullptr);
  HIP_TRY(hipMalloc(&bp->dev, 2 * bp->region));
  HIP_TRY(hipHostMalloc((void**)&bp->stage, bp->region, hipHostMallocDefault));
  std::vector<unsigned char> host(bp->region, 0);
  unsigned char* d = static_cast<unsigned char*>(bp->dev);
  (void)batch_plan(*bp, cs, all, host.data(), d, bp->region, &bp->full);
  HIP_TRY(hipMemcpy(bp->dev, host.data(), bp->region, hipMemcpyHostToDevice));
  bp->count = n;
  HIP_TRY(hipHostMalloc((void**)&bp->h_flags, sizeof(int) * n, hipHostMallocDefault));
  HIP_TRY(hipEventCreateWithFlags(&bp->ev, hipEventDisableTiming));
  HIP_TRY(hipStreamCreateWithFlags(&bp->cap, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(bp->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int k = 0; k < kGraphIters && e == hipSuccess; ++k) e = batch_pcg_iteration(bp->full, bp->cap);
  const hipError_t e2 = hipStreamEndCapture(bp->cap, &bp->graph);
  if (e != hipSuccess || e2 != hipSuccess)
    return (fde_status)fail(FDE_EHIP, std::string("batch graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
  HIP_TRY(hipGraphInstantiate(&bp->exec, bp->graph, nullptr, nullptr, 0));
  return FDE_OK;
}

// Plan over a subset of the instances in region 1, uploaded on stream s (the
// previous subset plan's launches on s have finished: the caller waited).
fde_status batch_subset(BatchPcg* bp, const std::vector<fde_ctx*>& cs, const std::vector<int>& members, hipStream_t s) {
  std::memset(bp->stage, 0, bp->region);
  unsigned char* d1 = static_cast<unsigned char*>(bp->dev) + bp->region;
  const size_t used = batch_plan(*bp, cs, members, bp->stage, d1, bp->region, &bp->sub);
  if (used == 0) return (fde_status)fail(FDE_EHIP, "batch: subset tables exceed the region");
  HIP_TRY(hipMemcpyAsync(d1, bp->stage, used, hipMemcpyHostToDevice, s));
  return FDE_OK;
}

// Enqueue `iters` batch iterations of plan pl (the full plan as whole graphs),
// then gather its members' done flags into pinned memory behind bp->ev.
fde_status batch_chunk(BatchPcg* bp, const BatchPlan& pl, bool full, int iters, hipStream_t s) {
  if (full) {
    for (int k = 0; k < iters; k += kGraphIters) HIP_TRY(hipGraphLaunch(bp->exec, s));
  } else {
    for (int k = 0; k < iters; ++k) HIP_TRY(batch_pcg_iteration(pl, s));
  }
  const int m = (int)pl.members.size();
  HIP_TRY(fde::launch_gather_done(pl.ints, m, pl.flags, s));
  HIP_TRY(hipMemcpyAsync(bp->h_flags, pl.flags, sizeof(int) * m, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipEventRecord(bp->ev, s));
  return FDE_OK;
}
}  // namespace

extern "C" {

fde_status fde_batch_create(int count, const fde_problem* probs, const fde_admm_params* prms, fde_batch** out) {
  if (!out || !probs || !prms || count <= 0) return (fde_status)fail(FDE_EINVAL, "fde_batch_create: bad arguments");
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    const fde_status v = fde_validate(&probs[i], &prms[i]);
    if (v != FDE_OK) return (fde_status)fail(v, "instance " + std::to_string(i) + ": " + g_err);
  }
  auto* b = new fde_batch();
  for (int i = 0; i < count; ++i) {
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) {
      batch_free(b);
      return (fde_status)fail(FDE_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    b->streams.push_back(s);
    fde_ctx* c = nullptr;
    const fde_status st = fde_create(&probs[i], &prms[i], s, &c);
    if (st != FDE_OK) {
      const std::string msg = g_err;
      batch_free(b);
      return (fde_status)fail(st, "instance " + std::to_string(i) + ": " + msg);
    }
    b->ctx.push_back(c);
    // the PCG convergence test rides in the y-forward pass (the batched PCG
    // iteration has only pass launches); results are identical either way
    c->conv_sep = 0;
    const fde_status ts = fde_autotune(c, nullptr);  // cached per shape
    if (ts != FDE_OK) {
      const std::string msg = g_err;
      batch_free(b);
      return (fde_status)fail(ts, "instance " + std::to_string(i) + " autotune: " + msg);
    }
  }
  *out = b;
  return FDE_OK;
}

fde_status fde_batch_destroy(fde_batch* b) {
  if (b) batch_free(b);
  return FDE_OK;
}

}  // extern "C"

namespace {
// Lockstep mode of fde_batch_solve.  Each instance runs its ADMM phases on its
// own stream; the Krylov iterations of the x-steps run as batched pass
// launches on one more stream.  A batch starts when every live instance has
// enqueued its x-step set-up (the instances' ADMM iterations stay in step);
// its first chunk covers the largest iteration count of the previous x-steps.
// After each chunk the converged instances leave the launch plan (their blocks
// would only return at once) and go on with their update phases on their own
// streams while the others continue in the batch.  FDE_EINVAL (nothing run)
// when an instance has no batched form (MINRES x-step, a fractional time
// order, lengths without batched twins): the caller then runs the concurrent
// mode.
fde_status batch_lockstep(fde_batch* b, const double* const* yhat, const double* const* g, double* const* y,
                          double* const* u, double* const* zy, double* const* zu, double* const* p,
                          double* const* wy, double* const* wu, std::vector<AdmmRun>& R,
                          std::vector<fde_status>& res) {
  const int n = (int)b->ctx.size();
  for (fde_ctx* c : b->ctx)
    if (c->prm.krylov_solver != 0 || c->frac_t)
      return (fde_status)fail(FDE_EINVAL, "lockstep batch: an instance without batched passes");
  if (!b->lockstep) HIP_TRY(hipStreamCreateWithFlags(&b->lockstep, hipStreamNonBlocking));
  hipStream_t ls = b->lockstep;
  for (int i = 0; i < n; ++i) HIP_TRY(hipStreamSynchronize(b->ctx[i]->stream));
  const std::vector<fde_ctx*>& cs = b->ctx;
  const std::vector<double*> xs(y, y + n);
  BatchPcg bp;
  std::vector<hipEvent_t> join(n, nullptr);
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(ls);
    for (fde_ctx* c : cs) (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : join)
      if (e) (void)hipEventDestroy(e);
    batch_pcg_free(&bp);
  };
  fde_status st = batch_pcg_build(cs, xs, &bp);
  for (int i = 0; i < n && st == FDE_OK; ++i) {
    const hipError_t e = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
    if (e != hipSuccess) st = (fde_status)fail(FDE_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
  }
  if (st != FDE_OK) {
    cleanup();
    return st;
  }
  enum : char { LS_WAIT, LS_BATCH, LS_RUN };  // set-up enqueued / in the batch / own-stream phase pending
  std::vector<char> live(n, 0), state(n, LS_RUN);
  int remaining = 0, maxit = 0;
  for (int i = 0; i < n; ++i) {
    res[i] = admm_begin(cs[i], &R[i], yhat[i], g ? g[i] : nullptr, y[i], u[i], zy[i], zu[i], p[i], wy[i], wu[i],
                        true);
    R[i].st.batched = 1;
    maxit = std::max(maxit, cs[i]->prm.krylov_maxit);
    if (res[i] >= 0) {
      live[i] = 1;
      ++remaining;
      state[i] = R[i].phase == PH_PCG ? LS_WAIT : LS_RUN;
    }
  }
  auto drop = [&](int i, fde_status s2) {
    res[i] = s2;
    live[i] = 0;
    --remaining;
  };
  // Iterations of the next chunk: up to the first predicted convergence among
  // the members (each x-step usually needs about as many iterations as the
  // previous one), so that finished instances leave the plan soon after.
  auto next_chunk = [&](const std::vector<int>& members, int done_iters) {
    int lo = INT_MAX;
    for (int i : members) lo = std::min(lo, R[i].predict - done_iters);
    return std::max(kGraphIters, ((lo + kGraphIters - 1) / kGraphIters) * kGraphIters);
  };
  bool in_flight = false, full = false;
  int enqueued = 0;
  while (remaining > 0 && st == FDE_OK) {
    bool progress = false;
    if (!in_flight) {
      std::vector<int> members;
      bool all_wait = true;
      for (int i = 0; i < n; ++i) {
        if (!live[i]) continue;
        if (state[i] == LS_WAIT) members.push_back(i);
        else all_wait = false;
      }
      if (all_wait && !members.empty()) {
        for (int i : members) {
          hipError_t e = hipEventRecord(join[i], cs[i]->stream);
          if (e == hipSuccess) e = hipStreamWaitEvent(ls, join[i], 0);
          if (e != hipSuccess) st = (fde_status)fail(FDE_EHIP, std::string("lockstep join: ") + hipGetErrorString(e));
          state[i] = LS_BATCH;
        }
        full = (int)members.size() == n;
        if (!full && st == FDE_OK) st = batch_subset(&bp, cs, members, ls);
        enqueued = 0;
        const int chunk = next_chunk(members, 0);
        if (st == FDE_OK) st = batch_chunk(&bp, full ? bp.full : bp.sub, full, chunk, ls);
        enqueued = chunk;
        in_flight = true;
        progress = true;
      }
    } else {
      const hipError_t q = hipEventQuery(bp.ev);
      if (q == hipSuccess) {
        progress = true;
        const BatchPlan& pl = full ? bp.full : bp.sub;
        std::vector<int> done, still;
        for (size_t k = 0; k < pl.members.size(); ++k) (bp.h_flags[k] ? done : still).push_back(pl.members[k]);
        // the finished instances go on behind the chunk (their own streams wait for it)
        for (int i : done) {
          state[i] = LS_RUN;
          const hipError_t e = hipStreamWaitEvent(cs[i]->stream, bp.ev, 0);
          const fde_status s2 = e != hipSuccess ? (fde_status)fail(FDE_EHIP, std::string("lockstep: ") +
                                                                                   hipGetErrorString(e))
                                                : post_readback(cs[i]);
          if (s2 != FDE_OK) drop(i, s2);
        }
        if (still.empty()) {
          in_flight = false;
        } else if (enqueued > maxit + kGraphIters) {
          // every instance stops by its own iteration limit; this is a guard only
          st = (fde_status)fail(FDE_EHIP, "batched PCG: done flags not set");
        } else {
          if (!done.empty()) {
            full = false;
            st = batch_subset(&bp, cs, still, ls);
          }
          const int chunk = next_chunk(still, enqueued);
          if (st == FDE_OK) st = batch_chunk(&bp, full ? bp.full : bp.sub, full, chunk, ls);
          enqueued += chunk;
        }
      } else if (q != hipErrorNotReady) {
        st = (fde_status)fail(FDE_EHIP, std::string("lockstep batch: ") + hipGetErrorString(q));
      }
    }
    for (int i = 0; i < n && st == FDE_OK; ++i) {
      if (!live[i] || state[i] != LS_RUN) continue;
      const int r = readback_ready(cs[i]);
      if (r == 0) continue;
      progress = true;
      const fde_status s2 = r < 0 ? FDE_EHIP : admm_advance(cs[i], &R[i]);
      if (s2 < 0 || R[i].phase == PH_DONE) drop(i, s2 < 0 ? s2 : R[i].status);
      else if (R[i].phase == PH_PCG) state[i] = LS_WAIT;
    }
    if (!progress) std::this_thread::yield();
  }
  cleanup();
  return st;
}
}  // namespace

extern "C" {

fde_status fde_batch_solve(fde_batch* b, int concurrent, const double* const* yhat, const double* const* g,
                           double* const* y, double* const* u, double* const* zy, double* const* zu, double* const* p,
                           double* const* wy, double* const* wu, fde_admm_stats* stats, int32_t* status) {
  if (!b || !yhat || !y || !u || !zy || !zu || !p || !wy || !wu)
    return (fde_status)fail(FDE_EINVAL, "fde_batch_solve: null argument");
  const int n = (int)b->ctx.size();
  std::vector<fde_status> res(n, FDE_OK);
  if (concurrent == 2) {
    std::vector<AdmmRun> R(n);
    const fde_status ls = batch_lockstep(b, yhat, g, y, u, zy, zu, p, wy, wu, R, res);
    if (ls == FDE_OK) {
      for (hipStream_t s : b->streams) (void)hipStreamSynchronize(s);
      fde_status worst = FDE_OK;
      for (int i = 0; i < n; ++i) {
        if (stats) stats[i] = R[i].st;
        if (status) status[i] = res[i];
        if (res[i] < 0 && worst >= 0) worst = res[i];
        if (res[i] == FDE_ENOTCONV && worst == FDE_OK) worst = FDE_ENOTCONV;
      }
      return worst;
    }
    if (ls != FDE_EINVAL) return ls;
    concurrent = 1;  // no batched form for these instances: the concurrent mode
  }
  if (!concurrent) {
    for (int i = 0; i < n; ++i) {
      fde_admm_stats st{};
      res[i] = fde_admm_solve(b->ctx[i], yhat[i], g ? g[i] : nullptr, y[i], u[i], zy[i], zu[i], p[i], wy[i], wu[i],
                              &st);
      if (stats) stats[i] = st;
    }
  } else {
    std::vector<AdmmRun> R(n);
    std::vector<char> live(n, 0);
    int remaining = 0;
    for (int i = 0; i < n; ++i) {
      res[i] = admm_begin(b->ctx[i], &R[i], yhat[i], g ? g[i] : nullptr, y[i], u[i], zy[i], zu[i], p[i], wy[i], wu[i]);
      if (res[i] >= 0) {
        live[i] = 1;
        ++remaining;
      }
    }
    while (remaining > 0) {
      bool progress = false;
      for (int i = 0; i < n; ++i) {
        if (!live[i]) continue;
        const int r = readback_ready(b->ctx[i]);
        if (r == 0) continue;
        progress = true;
        fde_status st = (r < 0) ? FDE_EHIP : admm_advance(b->ctx[i], &R[i]);
        if (st < 0 || R[i].phase == PH_DONE) {
          res[i] = st < 0 ? st : R[i].status;
          live[i] = 0;
          --remaining;
        }
      }
      if (!progress) std::this_thread::yield();
    }
    for (int i = 0; i < n; ++i)
      if (stats) stats[i] = R[i].st;
  }
  for (hipStream_t s : b->streams) (void)hipStreamSynchronize(s);
  fde_status worst = FDE_OK;
  for (int i = 0; i < n; ++i) {
    if (status) status[i] = res[i];
    if (res[i] < 0 && worst >= 0) worst = res[i];
    if (res[i] == FDE_ENOTCONV && worst == FDE_OK) worst = FDE_ENOTCONV;
  }
  return worst;
}

fde_status fde_grad(fde_ctx* ctx, const double* yhat, const double* y, const double* p, const double* wy,
                    int adjoint_solve, double* dyhat, double* dab, double* lambda_out) {
  using namespace fde;
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  if (!yhat || !y || !p || !dab) return (fde_status)fail(FDE_EINVAL, "fde_grad: null argument");
  CHECK_ALIGNED("fde_grad", yhat, y, p, wy, dyhat, lambda_out);
  fde_ctx* c = ctx;
  double* lam = lambda_out ? lambda_out : c->z;
  if (adjoint_solve) {
    if (!wy) return (fde_status)fail(FDE_EINVAL, "fde_grad: the adjoint solve needs wy");
    const fde_status st = adjoint_solve_impl(c, yhat, y, wy, lam);
    if (st < 0) return st;
    HIP_TRY(launch_grad_fields(c->N, c->nx * c->ny, c->wts, y, yhat, p, c->su.psi, dyhat, nullptr, c->stream));
  } else {
    HIP_TRY(launch_grad_fields(c->N, c->nx * c->ny, c->wts, y, yhat, p, c->su.psi, dyhat, lam, c->stream));
  }
  // dJ/dalpha = -lambda^T (dL_x/dalpha) y ; dJ/dbeta = -lambda^T (dL_y/dbeta) y
  fde::LinePassArgs a = line_args(c);
  a.in = y;
  a.out = c->fa;
  a.L = c->su.x.L;
  a.tw = c->twx_emb;
  a.lamA = c->dxA;
  a.lamB = c->dxB;
  a.s_time = 0.0;
  a.s_sp = 1.0;
  HIP_TRY(launch_xpass(a, false, c->var, c->stream, nullptr));
  fde::LinePassArgs b = line_args(c);
  b.in = y;
  b.out = c->fb;
  b.L = c->su.y.L;
  b.tw = c->twy_emb;
  b.lamA = c->dyA;
  b.lamB = c->dyB;
  b.s_sp = 1.0;
  b.tile = c->tile_line_y;
  HIP_TRY(launch_ypass(b, false, c->var, c->stream, nullptr));
  double out[2];
  const double* fld[2] = {c->fa, c->fb};
  for (int i = 0; i < 2; ++i) {
    int nb = 0;
    HIP_TRY(launch_axpy_dot(VEC_DOT, c->N, lam, fld[i], nullptr, c->scal, c->part_pq, nullptr, c->stream, &nb));
    HIP_TRY(launch_pcg_scalar(FIN_DOT, c->part_pq, nb, c->scal, c->ints, c->stream));
    const fde_status ss = sync_scalars(c);
    if (ss != FDE_OK) return ss;
    out[i] = -c->h_scal[kDot];
  }
  dab[0] = out[0];
  dab[1] = out[1];
  return FDE_OK;
}

}  // extern "C"

namespace {
// process-wide cache of tuned tile variants, keyed by the shape of the problem
std::mutex g_tune_mu;
std::map<std::string, std::array<int, 3>> g_tune;
bool g_tune_loaded = false;

std::string tune_key(fde_ctx* c) {
  std::ostringstream k;
  k << "nx=" << c->nx << ",ny=" << c->ny << ",nt=" << c->nt << ",var=" << (int)c->var << ",fp32=" << (int)c->fp32;
  return k.str();
}

void tune_db_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("FDE_TUNE_DB");
  if (!path) return;
  std::ifstream f(path);
  std::string key;
  std::array<int, 3> v{};
  while (f >> key >> v[0] >> v[1] >> v[2]) g_tune[key] = v;
}

void tune_db_append(const std::string& key, const std::array<int, 3>& v) {
  const char* path = std::getenv("FDE_TUNE_DB");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << v[0] << " " << v[1] << " " << v[2] << "\n";
}

// mean microseconds of `reps` back-to-back launches between two events
template <typename F>
hipError_t time_launches(fde_ctx* c, int reps, F&& launch, double* us) {
  hipError_t e = launch();
  if (e != hipSuccess) return e;
  hipEvent_t e0, e1;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
  if ((e = hipEventCreate(&e1)) != hipSuccess) return e;
  (void)hipEventRecord(e0, c->stream);
  for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch();
  (void)hipEventRecord(e1, c->stream);
  (void)hipEventSynchronize(e1);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *us = 1000.0 * ms / reps;
  return e;
}
// Algorithmic bytes of one launch of PCG pass `which` (every field it reads or
// writes counted once; the half spectrum in the preconditioner's precision)
double pass_bytes(fde_ctx* c, int which) {
  const double f8 = 8.0 * (double)c->N;
  const double sb = (double)c->H * c->ny * c->nt * (c->fp32 ? 8 : 16);
  switch (which) {
    case 0: case 2: return 2 * f8;     // read v, write out
    case 1: return 3 * f8;             // read v, acc; write out
    case 3: return 4 * f8;             // read v, acc, extra (= the dot operand); write out
    case 4: return 6 * f8 + sb;        // read r, q, x, p; write r, x, spectrum
    case 5: case 6: case 7: return 2 * sb;
    case 8: return 2 * f8 + sb;        // read spectrum, p; write p
    default: return 0;
  }
}

}  // namespace

extern "C" {

fde_status fde_autotune(fde_ctx* ctx, int32_t* choices) {
  using namespace fde;
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  fde_ctx* c = ctx;
  const std::string key = tune_key(c);
  std::array<int, 3> best{0, 0, 0};
  bool cached = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_db_load();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      best = it->second;
      cached = true;
    }
  }
  if (!cached) {
    const size_t N = (size_t)c->N;
    double* fields[] = {c->fa, c->fw, c->fb, c->q, c->pk};
    for (double* f : fields) HIP_TRY(hipMemsetAsync(f, 0, N * sizeof(double), c->stream));
    const size_t sb = (size_t)c->H * c->ny * c->nt * (c->fp32 ? 8 : 16);
    HIP_TRY(hipMemsetAsync(c->spec, 0, sb, c->stream));
    const double psi = c->su.psi;
    const int reps = 10;
    double t_best[3] = {1e30, 1e30, 1e30};
    for (int v = 0; v < 3; ++v) {
      double us = 0;
      // the two y-passes of the S apply
      c->tile_line_y = v;
      HIP_TRY(time_launches(c, reps, [&]() -> hipError_t {
        hipError_t e = ypass(c, c->pk, c->fa, c->fw, false, -psi, c->invMp, nullptr, nullptr, nullptr, nullptr,
                             nullptr, nullptr);
        if (e != hipSuccess) return e;
        return ypass(c, c->fw, c->fb, c->q, true, -psi, nullptr, c->pk, c->My, c->pk, c->part_pq, nullptr, nullptr);
      }, &us));
      if (us < t_best[0]) { t_best[0] = us; best[0] = v; }
      // preconditioner y and t passes
      c->tile_pre_y = v;
      c->tile_pre_t = v;
      PrecondArgs a = pre_args(c, c->r, c->z);
      a.rzs_partial = c->part_rz;  // the t-pass as in PCG, with its (r, z) partials
      HIP_TRY(time_launches(c, reps, [&]() { return launch_precond_stage(a, c->fp32, 12, c->stream, nullptr, nullptr); },
                            &us));
      if (us < t_best[1]) { t_best[1] = us; best[1] = v; }
      HIP_TRY(time_launches(c, reps, [&]() { return launch_precond_stage(a, c->fp32, 13, c->stream, nullptr, nullptr); },
                            &us));
      if (us < t_best[2]) { t_best[2] = us; best[2] = v; }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    tune_db_append(key, best);
  }
  c->tile_line_y = best[0];
  c->tile_pre_y = best[1];
  c->tile_pre_t = best[2];
  drop_pcg_graph(c);  // the captured iteration used the previous tiles
  if (choices) {
    choices[0] = ypass_tile_width(c->su.y.L, best[0]);
    choices[1] = best[1];
    choices[2] = best[2];
  }
  return FDE_OK;
}

// Mean duration of pass `which`: `reps` launches back to back between two
// HIP events on the context stream (the event overhead is spread over the
// launches).  The field passes alternate between two disjoint sets of
// workspace fields, so that a launch finds its inputs about as warm in the
// last-level cache as inside an iteration (at the headline size the two sets
// together are about the cache size) rather than left by the launch before;
// the spectrum passes work in place on the half spectrum, as in the solve.
fde_status fde_time_pass(fde_ctx* ctx, int which, int reps, double* us, double* bytes) {
  using namespace fde;
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  if (which < 0 || which > 8 || reps <= 0) return (fde_status)fail(FDE_EINVAL, "fde_time_pass: bad pass or reps");
  if (ctx->frac_t) return (fde_status)fail(FDE_EINVAL, "fde_time_pass: the pass list is that of alpha_t = 1");
  fde_ctx* c = ctx;
  const size_t N = (size_t)c->N;
  const size_t sb = (size_t)c->H * c->ny * c->nt * (c->fp32 ? 8 : 16);
  double* sets[2][4] = {{c->pk, c->fa, c->fw, c->fb}, {c->r, c->z, c->bvec, c->ar}};
  for (auto& set : sets)
    for (double* f : set) HIP_TRY(hipMemsetAsync(f, 0, N * sizeof(double), c->stream));
  HIP_TRY(hipMemsetAsync(c->q, 0, N * sizeof(double), c->stream));
  HIP_TRY(hipMemsetAsync(c->spec, 0, sb, c->stream));
  HIP_TRY(hipMemsetAsync(c->ints, 0, sizeof(int) * kNumInts, c->stream));
  // The passes 4 and 5 run with their fused reductions as in the solve: the
  // step length from the (p, q) partials of the y-pass of B^T (filled with
  // about 1.0 each, so alpha = 0 / (p, q) = 0) and the convergence test on
  // the (r, r) partials (zero, against a negative tolerance: never met).
  int nbS = 0, nb1 = 0;
  if (which == 4) {
    const int P = ypass_tile_width(c->su.y.L, c->tile_line_y);
    nbS = ((c->nx + 2 * P - 1) / (2 * P)) * c->nt;
    HIP_TRY(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(c->part_pq), 0x3FF00000, 2 * (size_t)nbS,
                              c->stream));
  }
  if (which == 5) {
    PrecondArgs a0 = pre_args(c, c->r, c->z);
    HIP_TRY(launch_precond_stage(a0, c->fp32, 1, c->stream, &nb1, nullptr));
    HIP_TRY(hipMemsetAsync(c->part_rr, 0, sizeof(double) * nb1, c->stream));
  }
  // passes 6 and 7 with the (r, z) partials of the spectrum, as in the solve,
  // and pass 8 writing the direction p = z + beta p
  const int nb3 = precond_t_blocks(pre_args(c, c->r, c->z));
  if (which == 7) HIP_TRY(hipMemsetAsync(c->part_rz, 0, sizeof(double) * nb3, c->stream));
  {
    std::vector<double> h(kNumScalars, 0.0);
    h[kBB] = 1.0;
    h[kTol2] = -1.0;
    h[kRZ] = h[kRZ1] = 1.0;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(c->scal, h.data(), sizeof(double) * kNumScalars, hipMemcpyHostToDevice));
  }
  const double psi = c->su.psi, sti = psi / c->su.ht;
  const double b = pass_bytes(c, which);
  auto launch = [&](int rot) -> hipError_t {
    double* const* f = sets[rot & 1];
    switch (which) {
      case 0: return xpass(c, f[0], f[1], false, sti, -psi, nullptr);
      case 1: return ypass(c, f[0], f[1], f[2], false, -psi, c->invMp, nullptr, nullptr, nullptr, nullptr,
                           nullptr, nullptr);
      case 2: return xpass(c, f[2], f[3], true, sti, -psi, nullptr);
      case 3: return ypass(c, f[2], f[3], f[1], true, -psi, nullptr, f[0], c->My, f[0], c->part_pq, nullptr,
                           nullptr);
      default: {
        PrecondArgs a = pre_args(c, f[0], f[1]);  // r, z
        a.scal_w = c->scal;
        a.ints = c->ints;
        if (which == 4) {
          a.q = f[1];
          a.xvec = f[2];
          a.pvec = f[3];
          a.partial = c->part_rr;
          a.pq_partial = c->part_pq;
          a.pq_n = nbS;
        }
        if (which == 5) {
          a.rr_partial = c->part_rr;
          a.rr_n = nb1;
        }
        if (which == 6 || which == 7) {
          a.rzs_partial = c->part_rz;
          a.rzs_n = nb3;
          a.pdir = 1;
        }
        if (which == 8) a.pdir = 1;
        return launch_precond_stage(a, c->fp32, 10 + (which - 3), c->stream, nullptr, nullptr);
      }
    }
  };
  for (int k = 0; k < 2; ++k) HIP_TRY(launch(k));  // warm
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, c->stream));
  for (int i = 0; i < reps; ++i) HIP_TRY(launch(i));
  HIP_TRY(hipEventRecord(e1, c->stream));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (us) *us = 1000.0 * ms / reps;
  if (bytes) *bytes = b;
  return FDE_OK;
}

fde_status fde_pass_timing(fde_ctx* ctx, int enable) {
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  if (ctx->frac_t) return (fde_status)fail(FDE_EINVAL, "fde_pass_timing: the pass list is that of alpha_t = 1");
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->ptime = enable != 0;
  ctx->pt_used = 0;
  if (ctx->ptime) {
    for (int k = 0; k < fde::kNumPasses; ++k) {
      ctx->pt_us[k] = 0;
      ctx->pt_n[k] = 0;
    }
  }
  return FDE_OK;
}

fde_status fde_pass_stats(fde_ctx* ctx, double* us, int32_t* launches, double* bytes) {
  if (check_ctx(ctx) != FDE_OK) return FDE_EINVAL;
  for (int k = 0; k < fde::kNumPasses; ++k) {
    const int64_t n = ctx->pt_n[k];
    if (us) us[k] = n > 0 ? ctx->pt_us[k] / (double)n : 0.0;
    if (launches) launches[k] = (int32_t)n;
    if (bytes) bytes[k] = pass_bytes(ctx, k);
  }
  return FDE_OK;
}

}  // extern "C"

