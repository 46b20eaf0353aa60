// Internal declarations shared by the host code and the kernel translation units.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/fde.h"

namespace fde {

constexpr int kBlock = 256;        // threads per block of the elementwise / reduction kernels
constexpr int kMaxPartials = 4096;  // partial-sum slots per reduction

// Logical tile of block b (of nb): the hardware hands consecutive blocks to
// the 8 XCDs in turn, each XCD with its own L2; this bijection gives each XCD
// a contiguous run of tiles, so neighbouring tiles that share cache lines or
// DRAM pages run under one L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  constexpr int kXcd = 8;
  const int per = nb / kXcd, rem = nb % kXcd;
  const int x = b % kXcd, k = b / kXcd;
  return x * per + (x < rem ? x : rem) + k;
}

// ---------------------------------------------------------------------------
// In-solve pass timing.  The host may queue pairs of HIP events for the next
// pass launches of its thread; each launch of a line pass or a preconditioner
// pass then takes the next pair, which hipExtLaunchKernel binds to that
// dispatch (start and end of the kernel's own execution).  Without queued
// events the launch is a plain one.
// ---------------------------------------------------------------------------
constexpr int kNumPasses = 9;  // passes of one PCG iteration (implicit Euler)
struct PassEventQueue {
  const hipEvent_t* ev = nullptr;  // n pairs (start, stop)
  int n = 0, next = 0;
};
extern thread_local PassEventQueue t_pass_events;

// 16-byte accesses of two adjacent doubles (fields are 16-byte aligned and nx is even)
__device__ __forceinline__ double2 ld2(const double* p) { return *reinterpret_cast<const double2*>(p); }
__device__ __forceinline__ void st2(double* p, double2 v) { *reinterpret_cast<double2*>(p) = v; }

// ---------------------------------------------------------------------------
// Toeplitz line passes (operator D and D^T)
//
//   x-pass:  out = s_time * (E or E^T) in + s_sp * (L_x or L_x^T) in
//   y-pass:  out_t = oscale[t] * (acc + s_sp * (L_y or L_y^T) in) + escale[t] * extra
//            (+ optional partial sums of dotv * out)
//   t-pass (fractional time order): the y-pass kernel on the field viewed as
//            [nt][nx*ny] with the time-matrix tables, oscale/escale by row
// E is the implicit-Euler time difference (v_t - v_{t-1}) / h_t, E^T uses
// v_{t+1}.  The spatial operators are (c_a/h^a)(diag(d+) G + diag(d-) G^T)
// applied by a 2n circulant embedding; the eigenvalue tables already carry
// c_a/h^a and the 1/(2n) of the inverse transform.
// ---------------------------------------------------------------------------
struct LinePassArgs {
  const double* in;
  double* out;
  int nx, ny, nt;
  int L;  // embedding length of the transformed axis (x-pass: of nx, y-pass: of ny), >= 2n
  // spectral multipliers of the embedding circulants (length 2n, complex)
  const double2* lamA;  // constant coefficients: combined operator; variable: G
  const double2* lamB;  // variable coefficients: G^T (unused otherwise)
  const double2* tw;    // twiddles of length 2n
  const double* dplus;  // (ny, nx) or nullptr for constant coefficients
  const double* dminus;
  double s_time;  // x-pass only: coefficient of the time difference
  double s_sp;    // coefficient of the spatial operator
  // y-pass epilogue
  const double* acc;     // may be nullptr
  const double* oscale;  // per time slice, may be nullptr (= 1)
  const double* extra;   // may be nullptr
  const double* escale;  // per time slice
  const double* dotv;    // may be nullptr: then no partial sums
  double* partial;       // one slot per block
  const int* done;       // early-exit flag (may be nullptr)
  int tile;              // y-pass tile variant (autotuned): 0 widest, 1 half, 2 quarter
  int row_scale;         // y-pass kernel run along t (rows = time levels): oscale and
                         // escale are indexed by the row, not the slice
  int col_coef;          // y-pass: coefficients constant along every y-line; column x
                         // takes d+[x], d-[x] (row 0 of the planes) inside the multiplier
};

// Embedding lengths longer than 2n: for axis lengths whose 2n is not an FFT
// length of the line passes (n = 50, 80, 100, 160), the next one that is.
__host__ __device__ constexpr bool padded_embedding(int L) {
  return L == 128 || L == 192 || L == 256 || L == 384;
}

// launchers (return hipError_t of the launch)
hipError_t launch_xpass(const LinePassArgs& a, bool transpose, bool varcoef, hipStream_t s, int* nblocks);
hipError_t launch_ypass(const LinePassArgs& a, bool transpose, bool varcoef, hipStream_t s, int* nblocks);
int ypass_tile_width(int L, int variant);  // column pairs per block of a variant (0 if unsupported)

// ---------------------------------------------------------------------------
// preconditioner passes: z = S~^{-1} r via a 3-D real FFT
// ---------------------------------------------------------------------------
struct PrecondArgs {
  int nx, ny, nt, H;  // H = nx/2 + 1 complex columns of the half spectrum
  double* r;          // input field (updated in place by the fused x-forward pass)
  double* z;          // output field
  void* spec;         // half spectrum [nt][ny][H], double2 or float2
  const void* twx;    // twiddles (length nx, ny, nt) in the spectrum precision
  const void* twy;
  const void* twt;
  const double2* lam_x;  // T. Chan eigenvalues (FP64 always)
  const double2* lam_y;
  const double2* lam_t;
  double psi, a, inv_mbar, inv_n;  // s = a + |psi (lt - ly - lx)|^2 * inv_mbar; 1/(nx ny nt)
  double match2;                   // + match2 * Re(psi (lt - ly - lx)): the matching form (0: S~)
  int div_mode;  // 0: divide by s (S~^{-1}); 1: multiply by 1/conj(psi (lt - ly - lx)) (C^{-T})
  int tile_y, tile_t;  // column-tile variants of the y and t passes (autotuned)
  // fused PCG pieces
  const double* q;        // x-forward: r -= alpha q (if non-null)
  double* xvec;           // x-forward: x += alpha p
  const double* pvec;
  const double* scal;     // device scalars (alpha at index kAlpha)
  double* partial;        // x-forward: partial sums of r.r (fused mode only)
  double* partial2;       // x-inverse: partial sums of r.z (nullptr: none)
  const int* done;
  // fused PCG scalar steps (nullptr: not fused)
  const double* pq_partial;  // x-forward: alpha = rz / sum(pq_partial[0..pq_n))
  int pq_n;
  const double* rr_partial;  // y-forward: (r, r) = sum(rr_partial[0..rr_n)), convergence test
  int rr_n;
  double* scal_w;            // device scalars written by block 0 (alpha, pq, rr, rz, beta)
  int* ints;                 // device flags written by block 0 (done, iteration count, convergence)
  // (r, z) taken from the spectrum (Parseval), so that the x-inverse pass can
  // write the PCG direction directly:
  double* rzs_partial;  // t-pass (divide by s): per-block partial sums of (r, z) (nullptr: none)
  int rzs_n;            // y-inverse: block 0 sums rzs_partial[0..rzs_n) into (r, z) and beta
  int pdir;             // x-inverse output into z: 0 the preconditioned residual; 1 p = z + beta p
                        // (z is the direction p, updated in place); 2 p = z (the first direction)
  // diagonal scaling Delta S~^{-1} Delta (nullptr: none): Delta at node (x, y, t) is
  // ds_tab[ds_class[t]][y][x]; the x-forward pass scales its FFT input, the x-inverse
  // pass its output
  const double* ds_tab;  // (classes, ny, nx)
  const int* ds_class;   // per time slice
};

// the row of the preconditioner's diagonal scaling for x-line l (t = l / ny, y = l % ny),
// nullptr without scaling; l must be a line of the field
__device__ __forceinline__ const double* precond_scale_row(const PrecondArgs& a, int l) {
  if (!a.ds_tab) return nullptr;
  const int t = l / a.ny;
  return a.ds_tab + ((size_t)a.ds_class[t] * a.ny + (l - t * a.ny)) * a.nx;
}

// ---------------------------------------------------------------------------
// Batched passes.  A pass kernel launched with batch arguments works on many
// independent instances at once: block b of the launch runs block
// b - first[i] (of first[i+1] - first[i]) of instance i, the largest i with
// first[i] <= b, with that instance's own arguments from the table args[i].
// Every instance keeps the block decomposition of its own single launch, so
// its results are bit for bit those of that launch.
// ---------------------------------------------------------------------------
template <typename Args> struct BatchArgs {
  const Args* args;   // [count] per-instance arguments (device)
  const int* first;   // [count + 1] first launch block of each instance (device)
  int count;
};

// Instance of launch block blk, wave-parallel: the active lanes of a wavefront
// test first[base + lane + 1] <= blk for a window of instances at a time (the
// lanes that hold form a prefix, so their count is the offset).  Called at
// kernel entry by every thread of the block.  One load round per 64
// instances, and the instance index stays wave-uniform (scalar), which also
// keeps the argument table's field pointers recognisable as global memory.
template <typename Args>
__device__ __forceinline__ int batch_instance(const BatchArgs<Args>& b, int blk) {
  const int lane = (int)(threadIdx.x & 63);
  const int width = __popcll(__ballot(1));
  int base = 0;
  for (;;) {
    const int k = base + lane + 1;
    const bool le = k < b.count && b.first[k] <= blk;
    const int c = __popcll(__ballot(le));
    if (c < width) return __builtin_amdgcn_readfirstlane(base + c);
    base += width;
  }
}

// A batched instance's arguments as the block's own copy, every field pointer
// marked as global memory: pointers read from the argument table would
// otherwise stay generic (each access through them a flat one) and be read
// again from the table after each store.  The pointers are wave-uniform.
template <typename T>
__device__ __forceinline__ T* as_global(T* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  using G = __attribute__((address_space(1))) T*;
  return (T*)(G)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ LinePassArgs batch_local(const LinePassArgs& s) {
  LinePassArgs a = s;
  a.in = as_global(a.in);
  a.out = as_global(a.out);
  a.lamA = as_global(a.lamA);
  a.lamB = as_global(a.lamB);
  a.tw = as_global(a.tw);
  a.dplus = as_global(a.dplus);
  a.dminus = as_global(a.dminus);
  a.acc = as_global(a.acc);
  a.oscale = as_global(a.oscale);
  a.extra = as_global(a.extra);
  a.escale = as_global(a.escale);
  a.dotv = as_global(a.dotv);
  a.partial = as_global(a.partial);
  a.done = as_global(a.done);
  return a;
}

__device__ __forceinline__ PrecondArgs batch_local(const PrecondArgs& s) {
  PrecondArgs a = s;
  a.r = as_global(a.r);
  a.z = as_global(a.z);
  a.spec = as_global(a.spec);
  a.twx = as_global(a.twx);
  a.twy = as_global(a.twy);
  a.twt = as_global(a.twt);
  a.lam_x = as_global(a.lam_x);
  a.lam_y = as_global(a.lam_y);
  a.lam_t = as_global(a.lam_t);
  a.q = as_global(a.q);
  a.xvec = as_global(a.xvec);
  a.pvec = as_global(a.pvec);
  a.scal = as_global(a.scal);
  a.partial = as_global(a.partial);
  a.partial2 = as_global(a.partial2);
  a.done = as_global(a.done);
  a.pq_partial = as_global(a.pq_partial);
  a.rr_partial = as_global(a.rr_partial);
  a.scal_w = as_global(a.scal_w);
  a.ints = as_global(a.ints);
  a.rzs_partial = as_global(a.rzs_partial);
  a.ds_tab = as_global(a.ds_tab);
  a.ds_class = as_global(a.ds_class);
  return a;
}

// A recorded pass launch (the host records an instance's PCG iteration once,
// then issues the passes of all instances as batched launches).
struct RecordedPass {
  const void* batch_kernel = nullptr;  // the BatchArgs twin of the kernel (null: no batched form)
  int blocks = 0, threads = 0;
  int kind = 0;                        // 0: LinePassArgs, 1: PrecondArgs
  alignas(16) unsigned char args[512];
};
extern thread_local std::vector<RecordedPass>* t_record;

template <typename Arg>
inline void launch_pass(void (*kern)(Arg), void (*batch_kern)(BatchArgs<Arg>), int blocks, int threads,
                        hipStream_t s, const Arg& a) {
  if (t_record) {
    static_assert(sizeof(Arg) <= sizeof(RecordedPass::args), "argument block");
    RecordedPass r;
    r.batch_kernel = reinterpret_cast<const void*>(batch_kern);
    r.blocks = blocks;
    r.threads = threads;
    r.kind = std::is_same<Arg, LinePassArgs>::value ? 0 : 1;
    std::memcpy(r.args, &a, sizeof(Arg));
    t_record->push_back(r);
    return;
  }
  PassEventQueue& q = t_pass_events;
  if (q.next < q.n) {
    const int k = q.next++;
    hipExtLaunchKernelGGL(kern, dim3(blocks), dim3(threads), 0, s, q.ev[2 * k], q.ev[2 * k + 1], 0, a);
  } else {
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), 0, s, a);
  }
}

// stage 0: all five passes; 1: the x-forward pass only; 2: passes 2-5; 11..15: pass 1..5 alone
hipError_t launch_precond_stage(const PrecondArgs& a, bool fp32, int stage, hipStream_t s, int* nb_fwd,
                                int* nb_inv);
// blocks of the t-pass for the context's tile variant: the count of rzs_partial
int precond_t_blocks(const PrecondArgs& a);
inline hipError_t launch_precond(const PrecondArgs& a, bool fp32, hipStream_t s, int* nb_fwd, int* nb_inv) {
  return launch_precond_stage(a, fp32, 0, s, nb_fwd, nb_inv);
}

// ---------------------------------------------------------------------------
// device scalar slots of the Krylov / ADMM state
// ---------------------------------------------------------------------------
enum ScalarSlot {
  kRZ = 0,    // (r, z) of even PCG iterations (0, 2, ...)
  kRZ1,       // (r, z) of odd iterations: the p update reads one slot and writes the other
  kPQ,        // (p, q)
  kAlpha,
  kBeta,
  kRR,        // (r, r)
  kBB,        // (b, b)
  kTol2,      // tol^2
  kResP,      // ADMM residuals
  kResY,
  kResU,
  kDot,       // scratch dot result
  kD0,        // four slots written by launch_dots
  kD1,
  kD2,
  kD3,
  kDual,      // dual infeasibility of the final ADMM iterate
  kNumScalars
};
// kStop: MINRES stop request, raised by its Givens step and turned into kDone
// by the first kernel of the next iteration (the current iteration's update
// of x must still run)
enum IntSlot { kDone = 0, kIter, kMaxit, kConv, kStop, kNumInts };
// slot of (r, z) after iteration `iter` (iteration 0 = the initial residual)
__host__ __device__ __forceinline__ int rz_slot(int iter) { return (iter & 1) ? kRZ1 : kRZ; }

// ---------------------------------------------------------------------------
// MINRES on the merged x-step system (3.8) with the block-diagonal K~ of
// eq. (3.12); a triple is the (y, u, p) blocks of one vector
// ---------------------------------------------------------------------------
struct Triple {
  double *y, *u, *p;
};
// device scalars of the MINRES recurrence (a separate small array)
enum MinresSlot {
  kMG = 0,   // gamma_j: M^{-1}-norm of the current unnormalised Lanczos vector
  kMGold,    // gamma_{j-1}
  kMD,       // delta_j
  kMC, kMCold, kMS, kMSold,  // Givens cosines / sines of the last two rotations
  kMEta,     // eta: signed M^{-1}-norm of the residual
  kMA1, kMA2, kMA3,  // this iteration's rotation coefficients
  kMX,       // step of x along the new direction (c_{j+1} eta_j)
  kMZ,       // 1 / gamma_j (normalises z_j in the direction update)
  kMNb,      // M^{-1}-norm of the right-hand side
  kMTol,
  kMRes,     // current residual norm
  kNumMinres
};
enum MinresVecMode { MR_RESID = 0, MR_LANCZOS, MR_RHS, MR_ZERO };
enum MinresScalarOp { MR_NB = 0, MR_INIT, MR_DELTA, MR_GIVENS };
struct MinresConsts {
  int64_t n;
  int plane;
  double k_u, dr;            // control coupling; delta / rho
  const double* My;          // per time slice
  const double* Mu;
};
// tmp = k_u z.u - (delta/rho) z.p ; q.u = M_u z.u + k_u z.p ; partial (z.u, q.u);
// block 0 also moves the stop request into kDone
hipError_t launch_minres_pre(const MinresConsts& k, Triple z, double* tmp, double* qu, double* partial, int* ints,
                             hipStream_t s, int* nb);
// MR_RESID:   out = b - q           (b passed as v)
// MR_LANCZOS: out = q / g - (delta / g) v - (g / g_old) out   (out holds v_{j-1} on entry)
// MR_RHS:     out unused; the M^{-1} blocks of b (passed as v)
// MR_ZERO:    out = 0 (all three blocks)
// then z.y = out.y / M_y, z.u = out.u / M_u and partial (z.y, out.y) + (z.u, out.u)
hipError_t launch_minres_vec(int mode, const MinresConsts& k, Triple q, Triple v, Triple out, Triple z,
                             const double* ms, double* partial, const int* done, hipStream_t s, int* nb);
// one block: the scalar step `op` from up to three partial arrays
hipError_t launch_minres_scalar(int op, const double* p0, int n0, const double* p1, int n1, const double* p2,
                                int n2, double* ms, int* ints, double tol, int maxit, hipStream_t s);
// w_new = (z / gamma_j - a3 w_old - a2 w) / a1 into w_old ; x += (c_{j+1} eta) w_new
hipError_t launch_minres_update(const MinresConsts& k, Triple z, Triple w_old, Triple w, Triple x, const double* ms,
                                const int* done, hipStream_t s);

// elementwise / reduction kernels
// (alpha, the convergence test and beta run fused inside the passes that need them;
// FIN_CONV is the stand-alone convergence test used when the fused form's
// redundant per-block sums would cost more than one small launch)
enum PcgOp { FIN_INIT = 0, FIN_DOT, FIN_CONV };
enum VecOp {
  VEC_RESID = 0,    // c = a - b ; partials (c,c) and (a,a)
  VEC_DOT,          // partial (a, b)
  VEC_ZERO_IF_BB0   // c = 0 when scal[kBB] == 0
};
// FIN_INIT also stores tol2 and maxit in the device slots
hipError_t launch_pcg_scalar(int op, const double* partial, int n, double* scal, int* ints, hipStream_t s,
                             double tol2 = 0.0, int maxit = 0);
hipError_t launch_axpy_dot(int op, int64_t n, const double* a, const double* b, double* c,
                           const double* scal, double* partial, const int* done, hipStream_t s,
                           int* nblocks);
// p = z + beta p with beta = (r, z)_k / (r, z)_{k-1}, (r, z)_k summed inside
// from the partials of the z pass (every block in the same order)

struct AdmmConsts {
  int64_t n;
  int plane;  // nx * ny
  int nt;
  double rho, delta, e_y, e_u, k_u, ya, yb, ua, ub;
  int prox;              // Algorithm 2: proximal terms rho R (y^j, u^j) in the right-hand side
  double cy, cu, gamma;  // R_y = cy - wts[t], R_u = cu - gamma wts[t]
  const double* wts;  // per time slice J1 diagonal
  const double* Mu;   // per time slice
  const double* Mp;
  const double* invMp;
  const double *lya, *lyb, *lua, *lub;  // per-point bounds (null: the scalars above)
};
struct AdmmFields {
  const double* yhat;
  const double* g;  // may be null
  double *y, *u, *zy, *zu, *p, *wy, *wu;
  double *r, *Ru, *v, *c, *By;
  double* byp;      // may be null: receives M_p^{-1} B y for the next x-step's initial residual
  double* partial;  // 3 * blocks
};
hipError_t launch_admm_rhs(const AdmmConsts& k, const AdmmFields& f, double psi, hipStream_t s);
// next_rhs: also write the next iteration's right-hand side pieces (Ru, r, v, c)
hipError_t launch_admm_update(const AdmmConsts& k, const AdmmFields& f, double psi, hipStream_t s,
                              int* nblocks, bool next_rhs);
hipError_t launch_max3_finalize(const double* partial, int nblocks, double* scal, hipStream_t s);
// per-point bound check: partial[3 b + c] = 1 where a lower bound exceeds its upper one or
// either is NaN (c = 0: y pair, c = 1: u pair; null arrays take the scalars), else 0
hipError_t launch_bounds_check(int64_t n, const double* ya, const double* yb, const double* ua, const double* ub,
                               double sya, double syb, double sua, double sub, double* partial, hipStream_t s,
                               int* nblocks);
// dual infeasibility max(|J1 (y - yhat) + btp + e_y wy|, |gamma J1 u + k_u p + e_u wu|) over the
// grid into scal[kDual]; btp = B^T p.  `partial` holds one slot per block.
hipError_t launch_dual_inf(const AdmmConsts& k, const AdmmFields& f, double gamma, const double* btp,
                           double* partial, double* scal, hipStream_t s);
// up to four dot products (a[j], b[j]) in one pass; sums land in scal[kD0 + j]
hipError_t launch_dots(int64_t n, int count, const double* const* a, const double* const* b, double* partial,
                       double* scal, hipStream_t s);
// out = c0 x0 + c1 x1 + c2 x2 (null inputs skipped); out may alias an input
hipError_t launch_lincomb(int64_t n, double c0, const double* x0, double c1, const double* x1, double c2,
                          const double* x2, double* out, hipStream_t s);
// f = -J1 (y - yhat) - wy
hipError_t launch_adjoint_rhs(int64_t n, int plane, const double* wts, const double* y, const double* yhat,
                              const double* wy, double* f, hipStream_t s);
// partial sums of 1/2 J1 (y - yhat)^2 + gamma/2 J1 u^2
hipError_t launch_objective(int64_t n, int plane, const double* wts, double gamma, const double* y,
                            const double* yhat, const double* u, double* partial, hipStream_t s, int* nb);
// out[i] = ints[i][kDone] for the count instances of a batch
hipError_t launch_gather_done(const int* const* ints, int count, int* out, hipStream_t s);
// gradient pieces: dyhat = -J1 (y - yhat), lam = psi p
hipError_t launch_grad_fields(int64_t n, int plane, const double* wts, const double* y, const double* yhat,
                              const double* p, double psi, double* dyhat, double* lam, hipStream_t s);

}  // namespace fde
