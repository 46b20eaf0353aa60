// Host-side setup (see host_setup.hpp).
#include "host_setup.hpp"

#include <algorithm>
#include <functional>
#include <thread>

#include <cmath>
#include <cstdio>

namespace fde {
namespace host {

namespace {
const double kPi = 3.14159265358979323846264338327950288;

bool finite(double v) { return std::isfinite(v); }

std::string fmt(const char* f, double a) {
  char buf[256];
  std::snprintf(buf, sizeof buf, f, a);
  return buf;
}
}  // namespace

bool length_supported(int n) {
  // n = 2^a 3^b with b <= 1 and 4 <= n <= 1024 (FFT radices 2/4/8 and one 3),
  // or one of the lengths with a factor 5 of the paper's grids (50, 80, 100)
  // and 160
  if (n == 50 || n == 80 || n == 100 || n == 160) return true;
  if (n < 4 || n > 1024) return false;
  int m = n;
  if (m % 3 == 0) m /= 3;
  while (m % 2 == 0) m /= 2;
  return m == 1;
}

int embed_length(int n) {
  // the circulant embedding needs L >= 2n - 1; the line passes transform
  // lengths 2^a 3^b (b <= 1), so the lengths with a factor 5 take the next one
  switch (n) {
    case 50: return 128;
    case 80: return 192;
    case 100: return 256;
    case 160: return 384;
    default: return 2 * n;
  }
}

int validate_params(const fde_admm_params* q, std::string* msg) {
  if (!q) { *msg = "params is NULL"; return FDE_EINVAL; }
  if (!(q->gamma > 0) || !finite(q->gamma)) { *msg = "gamma must be finite and > 0"; return FDE_EINVAL; }
  if (!(q->delta > 0) || !finite(q->delta)) { *msg = "delta must be finite and > 0"; return FDE_EINVAL; }
  const double rmax = 0.5 * (1.0 + std::sqrt(5.0));
  if (!(q->rho > 0 && q->rho < rmax)) { *msg = "rho must lie in (0, (1+sqrt5)/2)"; return FDE_EINVAL; }
  if (std::isnan(q->ya) || std::isnan(q->yb) || std::isnan(q->ua) || std::isnan(q->ub)) {
    *msg = "bounds must not be NaN";
    return FDE_EINVAL;
  }
  if (q->ya > q->yb || q->ua > q->ub) { *msg = "lower bound exceeds upper bound"; return FDE_EINVAL; }
  if (q->ya == INFINITY || q->yb == -INFINITY || q->ua == INFINITY || q->ub == -INFINITY) {
    *msg = "empty box (infinite bound on the wrong side)";
    return FDE_EINVAL;
  }
  if (!(q->krylov_tol >= 0) || !finite(q->krylov_tol)) { *msg = "krylov_tol must be >= 0"; return FDE_EINVAL; }
  if (q->krylov_maxit <= 0) { *msg = "krylov_maxit must be > 0"; return FDE_EINVAL; }
  if (q->pcg_cold_start != 0 && q->pcg_cold_start != 1) { *msg = "pcg_cold_start must be 0 or 1"; return FDE_EINVAL; }
  if (q->tol_mode != 0 && q->tol_mode != 1) { *msg = "tol_mode must be 0 or 1"; return FDE_EINVAL; }
  if (q->prox != 0 && q->prox != 1) { *msg = "prox must be 0 or 1"; return FDE_EINVAL; }
  if (q->precond_kind < 0 || q->precond_kind > 2) { *msg = "precond_kind must be 0, 1 or 2"; return FDE_EINVAL; }
  if (q->krylov_solver != 0 && q->krylov_solver != 1) { *msg = "krylov_solver must be 0 or 1"; return FDE_EINVAL; }
  if (q->precond_kind == 2 && q->krylov_solver != 0) {
    *msg = "precond_kind 2 (diagonally scaled S~) is a preconditioner of the PCG x-step (krylov_solver 0)";
    return FDE_EINVAL;
  }
  if (q->prox) {
    // Algorithm 2 takes its step in (0, 1]; R_y, R_u must not be indefinite
    if (!(q->rho <= 1.0)) { *msg = "prox = 1 (Algorithm 2) needs rho in (0, 1]"; return FDE_EINVAL; }
    if (!finite(q->prox_cy) || !(q->prox_cy == 0.0 || q->prox_cy >= 1.0)) {
      *msg = "prox_cy must be 0 or >= max diag J1 = 1";
      return FDE_EINVAL;
    }
    if (!finite(q->prox_cu) || !(q->prox_cu == 0.0 || q->prox_cu >= q->gamma)) {
      *msg = "prox_cu must be 0 or >= gamma";
      return FDE_EINVAL;
    }
  }
  if (!(q->admm_tol >= 0) || !finite(q->admm_tol)) { *msg = "admm_tol must be >= 0"; return FDE_EINVAL; }
  if (q->admm_maxit <= 0) { *msg = "admm_maxit must be > 0"; return FDE_EINVAL; }
  return FDE_OK;
}

int validate(const fde_problem* p, const fde_admm_params* q, std::string* msg) {
  if (!p) { *msg = "problem is NULL"; return FDE_EINVAL; }
  const int dims[3] = {p->nx, p->ny, p->nt};
  const char* names[3] = {"nx", "ny", "nt"};
  for (int i = 0; i < 3; ++i) {
    if (!length_supported(dims[i])) {
      *msg = std::string(names[i]) + "=" + std::to_string(dims[i]) +
             " unsupported: need 2^a*3^b (b <= 1) between 4 and 1024, or 50, 80, 100, 160";
      return FDE_EINVAL;
    }
  }
  if (!(p->T > 0) || !finite(p->T)) { *msg = "T must be finite and > 0"; return FDE_EINVAL; }
  if (!(p->alpha > 1.0 && p->alpha <= 2.0)) { *msg = fmt("alpha=%g outside (1, 2]", p->alpha); return FDE_EINVAL; }
  if (!(p->beta > 1.0 && p->beta <= 2.0)) { *msg = fmt("beta=%g outside (1, 2]", p->beta); return FDE_EINVAL; }
  if (!(p->alpha_t == 0.0 || (p->alpha_t > 0.0 && p->alpha_t <= 1.0))) {
    *msg = fmt("alpha_t=%g outside (0, 1]", p->alpha_t);
    return FDE_EINVAL;
  }
  if (p->ctrl_sign != 1.0 && p->ctrl_sign != -1.0) { *msg = "ctrl_sign must be +1 or -1"; return FDE_EINVAL; }
  if (p->psi_scaling < 0 || p->psi_scaling > 2) { *msg = "psi_scaling must be 0, 1 or 2"; return FDE_EINVAL; }
  if (p->obj_weights != 0 && p->obj_weights != 1) { *msg = "obj_weights must be 0 or 1"; return FDE_EINVAL; }
  if (p->precond_fp32 != 0 && p->precond_fp32 != 1) { *msg = "precond_fp32 must be 0 or 1"; return FDE_EINVAL; }
  const size_t plane = (size_t)p->nx * p->ny;
  const double* fields[2] = {p->dplus, p->dminus};
  for (int f = 0; f < 2; ++f) {
    if (!fields[f]) continue;
    for (size_t i = 0; i < plane; ++i) {
      if (!(fields[f][i] >= 0) || !finite(fields[f][i])) {
        *msg = "coefficient fields must be finite and >= 0";
        return FDE_EINVAL;
      }
    }
  }
  return validate_params(q, msg);
}

std::vector<double> grunwald_weights(double a, int n) {
  // g_0 = 1, g_k = (1 - (a+1)/k) g_{k-1} (Sec. 4, recurrence under eq. (4.4))
  std::vector<double> g(n + 1);
  g[0] = 1.0;
  for (int k = 1; k <= n; ++k) g[k] = (1.0 - (a + 1.0) / k) * g[k - 1];
  return g;
}

std::vector<double> grunwald_weight_derivs(double a, int n) {
  // differentiate the recurrence in a: g'_0 = 0, g'_k = (1-(a+1)/k) g'_{k-1} - g_{k-1}/k
  std::vector<double> g = grunwald_weights(a, n);
  std::vector<double> d(n + 1);
  d[0] = 0.0;
  for (int k = 1; k <= n; ++k) d[k] = (1.0 - (a + 1.0) / k) * d[k - 1] - g[k - 1] / k;
  return d;
}

std::vector<cd> twiddles(int L) {
  std::vector<cd> w(L);
  for (int m = 0; m < L; ++m) {
    const long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)L;
    w[m] = cd((double)std::cos(ang), (double)std::sin(ang));
  }
  return w;
}

std::vector<cd> dft(const std::vector<cd>& c) {
  // direct O(L^2) sum with the phase index reduced mod L, long double accumulation
  const int L = (int)c.size();
  std::vector<long double> cr(L), si(L);
  for (int m = 0; m < L; ++m) {
    const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)L;
    cr[m] = std::cos(ang);
    si[m] = std::sin(ang);
  }
  std::vector<cd> out(L);
  for (int k = 0; k < L; ++k) {
    long double re = 0, im = 0;
    for (int m = 0; m < L; ++m) {
      const int idx = (int)(((long long)k * m) % L);
      // exp(-i ang) = cos - i sin
      const long double a = c[m].real(), b = c[m].imag();
      re += a * cr[idx] + b * si[idx];
      im += b * cr[idx] - a * si[idx];
    }
    out[k] = cd((double)re, (double)im);
  }
  return out;
}

std::vector<cd> tchan_eigs(const std::vector<double>& t_pos, const std::vector<double>& t_neg) {
  // T. Chan optimal circulant (closed form under eq. (5.1)):
  //   c_i = ((n - i) t_i + i t_{i-n}) / n, eigenvalues = DFT(c) (Thm 2.2)
  // t_pos[k] = t_k (k = 0..n-1), t_neg[k] = t_{-k} (k = 1..n-1; t_neg[0] unused)
  const int n = (int)t_pos.size();
  std::vector<cd> c(n);
  for (int i = 0; i < n; ++i) {
    const double ti = t_pos[i];
    const double tin = (i > 0) ? t_neg[n - i] : 0.0;
    c[i] = cd(((n - i) * ti + i * tin) / n, 0.0);
  }
  return dft(c);
}

namespace {

// Toeplitz entries of the mean-coefficient operator c (dp G + dm G^T):
// G[i][j] = g_{i-j+1}: t_k = g_{k+1} for k >= -1; G^T: t_k = g_{1-k} for k <= 1
void mean_operator_entries(const std::vector<double>& g, double c, double dp, double dm, int n,
                           std::vector<double>* tp, std::vector<double>* tn) {
  tp->assign(n, 0.0);
  tn->assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double v = dp * g[k + 1];
    if (k <= 1) v += dm * g[1 - k];
    (*tp)[k] = c * v;
  }
  for (int k = 1; k < n; ++k) {
    double v = dm * g[k + 1];
    if (k == 1) v += dp * g[0];
    (*tn)[k] = c * v;
  }
}

void build_axis(int n, double h, double order, double dp, double dm, bool var, AxisTables* ax) {
  ax->n = n;
  ax->h = h;
  ax->order = order;
  ax->c = -1.0 / (2.0 * std::cos(order * kPi / 2.0)) / std::pow(h, order);  // eq. (4.7)
  ax->g = grunwald_weights(order, n);
  ax->dg = grunwald_weight_derivs(order, n);
  const int L = embed_length(n);
  ax->L = L;
  // first column of the L-point circulant embedding of G: (g_1, .., g_n, 0, .., 0, g_0)
  auto embed = [&](const std::vector<double>& gg) {
    std::vector<cd> col(L, cd(0, 0));
    for (int k = 0; k < n; ++k) col[k] = gg[k + 1];
    col[L - 1] = gg[0];
    return dft(col);
  };
  const double s = ax->c / L;
  std::vector<cd> lg = embed(ax->g);
  std::vector<cd> ldg = embed(ax->dg);
  ax->lamG.resize(L);
  ax->lamGT.resize(L);
  ax->lamFwd.resize(L);
  ax->lamTr.resize(L);
  ax->dopA.resize(L);
  ax->dopB.resize(L);
  // dL/da = kappa L + (c_a/h^a)(d+ G' + d- G'^T), kappa = (pi/2) tan(a pi/2) - ln h
  const double kappa = (kPi / 2.0) * std::tan(order * kPi / 2.0) - std::log(h);
  for (int k = 0; k < L; ++k) {
    // G^T embeds as the reversed column: its eigenvalues are the conjugates
    ax->lamG[k] = s * lg[k];
    ax->lamGT[k] = s * std::conj(lg[k]);
    ax->lamFwd[k] = s * (dp * lg[k] + dm * std::conj(lg[k]));
    ax->lamTr[k] = s * (dp * std::conj(lg[k]) + dm * lg[k]);
    if (var) {
      ax->dopA[k] = s * (kappa * lg[k] + ldg[k]);
      ax->dopB[k] = s * (kappa * std::conj(lg[k]) + std::conj(ldg[k]));
    } else {
      ax->dopA[k] = s * (kappa * (dp * lg[k] + dm * std::conj(lg[k])) + dp * ldg[k] + dm * std::conj(ldg[k]));
      ax->dopB[k] = cd(0, 0);
    }
  }
  std::vector<double> tp, tn;
  mean_operator_entries(ax->g, ax->c, dp, dm, n, &tp, &tn);
  ax->tchan = tchan_eigs(tp, tn);
  ax->tw_emb = twiddles(L);
  ax->tw = twiddles(n);
}

}  // namespace

void set_admm_scalings(const fde_admm_params* q, Setup* s) {
  const int nt = s->nt;
  s->wts.assign(nt, 1.0);
  if (s->obj_weights == 1) s->wts[nt - 1] = 0.5;  // trapezoidal, eq. (4.10)
  s->My.resize(nt);
  s->Mu.resize(nt);
  s->Mp.resize(nt);
  s->invMp.resize(nt);
  // Algorithm 2 (Sec. 3.3.2): J1 + R_y = cy I and J2 + R_u = cu I replace J1, J2
  // in the x-step's diagonal blocks; max diag J1 = 1 for both weightings
  s->cy = s->cu = 0.0;
  if (q->prox) {
    s->cy = q->prox_cy > 0 ? q->prox_cy : 1.0;
    s->cu = q->prox_cu > 0 ? q->prox_cu : q->gamma;
  }
  for (int k = 0; k < nt; ++k) {
    const double jy = q->prox ? s->cy : s->wts[k];
    const double ju = q->prox ? s->cu : q->gamma * s->wts[k];
    s->My[k] = q->rho * (jy + s->e_y * s->e_y / q->delta);
    s->Mu[k] = q->rho * (ju + s->e_u * s->e_u / q->delta);
    s->Mp[k] = s->k_u * s->k_u / s->Mu[k] + q->delta / q->rho;
    s->invMp[k] = 1.0 / s->Mp[k];
  }
  // preconditioner: J1 approximated by jbar = 1 (eq. (3.10) with circulant
  // blocks); under Algorithm 2 the blocks cy I, cu I are taken exactly
  const double jbar = 1.0;
  const double ay = q->prox ? s->cy : jbar, au = q->prox ? s->cu : q->gamma * jbar;
  s->a = q->rho * (ay + s->e_y * s->e_y / q->delta);
  const double mbar = s->k_u * s->k_u / (q->rho * (au + s->e_u * s->e_u / q->delta)) + q->delta / q->rho;
  s->inv_mbar = 1.0 / mbar;
  // eq. (3.11): |L + (a mbar)^{1/2}|^2 / mbar = a + |L|^2 / mbar + 2 (a / mbar)^{1/2} Re L
  s->match2 = q->precond_kind == 1 ? 2.0 * std::sqrt(s->a / mbar) : 0.0;
  // precond_kind 2: column (x, t) of B = psi D holds psi ct[t'-t] at the same
  // node of every later level t' and the spatial column at level t, so
  // diag(S) = My(t) + psi^2 (sum_{t'>t} ct[t'-t]^2 / Mp(t') + A(x, y) / Mp(t))
  s->ds_alpha.clear();
  s->ds_beta.clear();
  s->ds_class.clear();
  s->ds_tab.clear();
  if (q->precond_kind == 2) {
    if (s->dsA.empty()) diag_scaling_table(s);
    const double psi2 = s->psi * s->psi;
    s->ds_alpha.assign(nt, 0.0);
    s->ds_beta.assign(nt, 0.0);
    long double meanA = 0;
    for (double v : s->dsA) meanA += v;
    meanA /= (long double)s->dsA.size();
    long double s0 = 0;
    for (int t = 0; t < nt; ++t) {
      long double later = 0;
      for (int t2 = t + 1; t2 < nt; ++t2) later += (long double)s->ct[t2 - t] * s->ct[t2 - t] / s->Mp[t2];
      s->ds_alpha[t] = (double)(s->My[t] + psi2 * later);
      s->ds_beta[t] = psi2 / s->Mp[t];
      s0 += s->ds_alpha[t] + s->ds_beta[t] * meanA;
    }
    s0 /= nt;
    for (int t = 0; t < nt; ++t) {
      s->ds_alpha[t] = (double)(s->ds_alpha[t] / s0);
      s->ds_beta[t] = (double)(s->ds_beta[t] / s0);
    }
    // one table of Delta per distinct (alpha', beta'): implicit Euler has at most
    // three (interior levels, the last two), a fractional time order one per level
    const size_t plane = s->dsA.size();
    s->ds_class.assign(nt, 0);
    std::vector<int> first;  // a slice of each class
    for (int t = 0; t < nt; ++t) {
      int c = 0;
      while (c < (int)first.size() &&
             !(s->ds_alpha[first[c]] == s->ds_alpha[t] && s->ds_beta[first[c]] == s->ds_beta[t]))
        ++c;
      if (c == (int)first.size()) first.push_back(t);
      s->ds_class[t] = c;
    }
    s->ds_tab.resize(first.size() * plane);
    for (size_t c = 0; c < first.size(); ++c)
      for (size_t k = 0; k < plane; ++k)
        s->ds_tab[c * plane + k] = 1.0 / std::sqrt(s->ds_alpha[first[c]] + s->ds_beta[first[c]] * s->dsA[k]);
  }
}

namespace {
// Diagonal and squared off-diagonal column sums of one line operator
// L = c (diag(cp) G + diag(cm) G^T), G[r, i] = g_{r-i+1} (zero for r < i-1):
// column i holds c (cp[r] g_{r-i+1} + cm[r] g_{i-r+1}) in row r, the first
// term only for r >= i-1, the second only for r <= i+1.  Adds L_ii to dia[i]
// and sum_{r != i} L[r, i]^2 to off[i] (stride `st` between the line's nodes).
void line_column_sums(const AxisTables& ax, const double* cp, const double* cm, int n, double* dia, double* off,
                      size_t st) {
  const std::vector<double>& g = ax.g;
  std::vector<double> g2(n + 2, 0.0), cp2(n), cm2(n);
  for (int k = 0; k <= n && k < (int)g.size(); ++k) g2[k] = g[k] * g[k];
  for (int r = 0; r < n; ++r) {
    cp2[r] = cp[r] * cp[r];
    cm2[r] = cm[r] * cm[r];
  }
  const double c2 = ax.c * ax.c;
  for (int i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int r = i + 2; r < n; ++r) acc += cp2[r] * g2[r - i + 1];  // below the band: G only
    for (int r = 0; r <= i - 2; ++r) acc += cm2[r] * g2[i - r + 1];  // above it: G^T only
    if (i >= 1) {
      const double v = cp[i - 1] * g[0] + cm[i - 1] * g[2];
      acc += v * v;
    }
    if (i + 1 < n) {
      const double v = cp[i + 1] * g[2] + cm[i + 1] * g[0];
      acc += v * v;
    }
    dia[i * st] += ax.c * (cp[i] + cm[i]) * g[1];
    off[i * st] += c2 * acc;
  }
}
}  // namespace

void diag_scaling_table(Setup* s) {
  // A(x, y) = (ct[0] - Lx_ii - Ly_ii)^2 + sum_{r != i} Lx[r, i]^2 + sum_{r != i} Ly[r, i]^2,
  // with Lx[r, i] = cx (d+(r) G[r, i] + d-(r) G[i, r]) along the x-line of the node
  // (eq. (4.6)-(4.7)) and Ly the same along y; lines split over host threads
  const int nx = s->nx, ny = s->ny;
  const size_t plane = (size_t)nx * ny;
  std::vector<double> ones((size_t)std::max(nx, ny), 1.0);
  std::vector<double> off(plane, 0.0), dia(plane, 0.0), offy(plane, 0.0), diay(plane, 0.0);
  const int nthr = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  auto run = [&](int count, const std::function<void(int)>& f) {
    std::vector<std::thread> th;
    for (int w = 0; w < nthr; ++w)
      th.emplace_back([&, w]() {
        for (int k = w; k < count; k += nthr) f(k);
      });
    for (auto& t : th) t.join();
  };
  run(ny, [&](int j) {  // x-lines: contiguous coefficients of row j
    const double* cp = s->var ? &s->dplus[(size_t)j * nx] : ones.data();
    const double* cm = s->var ? &s->dminus[(size_t)j * nx] : ones.data();
    line_column_sums(s->x, cp, cm, nx, &dia[(size_t)j * nx], &off[(size_t)j * nx], 1);
  });
  run(nx, [&](int i) {  // y-lines: column i of the coefficient fields
    std::vector<double> cp(ny, 1.0), cm(ny, 1.0);
    if (s->var)
      for (int j = 0; j < ny; ++j) {
        cp[j] = s->dplus[(size_t)j * nx + i];
        cm[j] = s->dminus[(size_t)j * nx + i];
      }
    line_column_sums(s->y, cp.data(), cm.data(), ny, &diay[i], &offy[i], (size_t)nx);
  });
  s->dsA.resize(plane);
  for (size_t k = 0; k < plane; ++k) {
    const double d0 = s->ct[0] - dia[k] - diay[k];
    s->dsA[k] = d0 * d0 + off[k] + offy[k];
  }
}

int build_setup(const fde_problem* p, const fde_admm_params* q, Setup* s, std::string* msg) {
  const int st = validate(p, q, msg);
  if (st != FDE_OK) return st;
  s->nx = p->nx;
  s->ny = p->ny;
  s->nt = p->nt;
  s->T = p->T;
  s->ht = p->T / p->nt;
  const double hx = 1.0 / (p->nx + 1), hy = 1.0 / (p->ny + 1);
  s->var = (p->dplus != nullptr) || (p->dminus != nullptr);
  const size_t plane = (size_t)p->nx * p->ny;
  s->dplus.assign(p->dplus ? p->dplus : (const double*)nullptr, p->dplus ? p->dplus + plane : nullptr);
  s->dminus.assign(p->dminus ? p->dminus : (const double*)nullptr, p->dminus ? p->dminus + plane : nullptr);
  if (s->var) {
    if (s->dplus.empty()) s->dplus.assign(plane, 1.0);
    if (s->dminus.empty()) s->dminus.assign(plane, 1.0);
  }
  // arithmetic means over the interior nodes enter the circulant preconditioner
  auto mean = [&](const std::vector<double>& f) {
    if (f.empty()) return 1.0;
    long double acc = 0;
    for (double v : f) acc += v;
    return (double)(acc / f.size());
  };
  s->dbar_plus = mean(s->dplus);
  s->dbar_minus = mean(s->dminus);
  build_axis(p->nx, hx, p->alpha, s->dbar_plus, s->dbar_minus, s->var, &s->x);
  build_axis(p->ny, hy, p->beta, s->dbar_plus, s->dbar_minus, s->var, &s->y);
  // time: the Caputo matrix of eq. (4.5), lower-triangular Toeplitz with first
  // column g_k(alpha_t) / ht^alpha_t; order 1 gives (1, -1, 0, ..)/ht, implicit Euler
  s->alpha_t = (p->alpha_t == 0.0) ? 1.0 : p->alpha_t;
  s->frac_t = s->alpha_t != 1.0;
  const double hta = std::pow(s->ht, s->alpha_t);
  {
    const std::vector<double> gt = grunwald_weights(s->alpha_t, p->nt - 1);
    s->ct.assign(p->nt, 0.0);
    for (int k = 0; k < p->nt; ++k) s->ct[k] = s->frac_t ? gt[k] / hta : (k == 0 ? 1.0 : (k == 1 ? -1.0 : 0.0)) / s->ht;
  }
  std::vector<double> tn(p->nt, 0.0);
  s->tchan_t = tchan_eigs(s->ct, tn);  // T. Chan column c_i = (n - i) t_i / n
  s->tw_t = twiddles(p->nt);
  if (s->frac_t) {
    // circulant embedding of C_t (length L >= 2nt): first column (c_0 .. c_{nt-1}, 0 .. 0)
    const int L = embed_length(p->nt);
    s->Lt = L;
    std::vector<cd> col(L, cd(0, 0));
    for (int k = 0; k < p->nt; ++k) col[k] = s->ct[k];
    const std::vector<cd> lam = dft(col);
    s->lam_t.resize(L);
    s->lam_tT.resize(L);
    for (int k = 0; k < L; ++k) {
      s->lam_t[k] = lam[k] / (double)L;
      s->lam_tT[k] = std::conj(lam[k]) / (double)L;  // C_t^T embeds as the reversed column
    }
    s->tw_t_emb = twiddles(L);
  }
  // psi = min{ht^alpha_t, hx^alpha, hy^beta} (Sec. 5)
  s->psi = p->psi_scaling ? std::fmin(hta, std::fmin(std::pow(hx, p->alpha), std::pow(hy, p->beta))) : 1.0;
  s->e_y = 1.0;
  s->e_u = (p->psi_scaling == 1) ? s->psi : 1.0;
  s->k_u = s->psi * p->ctrl_sign;
  s->obj_weights = p->obj_weights;
  set_admm_scalings(q, s);
  return FDE_OK;
}

}  // namespace host
}  // namespace fde
