// Drives the host-side setup (validation, Grünwald weights, embedding and
// T. Chan tables, twiddles, ADMM scalings, the threaded diagonal-scaling
// tables) over the supported size range and the parameter variants, for a
// build under AddressSanitizer and
// UndefinedBehaviorSanitizer.  Exit status 0 when every table is finite and
// every invalid input is rejected.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "host_setup.hpp"

namespace {
int failures = 0;

void check(bool ok, const std::string& what) {
  if (!ok) {
    std::fprintf(stderr, "FAIL: %s\n", what.c_str());
    ++failures;
  }
}

bool finite_all(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

bool finite_all(const std::vector<fde::host::cd>& v) {
  for (const auto& x : v)
    if (!std::isfinite(x.real()) || !std::isfinite(x.imag())) return false;
  return true;
}

fde_admm_params params() {
  fde_admm_params q{};
  q.gamma = 1e-4;
  q.delta = 1.0;
  q.rho = 1.0;
  q.ya = -INFINITY;
  q.yb = INFINITY;
  q.ua = -1.0;
  q.ub = 1.0;
  q.krylov_tol = 1e-10;
  q.krylov_maxit = 1000;
  q.admm_tol = 1e-6;
  q.admm_maxit = 100;
  return q;
}

fde_problem problem(int nx, int ny, int nt) {
  fde_problem p{};
  p.nx = nx;
  p.ny = ny;
  p.nt = nt;
  p.T = 1.0;
  p.alpha = 1.5;
  p.beta = 1.3;
  p.ctrl_sign = 1.0;
  p.psi_scaling = 1;
  return p;
}

void run(const fde_problem& p, const fde_admm_params& q, const std::string& tag) {
  fde::host::Setup s;
  std::string msg;
  const int st = fde::host::build_setup(&p, &q, &s, &msg);
  check(st == FDE_OK, tag + ": build_setup " + msg);
  if (st != FDE_OK) return;
  for (const fde::host::AxisTables* ax : {&s.x, &s.y}) {
    check(finite_all(ax->g) && finite_all(ax->dg), tag + ": weights");
    check(finite_all(ax->lamG) && finite_all(ax->lamGT) && finite_all(ax->lamFwd) && finite_all(ax->lamTr),
          tag + ": embedding eigenvalues");
    check(finite_all(ax->tchan) && finite_all(ax->tw) && finite_all(ax->tw_emb), tag + ": T. Chan / twiddles");
  }
  check(finite_all(s.tchan_t) && finite_all(s.tw_t) && finite_all(s.ct), tag + ": time tables");
  check(finite_all(s.My) && finite_all(s.Mu) && finite_all(s.Mp) && finite_all(s.invMp), tag + ": scalings");
  check(std::isfinite(s.psi) && s.psi > 0 && std::isfinite(s.a) && std::isfinite(s.inv_mbar), tag + ": scalars");
  if (q.precond_kind == 2) {
    // diagonal scaling: one positive table per class, every time slice in a class
    const size_t plane = (size_t)p.nx * p.ny;
    check(s.dsA.size() == plane && finite_all(s.dsA), tag + ": diag(S) spatial table");
    check(s.ds_class.size() == (size_t)p.nt && !s.ds_tab.empty() && s.ds_tab.size() % plane == 0,
          tag + ": scaling table sizes");
    const int classes = (int)(s.ds_tab.size() / plane);
    bool in_range = true, positive = true;
    for (int c : s.ds_class) in_range = in_range && c >= 0 && c < classes;
    for (double v : s.ds_tab) positive = positive && std::isfinite(v) && v > 0;
    check(in_range, tag + ": scaling classes");
    check(positive, tag + ": scaling table positive");
  }
}
}  // namespace

int main() {
  const fde_admm_params q = params();
  const int sizes[] = {4, 6, 8, 12, 24, 96, 256, 384, 1024};
  for (int n : sizes) run(problem(n, 4, 6), q, "nx=" + std::to_string(n));
  for (int n : sizes) run(problem(8, n, 4), q, "ny=" + std::to_string(n));
  for (int n : sizes) run(problem(4, 6, n), q, "nt=" + std::to_string(n));
  {
    fde_problem p = problem(24, 16, 8);
    std::vector<double> dp(24 * 16), dm(24 * 16);
    for (size_t i = 0; i < dp.size(); ++i) {
      dp[i] = 1.0 + 0.5 * std::sin(0.1 * (double)i);
      dm[i] = 0.7;
    }
    p.dplus = dp.data();
    p.dminus = dm.data();
    run(p, q, "variable coefficients");
    p.alpha_t = 0.7;
    run(p, q, "Caputo order 0.7");
    fde_admm_params q2 = q;
    q2.prox = 1;
    q2.prox_cy = 1.5;
    q2.rho = 0.9;
    q2.precond_kind = 1;
    run(p, q2, "Algorithm 2, matching preconditioner");
    p.psi_scaling = 2;
    p.obj_weights = 1;
    run(p, q, "psi scaling 2, trapezoidal weights");
    fde_admm_params q3 = q;
    q3.precond_kind = 2;
    run(p, q3, "diagonally scaled preconditioner, Caputo order 0.7");
    p.alpha_t = 0.0;
    run(p, q3, "diagonally scaled preconditioner, implicit Euler");
  }
  {
    fde_admm_params q3 = q;
    q3.precond_kind = 2;
    for (int n : sizes) run(problem(n, 6, 4), q3, "scaled preconditioner nx=" + std::to_string(n));
    for (int n : sizes) run(problem(4, n, 6), q3, "scaled preconditioner ny=" + std::to_string(n));
    q3.krylov_solver = 1;
    fde_problem pk = problem(8, 8, 8);
    fde::host::Setup sk;
    std::string mk;
    check(fde::host::build_setup(&pk, &q3, &sk, &mk) == FDE_EINVAL && !mk.empty(), "MINRES with kind 2 rejected");
  }
  // invalid inputs are rejected with a message, before any table is built
  std::string msg;
  fde::host::Setup s;
  fde_problem bad = problem(5, 8, 8);
  check(fde::host::build_setup(&bad, &q, &s, &msg) == FDE_EINVAL && !msg.empty(), "nx=5 rejected");
  bad = problem(8, 8, 2048);
  check(fde::host::build_setup(&bad, &q, &s, &msg) == FDE_EINVAL, "nt=2048 rejected");
  bad = problem(8, 8, 8);
  bad.alpha = 2.5;
  check(fde::host::build_setup(&bad, &q, &s, &msg) == FDE_EINVAL, "alpha=2.5 rejected");
  fde_admm_params qb = q;
  qb.rho = 2.0;
  check(fde::host::validate_params(&qb, &msg) == FDE_EINVAL, "rho=2 rejected");
  qb = q;
  qb.ua = NAN;
  check(fde::host::validate_params(&qb, &msg) == FDE_EINVAL, "NaN bound rejected");
  check(fde::host::validate(nullptr, &q, &msg) == FDE_EINVAL, "null problem rejected");
  if (failures == 0) std::printf("host setup: all checks passed\n");
  return failures == 0 ? 0 : 1;
}
