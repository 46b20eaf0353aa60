// Host-side (CPU, FP64) setup of the GPU path: validation, Grünwald weights,
// embedding-circulant and T. Chan eigenvalue tables, twiddles and the
// diagonal scalings of the ADMM x-step.  Pure C++: no HIP dependency, so it
// can be built and tested on a machine without a GPU.
#pragma once
#include <complex>
#include <string>
#include <vector>

#include "../../include/fde.h"

namespace fde {
namespace host {

using cd = std::complex<double>;

struct AxisTables {
  int n = 0;
  int L = 0;                           // embedding length of the line passes (2n, or longer)
  double h = 0, order = 0, c = 0;      // mesh size, fractional order, c_a / h^a
  std::vector<double> g, dg;           // weights g_0..g_n and d g_k / d a
  std::vector<cd> lamG, lamGT;         // L-point embedding eigenvalues of G, G^T, scaled by c/L
  std::vector<cd> lamFwd, lamTr;       // constant-coefficient combined operator (mean coeffs)
  std::vector<cd> dopA, dopB;          // d L_a / d a: variable coeffs (G-part, G^T-part), else combined in A
  std::vector<cd> tchan;               // T. Chan eigenvalues (length n) of the mean operator
  std::vector<cd> tw_emb, tw;          // twiddles exp(-2 pi i m / L') for L' = L and L' = n
};

struct Setup {
  int nx = 0, ny = 0, nt = 0;
  double T = 1, ht = 0, psi = 1, e_y = 1, e_u = 1, k_u = 1;
  double a = 0, inv_mbar = 0;          // preconditioner scalars
  double cy = 0, cu = 0;               // Algorithm 2: J1 + R_y = cy I, J2 + R_u = cu I (0: Algorithm 1)
  double match2 = 0;                   // matching approximation: 2 (a / mbar)^{1/2} (0: S~)
  bool var = false;                    // variable coefficient fields present
  int obj_weights = 0;                 // 0: J1 = I, 1: trapezoidal in time
  double dbar_plus = 1, dbar_minus = 1;
  AxisTables x, y;
  double alpha_t = 1;                  // time order; 1 = implicit Euler
  bool frac_t = false;                 // alpha_t < 1: the time term is its own line pass
  std::vector<double> ct;              // first column of the time matrix (length nt)
  std::vector<cd> tchan_t, tw_t;       // time T. Chan eigenvalues, twiddles (length nt)
  int Lt = 0;                          // embedding length along t (fractional order)
  std::vector<cd> lam_t, lam_tT, tw_t_emb;  // Lt-point embedding eigenvalues of C_t, C_t^T (with 1/Lt), twiddles
  std::vector<double> wts, My, Mu, Mp, invMp;  // per time slice
  std::vector<double> dplus, dminus;   // (ny*nx) copies when var
  // precond_kind 2: diag(S) = alpha_t + beta_t A(x, y) (eq. (3.9) in the psi-scaled
  // form), A the spatial part of the squared column norms of D; the kernels scale
  // by Delta = (alpha'_t + beta'_t A)^{-1/2}, primes: divided by s0 = mean diag(S).
  // Slices with equal (alpha', beta') share one table of Delta (a class).
  std::vector<double> dsA;                 // (ny*nx); computed when first needed
  std::vector<double> ds_alpha, ds_beta;   // per time slice (alpha', beta')
  std::vector<int> ds_class;               // per time slice: its table
  std::vector<double> ds_tab;              // (classes, ny*nx): Delta
};

bool length_supported(int n);
int embed_length(int n);  // FFT length of the Toeplitz line passes along an axis of n nodes
int validate(const fde_problem* p, const fde_admm_params* q, std::string* msg);
int validate_params(const fde_admm_params* q, std::string* msg);
int build_setup(const fde_problem* p, const fde_admm_params* q, Setup* s, std::string* msg);
// ADMM scalings that depend on (gamma, delta, rho) only
void set_admm_scalings(const fde_admm_params* q, Setup* s);
// the spatial table A(x, y) of precond_kind 2 (fills s->dsA)
void diag_scaling_table(Setup* s);

std::vector<double> grunwald_weights(double a, int n);
std::vector<double> grunwald_weight_derivs(double a, int n);
std::vector<cd> dft(const std::vector<cd>& c);  // lambda_k = sum_m c_m exp(-2 pi i k m / L)
std::vector<cd> twiddles(int L);
std::vector<cd> tchan_eigs(const std::vector<double>& t_pos, const std::vector<double>& t_neg);

}  // namespace host
}  // namespace fde
