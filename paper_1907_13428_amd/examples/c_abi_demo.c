/* A plain C client of libfde: no Python, no PyTorch.  It builds a problem,
 * creates a context, moves a field to the device with the HIP runtime, and
 * calls the operator, its transpose, the preconditioner and the PCG solve
 * through include/fde.h.
 *
 *     c_abi_demo nx ny nt alpha beta out.bin
 *
 * The input field is x[i] = ((37 i) mod 101) / 101 - 1/2 over [nt][ny][nx]
 * (exact in binary floating point, so any reader can regenerate it).  out.bin
 * receives D x, D^T x, S~^{-1} x and the PCG solution of S w = x, each as N
 * float64 values in that order.  The PCG iteration count and relative residual
 * go to stdout.  Exit status 0 on success. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "fde.h"

#define CHECK_FDE(call)                                                             \
  do {                                                                              \
    fde_status s_ = (call);                                                         \
    if (s_ != FDE_OK) {                                                             \
      fprintf(stderr, "%s failed (%d): %s\n", #call, (int)s_, fde_last_error());    \
      return 1;                                                                     \
    }                                                                               \
  } while (0)

#define CHECK_HIP(call)                                                             \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));             \
      return 1;                                                                     \
    }                                                                               \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 7) {
    fprintf(stderr, "usage: %s nx ny nt alpha beta out.bin\n", argv[0]);
    return 2;
  }
  fde_problem prob = {0};
  prob.nx = atoi(argv[1]);
  prob.ny = atoi(argv[2]);
  prob.nt = atoi(argv[3]);
  prob.T = 1.0;
  prob.alpha = atof(argv[4]);
  prob.beta = atof(argv[5]);
  prob.dplus = NULL;
  prob.dminus = NULL;
  prob.ctrl_sign = 1.0;
  prob.psi_scaling = 1;
  prob.obj_weights = 0;
  prob.precond_fp32 = 0;
  prob.alpha_t = 1.0;

  fde_admm_params prm = {0};
  prm.gamma = 1e-4;
  prm.delta = 1.0;
  prm.rho = 1.0;
  prm.ya = -1e300;
  prm.yb = 1e300;
  prm.ua = -1.0;
  prm.ub = 1.0;
  prm.krylov_tol = 1e-10;
  prm.krylov_maxit = 1000;
  prm.admm_tol = 1e-6;
  prm.admm_maxit = 100;
  CHECK_FDE(fde_validate(&prob, &prm));

  const size_t n = (size_t)prob.nx * prob.ny * prob.nt;
  double* hx = (double*)malloc(n * sizeof(double));
  double* hout = (double*)malloc(4 * n * sizeof(double));
  if (!hx || !hout) {
    fprintf(stderr, "host allocation failed\n");
    return 1;
  }
  for (size_t i = 0; i < n; ++i) hx[i] = (double)((37 * i) % 101) / 101.0 - 0.5;

  fde_ctx* ctx = NULL;
  CHECK_FDE(fde_create(&prob, &prm, NULL, &ctx));
  double *dx = NULL, *dy = NULL;
  CHECK_HIP(hipMalloc((void**)&dx, n * sizeof(double)));
  CHECK_HIP(hipMalloc((void**)&dy, n * sizeof(double)));
  CHECK_HIP(hipMemcpy(dx, hx, n * sizeof(double), hipMemcpyHostToDevice));

  CHECK_FDE(fde_apply_A(ctx, dx, dy, 0));
  CHECK_HIP(hipMemcpy(hout, dy, n * sizeof(double), hipMemcpyDeviceToHost));
  CHECK_FDE(fde_apply_A(ctx, dx, dy, 1));
  CHECK_HIP(hipMemcpy(hout + n, dy, n * sizeof(double), hipMemcpyDeviceToHost));
  CHECK_FDE(fde_precond(ctx, dx, dy));
  CHECK_HIP(hipMemcpy(hout + 2 * n, dy, n * sizeof(double), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemset(dy, 0, n * sizeof(double)));
  int iters = 0;
  double relres = 0.0;
  CHECK_FDE(fde_krylov(ctx, dx, dy, &iters, &relres));
  CHECK_HIP(hipMemcpy(hout + 3 * n, dy, n * sizeof(double), hipMemcpyDeviceToHost));

  CHECK_HIP(hipFree(dx));
  CHECK_HIP(hipFree(dy));
  CHECK_FDE(fde_destroy(ctx));

  FILE* f = fopen(argv[6], "wb");
  if (!f || fwrite(hout, sizeof(double), 4 * n, f) != 4 * n) {
    fprintf(stderr, "cannot write %s\n", argv[6]);
    return 1;
  }
  fclose(f);
  printf("%s pcg_iters=%d relres=%.3e\n", fde_version(), iters, relres);
  free(hx);
  free(hout);
  return 0;
}
