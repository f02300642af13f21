// Device-resident small dense state of the implicitly restarted Arnoldi
// method (Algorithm 1).
#pragma once

#include "sa_internal.h"

namespace sa {

constexpr int MMAX = 64;   // largest Arnoldi dimension m

struct IState {
  double H[(MMAX + 1) * MMAX];   // Arnoldi Hessenberg, column-major, ld MMAX+1
  double Hm[MMAX * MMAX];        // working copy of H_m (ld MMAX)
  double Q[MMAX * MMAX];         // accumulated orthogonal factor of the shifts
  double M[MMAX * MMAX];         // QR workspace
  double HQ[MMAX * MMAX];        // product workspace
  double Tr[MMAX * MMAX], Ti[MMAX * MMAX];   // complex Schur form of H_m
  double Zr[MMAX * MMAX], Zi[MMAX * MMAX];   // Schur vectors
  double Yr[MMAX * MMAX], Yi[MMAX * MMAX];   // unit eigenvectors of H_m, sorted order
  double wr[MMAX], wi[MMAX];     // Ritz values, sorted by decreasing |theta|
  double est[MMAX];              // Ritz estimates ||f_m|| |e_m^T y|
  double er[MMAX], ei[MMAX];     // unsorted eigenvalues
  int order[MMAX];
  int partner[MMAX];
  double d1[MMAX + 2], d2[MMAX + 1], wn2, inv;
  double coef[2];                // beta_hat, Q(m,k) * H(m+1,m)
  double fnorm, hnorm, tol, sigma, mu;
  double lam_r[MMAX], lam_i[MMAX];
  int m, nev, k, nconv, done, fail, restarts, max_restarts;
};

// One Arnoldi column after the two Gram-Schmidt passes:
// H(0..j, j) = d1 + d2, H(j+1, j) = sqrt(wn2), inv = 1/H(j+1, j).
void iram_column(IState* st, int j, hipStream_t s);
// Restart step: Ritz values/vectors of H_m, Ritz estimates, convergence test;
// if not converged, the exact-shift QR steps, Q, H_k and the coefficients of
// the k-step update (done = 1 when converged or out of restarts).
void iram_restart(IState* st, int m, hipStream_t s);   // m: the Arnoldi dimension given to iram_init
// After V_k and f_k are formed: H(k, k-1) = ||f_k|| from wn2, inv = 1/||f_k||.
void iram_set_fk(IState* st, hipStream_t s);
void iram_init(IState* st, int m, int nev, double tol, double sigma, double mu, int max_restarts,
               hipStream_t s);
// inv = 1/sqrt(wn2)
void iram_inv_norm(IState* st, hipStream_t s);

// out[:, c] = sum_{r < nrow} V[:, r] C[r + c*ldc] for c < ncol (tall-skinny product)
void gemm_tall(long long n, const double* V, long long ldv, int nrow, const double* C, int ldc, int ncol,
               double* out, long long ldo, hipStream_t s);
// y = a[0] * x1 + a[1] * x2 (coefficients on the device)
void combine2(long long n, const double* x1, const double* x2, const double* a, double* y, hipStream_t s);
// partial sums for complex eigen-residuals: r = J x - lam x with x = xr + i xi.
// out[0] = ||r||^2, out[1] = ||x||^2
void eig_residual(long long n, const double* Jxr, const double* Jxi, const double* xr, const double* xi,
                  double lr, double li, double* partial, double* out, hipStream_t s);

}  // namespace sa
