// Small dense state of restarted GMRES kept on the device (Section
// "Iterative solvers"): the Hessenberg column of each Arnoldi step, the
// Givens rotations that reduce it to triangular form, the rotated right-hand
// side g whose last entry is the residual estimate, and the triangular
// solve at the end of a cycle.  One thread per system does this O(m) work per
// step; the flags it writes (active / converged / breakdown / exhausted) let
// the remaining kernels of a cycle return immediately for that system.
#include "gmres_small.h"

namespace sa {
namespace {

__global__ void init_kernel(GState* base, double tol, int restart, long long max_matvec) {
  if (threadIdx.x != 0) return;
  GState* st = base + blockIdx.x;
  st->t.tol = tol;
  st->t.restart = restart;
  st->t.jlimit = restart;
  st->t.max_matvec = max_matvec;
  st->t.active = 0;
  st->t.converged = 0;
  st->t.breakdown = 0;
  st->t.nonfinite = 0;
  st->t.exhausted = 0;
  st->t.iters = 0;
  st->t.matvecs = 0;
  st->t.have_update = 0;
  st->t.jdone = 0;
}

__global__ void set_bnorm_kernel(GState* base) {
  if (threadIdx.x != 0) return;
  GState* st = base + blockIdx.x;
  st->t.bnorm = sqrt(st->t.bnorm2);
}

__global__ void cycle_start_kernel(GState* base) {
  if (threadIdx.x != 0) return;
  GState* st = base + blockIdx.x;
  st->t.jdone = 0;
  st->t.have_update = 0;
  if (st->t.converged || st->t.nonfinite || st->t.exhausted) {
    st->t.active = 0;
    return;
  }
  const double beta = sqrt(st->t.rnorm2);
  st->t.beta = beta;
  st->t.relres = st->t.bnorm > 0.0 ? beta / st->t.bnorm : 0.0;
  st->t.matvecs += 1;   // the residual product of this cycle
  st->t.active = 0;
  if (!isfinite(beta)) {
    st->t.nonfinite = 1;
    return;
  }
  if (st->t.bnorm == 0.0 || beta <= st->t.tol * st->t.bnorm) {
    st->t.converged = 1;
    return;
  }
  const long long left = st->t.max_matvec - st->t.matvecs;
  if (left <= 0) {
    st->t.exhausted = 1;
    return;
  }
  st->t.jlimit = left < st->t.restart ? (int)left : st->t.restart;
  st->g[0] = beta;
  st->t.inv = 1.0 / beta;
  st->t.active = 1;
}

// Column j of H is d1[0..j] + d2[0..j] (the two Gram-Schmidt passes) with
// H(j+1, j) = sqrt(wn2); d1[j+1] holds ||A z_j||^2 before orthogonalisation.
__global__ void step_kernel(GState* base, int j) {
  if (threadIdx.x != 0) return;
  GState* st = base + blockIdx.x;
  if (!st->t.active) return;
  const int ld = GMAX + 1;
  double* Hj = st->H + (long long)j * ld;
  for (int i = 0; i <= j; ++i) Hj[i] = st->d1[i] + st->d2[i];
  const double hn = sqrt(st->wn2);
  Hj[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double t = st->cs[i] * Hj[i] + st->sn[i] * Hj[i + 1];
    Hj[i + 1] = -st->sn[i] * Hj[i] + st->cs[i] * Hj[i + 1];
    Hj[i] = t;
  }
  const double a = Hj[j], b = Hj[j + 1];
  double c = 1.0, s = 0.0;
  if (b != 0.0) {
    const double r = hypot(a, b);
    c = a / r;
    s = b / r;
  }
  st->cs[j] = c;
  st->sn[j] = s;
  Hj[j] = c * a + s * b;
  Hj[j + 1] = 0.0;
  st->g[j + 1] = -s * st->g[j];
  st->g[j] = c * st->g[j];
  st->t.jdone = j + 1;
  st->t.have_update = 1;
  st->t.iters += 1;
  st->t.matvecs += 1;
  const double est = fabs(st->g[j + 1]);
  st->t.relres = est / st->t.bnorm;
  if (!isfinite(hn) || !isfinite(est)) {
    st->t.nonfinite = 1;
    st->t.active = 0;
    return;
  }
  if (hn <= 1e-14 * sqrt(st->d1[j + 1])) {
    st->t.breakdown = 1;
    st->t.active = 0;
    return;
  }
  st->t.inv = 1.0 / hn;
  if (est <= st->t.tol * st->t.bnorm || j + 1 >= st->t.jlimit) st->t.active = 0;
}

// y = R^{-1} g(0..jdone) by back substitution.
__global__ void finish_kernel(GState* base) {
  if (threadIdx.x != 0) return;
  GState* st = base + blockIdx.x;
  const int n = st->t.jdone;
  const int ld = GMAX + 1;
  for (int i = n - 1; i >= 0; --i) {
    double s = st->g[i];
    for (int k = i + 1; k < n; ++k) s -= st->H[(long long)k * ld + i] * st->y[k];
    st->y[i] = s / st->H[(long long)i * ld + i];
  }
  for (int i = n; i < GMAX; ++i) st->y[i] = 0.0;
  st->t.active = 0;
}

}  // namespace

void gstate_init(GState* st, int nsys, double tol, int restart, long long max_matvec, hipStream_t s) {
  init_kernel<<<nsys, 64, 0, s>>>(st, tol, restart, max_matvec);
}
void gstate_set_bnorm(GState* st, int nsys, hipStream_t s) { set_bnorm_kernel<<<nsys, 64, 0, s>>>(st); }
void gstate_cycle_start(GState* st, int nsys, hipStream_t s) { cycle_start_kernel<<<nsys, 64, 0, s>>>(st); }
void gstate_step(GState* st, int nsys, int j, hipStream_t s) { step_kernel<<<nsys, 64, 0, s>>>(st, j); }
void gstate_finish(GState* st, int nsys, hipStream_t s) { finish_kernel<<<nsys, 64, 0, s>>>(st); }

}  // namespace sa
