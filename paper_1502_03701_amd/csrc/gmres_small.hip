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
  st->t.naug = 0;
  st->t.max_matvec = max_matvec;
  st->t.active = 0;
  st->t.converged = 0;
  st->t.breakdown = 0;
  st->t.nonfinite = 0;
  st->t.exhausted = 0;
  st->t.iters = 0;
  st->t.matvecs = 0;
  st->t.krylov = 0;
  st->t.have_update = 0;
  st->t.jdone = 0;
}

__global__ void set_bnorm_kernel(GState* base) {
  if (threadIdx.x != 0) return;
  GState* st = base + blockIdx.x;
  st->t.bnorm = sqrt(st->t.bnorm2);
}

__global__ void cycle_start_kernel(GState* base, int naug, int products) {
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
  st->t.matvecs += products;   // the residual product of this cycle (0: x was zero)
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
  st->t.naug = naug;
  st->t.jlimit = left < st->t.restart ? (int)left : st->t.restart + naug;
  st->g[0] = beta;
  st->t.inv = 1.0 / beta;
  st->t.active = 1;
}

__global__ void step_kernel(GState* base, int j) { gstate_step_block(base + blockIdx.x, j); }

// y = R^{-1} g(0..jdone) by back substitution.  Up to 64 columns: the
// triangle is staged in LDS (all loads issued at once) and lane k keeps the
// running right-hand side of row k; column i is eliminated after y_i is
// known (fixed order, deterministic).  Longer cycles: one thread, in place.
constexpr int FIN_MAX = 64;
__global__ void __launch_bounds__(64) finish_kernel(GState* base) {
  GState* st = base + blockIdx.x;
  const int n = st->t.jdone;
  const int ld = GMAX + 1;
  const int lane = threadIdx.x;
  if (n <= FIN_MAX) {
    __shared__ double Rt[FIN_MAX * (FIN_MAX + 1) / 2];   // column k at k(k+1)/2, rows 0..k
    constexpr int PER = (FIN_MAX * (FIN_MAX + 1) / 2 + 63) / 64;
    const int total = n * (n + 1) / 2;
    double v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int f = lane + 64 * q;
      v[q] = 0.0;
      if (f < total) {
        int k = (int)((sqrt(8.0 * f + 1.0) - 1.0) * 0.5);
        if ((k + 1) * (k + 2) / 2 <= f) ++k;
        if (k * (k + 1) / 2 > f) --k;
        v[q] = st->H[(long long)k * ld + (f - k * (k + 1) / 2)];
      }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int f = lane + 64 * q;
      if (f < total) Rt[f] = v[q];
    }
    __syncthreads();
    double rhs = lane < n ? st->g[lane] : 0.0;
    double yk = 0.0;
    for (int i = n - 1; i >= 0; --i) {
      const double yi = __shfl(rhs, i, 64) / Rt[i * (i + 1) / 2 + i];
      if (lane == i) yk = yi;
      if (lane < i) rhs -= Rt[i * (i + 1) / 2 + lane] * yi;
    }
    for (int i = lane; i < GMAX; i += 64) st->y[i] = (i == lane && i < n) ? yk : 0.0;
    if (lane == 0) st->t.active = 0;
    return;
  }
  if (lane != 0) return;
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
void gstate_cycle_start(GState* st, int nsys, hipStream_t s, int naug, int products) {
  cycle_start_kernel<<<nsys, 64, 0, s>>>(st, naug, products);
}
void gstate_step(GState* st, int nsys, int j, hipStream_t s) { step_kernel<<<nsys, 64, 0, s>>>(st, j); }
void gstate_finish(GState* st, int nsys, hipStream_t s) { finish_kernel<<<nsys, 64, 0, s>>>(st); }

}  // namespace sa
