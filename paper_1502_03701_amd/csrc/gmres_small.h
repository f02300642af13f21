// Device-resident small state of GMRES solves (one GState per system).
#pragma once

#include "sa_internal.h"

namespace sa {

constexpr int GMAX = 128;   // largest restart length

struct GTail {
  double bnorm2, bnorm, rnorm2, beta, inv, tol, relres;
  int active, converged, breakdown, nonfinite, have_update, exhausted;
  int jdone, jlimit, restart;
  int naug;                      // augmentation steps after the restart Krylov steps this cycle
  long long iters, matvecs, max_matvec;
  long long krylov;              // Krylov steps (operator and preconditioner applications)
};

struct GState {
  double H[(GMAX + 1) * GMAX];   // column j at H + j*(GMAX+1)
  double cs[GMAX], sn[GMAX];
  double g[GMAX + 1];
  double y[GMAX];
  double d1[GMAX + 2];           // first CGS pass: V^T w, then ||w||^2 (A z_j, unorthogonalised)
  double d2[GMAX + 1];           // second CGS pass: V^T w
  double wn2;                    // ||w||^2 after both passes
  GTail t;                       // scalars, copied to the host once per cycle
};

// Strides of GState members in units of their element type.
constexpr long long GS_DOUBLES = sizeof(GState) / sizeof(double);
constexpr long long GS_INTS = sizeof(GState) / sizeof(int);
static_assert(sizeof(GState) % sizeof(double) == 0, "GState size");

// One Arnoldi step of the small state, done cooperatively by the threads of
// one block (any size >= 1): column j of H is d1[0..j] + d2[0..j] with
// H(j+1, j) = sqrt(wn2); the previous rotations are applied to it, a new
// rotation zeroes H(j+1, j), g is rotated and the flags are updated.
// d1[j+1] holds ||A z_j||^2 before orthogonalisation (breakdown test).
__device__ inline void gstate_step_block(GState* st, int j) {
  __shared__ double hc[GMAX + 2], rc[GMAX], rs[GMAX];
  if (!st->t.active) return;
  for (int i = threadIdx.x; i <= j; i += blockDim.x) hc[i] = st->d1[i] + st->d2[i];
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    rc[i] = st->cs[i];
    rs[i] = st->sn[i];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int ld = GMAX + 1;
  double* Hj = st->H + (long long)j * ld;
  const double hn = sqrt(st->wn2);
  hc[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double t = rc[i] * hc[i] + rs[i] * hc[i + 1];
    hc[i + 1] = -rs[i] * hc[i] + rc[i] * hc[i + 1];
    hc[i] = t;
  }
  const double a = hc[j], b = hc[j + 1];
  double c = 1.0, s = 0.0;
  if (b != 0.0) {
    const double r = hypot(a, b);
    c = a / r;
    s = b / r;
  }
  st->cs[j] = c;
  st->sn[j] = s;
  hc[j] = c * a + s * b;
  hc[j + 1] = 0.0;
  for (int i = 0; i <= j + 1; ++i) Hj[i] = hc[i];
  const double gj = st->g[j];
  st->g[j + 1] = -s * gj;
  st->g[j] = c * gj;
  st->t.jdone = j + 1;
  st->t.have_update = 1;
  st->t.iters += 1;
  if (j < st->t.restart) {   // augmentation steps reuse stored products
    st->t.matvecs += 1;
    st->t.krylov += 1;
  }
  const double est = fabs(s * gj);
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

// All launchers act on nsys consecutive states (one block each).
void gstate_init(GState* st, int nsys, double tol, int restart, long long max_matvec, hipStream_t s);
void gstate_set_bnorm(GState* st, int nsys, hipStream_t s);
// beta = ||r||, convergence / budget tests; the cycle runs `restart` Krylov
// steps (fewer if the operator budget is short) and then naug augmentation
// steps
// products: operator products behind this cycle's residual (0 when x was zero)
void gstate_cycle_start(GState* st, int nsys, hipStream_t s, int naug = 0, int products = 1);
void gstate_step(GState* st, int nsys, int j, hipStream_t s);
void gstate_finish(GState* st, int nsys, hipStream_t s);

}  // namespace sa
