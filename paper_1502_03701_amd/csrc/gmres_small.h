// Device-resident small state of GMRES solves (one GState per system).
#pragma once

#include "sa_internal.h"

namespace sa {

constexpr int GMAX = 128;   // largest restart length

struct GTail {
  double bnorm2, bnorm, rnorm2, beta, inv, tol, relres;
  int active, converged, breakdown, nonfinite, have_update, exhausted;
  int jdone, jlimit, restart;
  long long iters, matvecs, max_matvec;
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

// All launchers act on nsys consecutive states (one block each).
void gstate_init(GState* st, int nsys, double tol, int restart, long long max_matvec, hipStream_t s);
void gstate_set_bnorm(GState* st, int nsys, hipStream_t s);
// beta = ||r||, convergence / budget tests, jlimit = min(restart, budget left)
void gstate_cycle_start(GState* st, int nsys, hipStream_t s);
void gstate_step(GState* st, int nsys, int j, hipStream_t s);
void gstate_finish(GState* st, int nsys, hipStream_t s);

}  // namespace sa
