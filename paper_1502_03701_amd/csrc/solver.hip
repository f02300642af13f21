// Restarted GMRES (Section "Iterative solvers") for (J - sigma I) x = b, with
// classical Gram-Schmidt applied twice and optional right block-Jacobi
// preconditioning in the flexible form (the preconditioned directions are
// kept), plus the FP64-outer / FP32-inner iterative refinement form.
//
// One cycle is enqueued in full: residual, then per Arnoldi step the
// preconditioner, the operator, the two Gram-Schmidt passes and the Givens
// update.  Every kernel reads the device flag `active`, which the Givens
// kernel clears on convergence or breakdown, so the host synchronises only
// once per cycle to read the status.
#include <algorithm>
#include <cmath>

#include "sa_runtime.h"

namespace sa {
namespace {

hipError_t read_tail(GState* st, GTail& h, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(&h, &st->t, sizeof(GTail), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

}  // namespace

template <typename R>
int solve_gmres(Ctx* c, const sa_gmres_opts& o, double sigma, const R* b, R* x, int pc_shift,
                sa_gmres_info* info, const std::string& tag) {
  hipStream_t s = c->stream;
  const long long n = c->n;
  const int m = o.restart;
  const bool pc = pc_shift >= 0;
  const size_t vbytes = (size_t)n * sizeof(R);
  R* V = (R*)c->buffer(tag + "V", vbytes * (m + 1));
  R* Z = pc ? (R*)c->buffer(tag + "Z", vbytes * m) : V;
  GState* st = (GState*)c->buffer(tag + "state", sizeof(GState));
  Blas<R> bl;
  bl.partial = (double*)c->buffer("partial", sizeof(double) * RED_BLOCKS * PARTIAL_LD);
  bl.ldp = PARTIAL_LD;
  if (!V || !Z || !st || !bl.partial) return c->fail(SA_ENOMEM, "gmres: out of device memory");
  const int* act = &st->t.active;
  *info = sa_gmres_info{};

  gstate_init(st, o.tol, m, s);
  bl.nrm2sq(n, b, &st->t.bnorm2, nullptr, s);
  gstate_set_bnorm(st, s);
  long long matvecs = 0;
  int cycles = 0;
  hipError_t e;
  for (;;) {
    // r = b - (J - sigma I) x  -> V[:,0]
    e = c->jv<R>(x, V + n, 1, sigma, nullptr);
    if (e != hipSuccess) return c->hip_fail(e, "gmres residual");
    bl.residual(n, b, V + n, V, &st->t.rnorm2, nullptr, s);
    gstate_cycle_start(st, s);
    GTail h;
    e = read_tail(st, h, s);
    if (e != hipSuccess) return c->hip_fail(e, "gmres status");
    matvecs = h.matvecs;
    info->iters = h.iters;
    info->matvecs = h.matvecs;
    info->cycles = cycles;
    info->relres = h.relres;
    if (h.nonfinite) {
      info->status = SA_ENONFINITE;
      return c->fail(SA_ENONFINITE, "gmres: non-finite residual");
    }
    if (h.converged) {
      info->status = SA_OK;
      return SA_OK;
    }
    if (matvecs >= o.max_matvec) {
      info->status = SA_NOT_CONVERGED;
      return SA_NOT_CONVERGED;
    }
    const int jl = (int)std::min<long long>(m, o.max_matvec - matvecs);
    gstate_set_jlimit(st, jl, s);
    bl.scale(n, V, V, &st->t.inv, act, s);
    for (int j = 0; j < jl; ++j) {
      R* vj = V + (long long)j * n;
      R* w = V + (long long)(j + 1) * n;
      const R* zj = vj;
      if (pc) {
        R* zz = Z + (long long)j * n;
        e = precond_apply<R>(c, pc_shift, 1, vj, zz, act);
        if (e != hipSuccess) return c->hip_fail(e, "gmres precond");
        zj = zz;
      }
      e = c->jv<R>(zj, w, 1, sigma, act);
      if (e != hipSuccess) return c->hip_fail(e, "gmres jv");
      // CGS pass 1: d1 = V[0..j]^T w and ||w||^2
      bl.multidot(n, V, n, j + 2, w, st->d1, false, act, s);
      // pass 2: w -= V d1, d2 = V^T w
      bl.update(n, V, n, j + 1, st->d1, -1.0, w, w, 1, st->d2, false, act, s);
      // pass 3: w -= V d2, wn2 = ||w||^2
      bl.update(n, V, n, j + 1, st->d2, -1.0, w, w, 2, &st->wn2, false, act, s);
      gstate_step(st, j, s);
      bl.scale(n, w, w, &st->t.inv, act, s);
    }
    gstate_finish(st, s);
    // x += Z y  (Z = V without preconditioning)
    bl.update(n, Z, n, jl, st->y, 1.0, x, x, 0, nullptr, false, &st->t.have_update, s);
    e = hipGetLastError();
    if (e != hipSuccess) return c->hip_fail(e, "gmres cycle");
    ++cycles;
  }
}

template int solve_gmres<double>(Ctx*, const sa_gmres_opts&, double, const double*, double*, int,
                                 sa_gmres_info*, const std::string&);
template int solve_gmres<float>(Ctx*, const sa_gmres_opts&, double, const float*, float*, int,
                                sa_gmres_info*, const std::string&);

// Iterative refinement: FP64 residual and update, FP32 GMRES on the scaled
// residual equation.
int solve_ir(Ctx* c, const sa_gmres_opts& o, double sigma, const double* b, double* x, int pc_shift,
             sa_gmres_info* info) {
  hipStream_t s = c->stream;
  const long long n = c->n;
  double* r = (double*)c->buffer("ir_r", sizeof(double) * n);
  double* y = (double*)c->buffer("ir_y", sizeof(double) * n);
  float* r32 = (float*)c->buffer("ir_r32", sizeof(float) * n);
  float* d32 = (float*)c->buffer("ir_d32", sizeof(float) * n);
  GState* st = (GState*)c->buffer("ir_state", sizeof(GState));
  Blas<double> bl;
  bl.partial = (double*)c->buffer("partial", sizeof(double) * RED_BLOCKS * PARTIAL_LD);
  bl.ldp = PARTIAL_LD;
  Blas<float> bl32;
  bl32.partial = bl.partial;
  bl32.ldp = PARTIAL_LD;
  if (!r || !y || !r32 || !d32 || !st || !bl.partial) return c->fail(SA_ENOMEM, "ir: out of device memory");
  *info = sa_gmres_info{};
  gstate_init(st, o.tol, 0, s);
  bl.nrm2sq(n, b, &st->t.bnorm2, nullptr, s);
  gstate_set_bnorm(st, s);
  sa_gmres_opts in = o;
  in.prec = SA_F32;
  in.tol = o.inner_tol;
  long long inner_mv = 0, inner_it = 0;
  int inner_cycles = 0;
  hipError_t e;
  for (int outer = 0;; ++outer) {
    e = c->jv<double>(x, y, 1, sigma, nullptr);
    if (e != hipSuccess) return c->hip_fail(e, "ir residual");
    bl.residual(n, b, y, r, &st->t.rnorm2, nullptr, s);
    gstate_cycle_start(st, s);  // beta = ||r||, inv = 1/||r||, converged flag
    GTail h;
    e = read_tail(st, h, s);
    if (e != hipSuccess) return c->hip_fail(e, "ir status");
    info->outer = outer;
    info->relres = h.relres;
    info->iters = inner_it;
    info->matvecs = inner_mv + h.matvecs;
    info->cycles = inner_cycles;
    if (h.nonfinite) {
      info->status = SA_ENONFINITE;
      return c->fail(SA_ENONFINITE, "ir: non-finite residual");
    }
    if (h.converged) {
      info->status = SA_OK;
      return SA_OK;
    }
    if (outer >= o.max_outer || info->matvecs >= o.max_matvec) {
      info->status = SA_NOT_CONVERGED;
      return SA_NOT_CONVERGED;
    }
    // r32 = float(r / ||r||), d32 = 0
    cast_d2f(n, r, r32, &st->t.inv, s);
    bl32.fill(n, d32, 0.0f, s);
    sa_gmres_info ii{};
    in.max_matvec = std::max<long long>(1, o.max_matvec - info->matvecs);
    int rc = solve_gmres<float>(c, in, sigma, r32, d32, pc_shift, &ii, "ir32");
    if (rc < 0) return rc;
    inner_mv += ii.matvecs;
    inner_it += ii.iters;
    inner_cycles += ii.cycles;
        // x += ||r|| d
    axpy_f2d(n, d32, x, &st->t.beta, s);
  }
}

}  // namespace sa
