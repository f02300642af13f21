// Implicitly restarted Arnoldi method (Algorithm 1) on the Cayley transform
// C = (J - sigma I)^{-1} (J - mu I) (eq. cayley_transform): each Arnoldi
// step applies C by one operator product with shift mu and one GMRES (or
// refinement) solve with shift sigma (eq. cayley_arnoldi, applied inexactly
// to the inner tolerance), then orthogonalises in FP64 with classical
// Gram-Schmidt applied twice.  The small dense steps run in
// arnoldi_small.hip; the basis update V_k = V_m Q(:,1:k) and
// f_k = v_{k+1} beta_hat + f_m Q(m,k) are tall-skinny products.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "arnoldi_small.h"
#include "sa_runtime.h"

namespace sa {
namespace {

struct Iram {
  Ctx* c;
  const sa_eig_opts* o;
  double* V;      // n x (m+1)
  double* T;      // n x (m+1) temporaries (product output, Ritz vectors)
  double* tb;     // n
  IState* st;
  Blas<double> bl;
  sa_eig_result* res;
  long long n;
  int m;
};

int cayley_apply(Iram& w, const double* v, double* out) {
  Ctx* c = w.c;
  hipStream_t s = c->stream;
  const sa_eig_opts& o = *w.o;
  hipError_t e = c->jv<double>(v, w.tb, 1, o.mu, nullptr);
  if (e != hipSuccess) return c->hip_fail(e, "iram jv");
  w.bl.fill(w.n, out, 0.0, s);
  sa_gmres_info info{};
  int rc;
  const int pci = o.lin.use_precond ? 0 : -1;
  // out is zero: the solves start from x0 = 0 without an operator product
  if (o.lin.prec == SA_MIXED)
    rc = solve_ir(c, o.lin, o.sigma, w.tb, out, pci, &info, true);
  else
    rc = solve_gmres<double>(c, o.lin, 1, &o.sigma, w.tb, out, pci, &info, "g", false, true);
  if (rc < 0) return rc;
  w.res->n_cayley += 1;
  w.res->n_matvec += info.matvecs + 1;
  w.res->n_precond += info.precond_applies;
  return rc;   // SA_NOT_CONVERGED tolerated: the transform is applied inexactly
}

int extend(Iram& w, int j0) {
  Ctx* c = w.c;
  hipStream_t s = c->stream;
  const long long n = w.n;
  for (int j = j0; j < w.m; ++j) {
    double* vj = w.V + (long long)j * n;
    double* wv = w.V + (long long)(j + 1) * n;
    int rc = cayley_apply(w, vj, wv);
    if (rc < 0) return rc;
    w.bl.multidot(n, w.V, n, j + 2, wv, w.st->d1, false, nullptr, s);
    w.bl.update(n, w.V, n, j + 1, w.st->d1, -1.0, wv, wv, 1, w.st->d2, false, nullptr, s);
    w.bl.update(n, w.V, n, j + 1, w.st->d2, -1.0, wv, wv, 2, &w.st->wn2, false, nullptr, s);
    iram_column(w.st, j, s);
    w.bl.scale(n, wv, wv, &w.st->inv, nullptr, s);
  }
  return SA_OK;
}

int run_one(Ctx* c, const sa_eig_opts& o, const double* v0, sa_eig_result* res) {
  hipStream_t s = c->stream;
  Iram w;
  w.c = c;
  w.o = &o;
  w.n = c->n;
  w.m = o.ncv;
  w.res = res;
  const long long n = c->n;
  const int m = o.ncv;
  w.V = (double*)c->buffer("iramV", sizeof(double) * n * (m + 1));
  w.T = (double*)c->buffer("iramT", sizeof(double) * n * (m + 1));
  w.tb = (double*)c->buffer("iramB", sizeof(double) * n);
  w.st = (IState*)c->buffer("iramS", sizeof(IState));
  w.bl.partial = (double*)c->buffer("iram_partial", sizeof(double) * RED_BLOCKS * PARTIAL_LD);
  w.bl.ticket = (int*)c->buffer("iram_ticket", sizeof(int));
  w.bl.ldp = PARTIAL_LD;
  if (!w.V || !w.T || !w.tb || !w.st || !w.bl.partial || !w.bl.ticket)
    return c->fail(SA_ENOMEM, "iram: out of device memory");
  double* evr = res->evec_re_dev;
  double* evi = res->evec_im_dev;
  std::memset(res, 0, sizeof(*res));
  res->evec_re_dev = evr;
  res->evec_im_dev = evi;

  iram_init(w.st, m, o.nev, o.tol, o.sigma, o.mu, o.max_restarts, s);
  // v1 = v0 / ||v0||
  w.bl.nrm2sq(n, v0, &w.st->wn2, nullptr, s);
  iram_inv_norm(w.st, s);
  w.bl.scale(n, v0, w.V, &w.st->inv, nullptr, s);
  int rc = extend(w, 0);
  if (rc < 0) return rc;
  struct Small {
    int done, fail, k, nconv, restarts;
  } h{};
  for (;;) {
    iram_restart(w.st, m, s);
    hipError_t e = hipMemcpyAsync(&h.done, &w.st->done, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h.fail, &w.st->fail, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h.k, &w.st->k, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return c->hip_fail(e, "iram restart");
    if (h.fail) return c->fail(SA_EDEVICE, "iram: Hessenberg QR did not converge");
    if (h.done) break;
    const int k = h.k;
    // T[:, 0..k] = V_m Q(:, 0..k)
    gemm_tall(n, w.V, n, m, w.st->Q, MMAX, k + 1, w.T, n, s);
    // f_k = T[:, k] beta_hat + V[:, m] Q(m,k) H(m+1,m)  -> V[:, k] (unnormalised)
    combine2(n, w.T + (long long)k * n, w.V + (long long)m * n, w.st->coef, w.V + (long long)k * n, s);
    hipMemcpyAsync(w.V, w.T, sizeof(double) * n * k, hipMemcpyDeviceToDevice, s);
    w.bl.nrm2sq(n, w.V + (long long)k * n, &w.st->wn2, nullptr, s);
    iram_set_fk(w.st, s);
    w.bl.scale(n, w.V + (long long)k * n, w.V + (long long)k * n, &w.st->inv, nullptr, s);
    rc = extend(w, k);
    if (rc < 0) return rc;
  }
  // results
  double wr[MMAX], wi[MMAX], est[MMAX], lr[MMAX], li[MMAX];
  int small[4];
  hipMemcpyAsync(wr, w.st->wr, sizeof wr, hipMemcpyDeviceToHost, s);
  hipMemcpyAsync(wi, w.st->wi, sizeof wi, hipMemcpyDeviceToHost, s);
  hipMemcpyAsync(est, w.st->est, sizeof est, hipMemcpyDeviceToHost, s);
  hipMemcpyAsync(lr, w.st->lam_r, sizeof lr, hipMemcpyDeviceToHost, s);
  hipMemcpyAsync(li, w.st->lam_i, sizeof li, hipMemcpyDeviceToHost, s);
  hipMemcpyAsync(&small[0], &w.st->nconv, sizeof(int), hipMemcpyDeviceToHost, s);
  hipMemcpyAsync(&small[1], &w.st->restarts, sizeof(int), hipMemcpyDeviceToHost, s);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return c->hip_fail(e, "iram results");
  res->nconv = small[0];
  res->restarts = small[1];
  for (int i = 0; i < o.nev; ++i) {
    res->theta_re[i] = wr[i];
    res->theta_im[i] = wi[i];
    res->ritz_est[i] = est[i];
    res->lam_re[i] = lr[i];
    res->lam_im[i] = li[i];
    res->resid[i] = -1.0;
  }
  if (evr && evi) {
    // Ritz vectors x_i = V_m y_i (real and imaginary parts), true residuals
    gemm_tall(n, w.V, n, m, w.st->Yr, MMAX, o.nev, evr, n, s);
    gemm_tall(n, w.V, n, m, w.st->Yi, MMAX, o.nev, evi, n, s);
    double* Jr = w.T;
    double* Ji = w.T + n;
    double* out = (double*)c->buffer("iramR", sizeof(double) * 2);
    for (int i = 0; i < o.nev; ++i) {
      c->jv<double>(evr + (long long)i * n, Jr, 1, 0.0, nullptr);
      c->jv<double>(evi + (long long)i * n, Ji, 1, 0.0, nullptr);
      eig_residual(n, Jr, Ji, evr + (long long)i * n, evi + (long long)i * n, lr[i], li[i], w.bl.partial,
                   out, s);
      double hr[2];
      hipMemcpyAsync(hr, out, sizeof hr, hipMemcpyDeviceToHost, s);
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) return c->hip_fail(e, "iram residuals");
      const double al = std::hypot(lr[i], li[i]);
      res->resid[i] = std::sqrt(hr[0]) / (std::max(al, 1e-300) * std::sqrt(hr[1]));
    }
  }
  return res->nconv >= o.nev ? SA_OK : SA_NOT_CONVERGED;
}

}  // namespace
}  // namespace sa

using namespace sa;

extern "C" int sa_arnoldi_eigs(sa_ctx* const* ctxs, int nprob, const sa_eig_opts* o,
                               const double* const* v0_dev, sa_eig_result* res_host) {
  if (!ctxs || nprob < 1 || !ctxs[0]) return SA_EINVAL;
  Ctx* c0 = ctxs[0];
  if (!o || !v0_dev || !res_host) return c0->fail(SA_EINVAL, "sa_arnoldi_eigs: null argument");
  if (o->nev < 1 || o->nev > 32 || o->ncv < o->nev + 2 || o->ncv > MMAX)
    return c0->fail(SA_EINVAL, "sa_arnoldi_eigs: need 1 <= nev <= 32 and nev+2 <= ncv <= %d", MMAX);
  if (!(o->tol > 0) || o->max_restarts < 0) return c0->fail(SA_EINVAL, "sa_arnoldi_eigs: bad tol/max_restarts");
  if (std::fabs(o->sigma - o->mu) == 0.0) return c0->fail(SA_EINVAL, "sa_arnoldi_eigs: sigma == mu");
  const sa_gmres_opts& lin = o->lin;
  if (lin.restart < 1 || lin.augment < 0 || lin.restart + lin.augment > GMAX || !(lin.tol > 0) ||
      lin.max_matvec < 1 || (lin.prec == SA_MIXED && (!(lin.inner_tol > 0) || lin.max_outer < 1)))
    return c0->fail(SA_EINVAL, "sa_arnoldi_eigs: bad inner solver options (restart 1..%d, restart + augment <= %d, "
                               "tol > 0, max_matvec >= 1; MIXED: inner_tol > 0, max_outer >= 1)", GMAX, GMAX);
  bool same = true, distinct = true;
  for (int p = 0; p < nprob; ++p) {
    if (!ctxs[p] || !v0_dev[p]) return c0->fail(SA_EINVAL, "sa_arnoldi_eigs: null context or start vector");
    if (!ctxs[p]->has_base) return ctxs[p]->fail(SA_ESTATE, "sa_arnoldi_eigs: base state not set");
    if (o->lin.use_precond && !ctxs[p]->has_precond)
      return ctxs[p]->fail(SA_ESTATE, "sa_arnoldi_eigs: preconditioner not set up");
    same = same && ctxs[p]->stream == c0->stream;
    for (int q = 0; q < p; ++q) distinct = distinct && ctxs[q]->stream != ctxs[p]->stream && ctxs[q] != ctxs[p];
  }
  if (!same && !distinct)
    return c0->fail(SA_EINVAL, "sa_arnoldi_eigs: streams must be all one or pairwise distinct");
  std::vector<int> rcs(nprob, SA_OK);
  auto solve = [&](int p) {
    const auto t0 = std::chrono::steady_clock::now();
    rcs[p] = run_one(ctxs[p], *o, v0_dev[p], &res_host[p]);
    res_host[p].wall_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  if (same || nprob == 1) {
    for (int p = 0; p < nprob; ++p) {
      solve(p);
      if (rcs[p] < 0) break;
    }
  } else {
    // one host thread per problem, at most 16 at a time
    std::atomic<int> next{0};
    auto worker = [&]() {
      for (int p = next.fetch_add(1); p < nprob; p = next.fetch_add(1)) {
        if (hipSetDevice(ctxs[p]->device) != hipSuccess) {
          rcs[p] = ctxs[p]->fail(SA_EDEVICE, "sa_arnoldi_eigs: hipSetDevice failed");
          continue;
        }
        solve(p);
      }
    };
    const int nt = nprob < 16 ? nprob : 16;
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t) pool.emplace_back(worker);
    for (auto& th : pool) th.join();
  }
  int rc_all = SA_OK;
  for (int p = 0; p < nprob; ++p) {
    if (rcs[p] < 0) {
      if (p > 0) c0->err = "problem " + std::to_string(p) + ": " + ctxs[p]->err;
      return rcs[p];
    }
    if (rcs[p] > 0) rc_all = rcs[p];
  }
  return rc_all;
}
