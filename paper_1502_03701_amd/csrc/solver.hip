// Restarted GMRES (Section "Iterative solvers") for (J - sigma_s I) x_s = b_s,
// with classical Gram-Schmidt applied twice and optional right block-Jacobi
// preconditioning in the flexible form (the preconditioned directions are
// kept), plus the FP64-outer / FP32-inner iterative refinement form.
//
// Several systems (Cayley shifts) advance in lockstep: every kernel of an
// Arnoldi step handles all systems in one launch, each system with its own
// basis, device state and active flag.  One cycle is enqueued in full:
// residual, then per step the preconditioner, the operator, the two
// Gram-Schmidt passes and the Givens update.  The Givens kernel clears a
// system's active flag on convergence, breakdown or budget exhaustion, so the
// host synchronises once per cycle to read the states.
#include <algorithm>
#include <cmath>
#include <vector>

#include "sa_runtime.h"

namespace sa {
namespace {

hipError_t read_tails(GState* st, int nsys, std::vector<GTail>& h, hipStream_t s) {
  h.resize(nsys);
  hipError_t e = hipSuccess;
  for (int i = 0; i < nsys && e == hipSuccess; ++i)
    e = hipMemcpyAsync(&h[i], &st[i].t, sizeof(GTail), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

template <typename R>
const R* base_of(const Ctx* c) {
  return nullptr;
}
template <>
const double* base_of<double>(const Ctx* c) {
  return c->base64;
}
template <>
const float* base_of<float>(const Ctx* c) {
  return c->base32;
}
template <typename R>
const R* bdata_of(const Ctx* c) {
  return nullptr;
}
template <>
const double* bdata_of<double>(const Ctx* c) {
  return c->bdata64;
}
template <>
const float* bdata_of<float>(const Ctx* c) {
  return c->bdata32;
}

}  // namespace

// Key of a cycle graph: everything the captured launches bake in.
template <typename T>
void put(std::vector<unsigned char>& k, const T& v) {
  const unsigned char* b = reinterpret_cast<const unsigned char*>(&v);
  k.insert(k.end(), b, b + sizeof(T));
}

hipGraphExec_t find_graph(Ctx* c, const std::vector<unsigned char>& key) {
  for (auto& g : c->graphs)
    if (g.key == key) return g.exec;
  return nullptr;
}

constexpr size_t MAX_GRAPHS = 16;

template <typename R>
int solve_gmres(Ctx* c, const sa_gmres_opts& o, int nsys, const double* sigma, const R* b, R* x, int pc_shift0,
                sa_gmres_info* info, const std::string& tag, bool io_stable, bool x0_zero) {
  hipStream_t s = c->stream;
  const long long n = c->n;
  const int m = o.restart;
  const int k = o.augment;            // LGMRES: error approximations kept (0: GMRES)
  const bool pc = pc_shift0 >= 0;
  const bool graph = o.use_graph != 0;
  const long long sv = n * (m + k + 1);   // basis stride between systems
  R* V = (R*)c->buffer(tag + "V", sizeof(R) * sv * nsys);
  R* Z = pc ? (R*)c->buffer(tag + "Z", sizeof(R) * sv * nsys) : V;
  // LGMRES state per system: k corrections (newest first), their images
  // under A, the residual at the start of the cycle, x at its start
  const long long sa = n * (k > 0 ? k : 1);
  R* AUG = k ? (R*)c->buffer(tag + "aug", sizeof(R) * sa * nsys, false) : nullptr;
  R* AUGA = k ? (R*)c->buffer(tag + "augA", sizeof(R) * sa * nsys, false) : nullptr;
  R* RPREV = k ? (R*)c->buffer(tag + "rprev", sizeof(R) * n * nsys, false) : nullptr;
  R* XOLD = k ? (R*)c->buffer(tag + "xold", sizeof(R) * n * nsys, false) : nullptr;
  R* T = (R*)c->buffer(tag + "T", sizeof(R) * n * nsys, false);
  GState* st = (GState*)c->buffer(tag + "state", sizeof(GState) * nsys);
  double* sig = (double*)c->buffer(tag + "sigma", sizeof(double) * nsys, false);
  Blas<R> bl;
  bl.partial = (double*)c->buffer(tag + "partial", sizeof(double) * RED_BLOCKS * PARTIAL_LD * nsys);
  bl.ticket = (int*)c->buffer(tag + "ticket", sizeof(int) * nsys);
  // a captured cycle works on context-owned copies of b and x, so that one
  // graph serves every caller buffer; io_stable: b and x are themselves
  // context-owned buffers that every call passes again (the refinement
  // loop's), and the cycle works on them directly
  const bool copy_io = graph && !io_stable;
  R* X = copy_io ? (R*)c->buffer(tag + "X", sizeof(R) * n * nsys, false) : x;
  R* B = copy_io ? (R*)c->buffer(tag + "B", sizeof(R) * n * nsys, false) : const_cast<R*>(b);
  if (!V || !Z || !T || !st || !sig || !bl.partial || !bl.ticket || !X || !B ||
      (k && (!AUG || !AUGA || !RPREV || !XOLD)))
    return c->fail(SA_ENOMEM, "gmres: out of device memory");
  if (graph && !c->cap_stream) {
    hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return c->hip_fail(e, "gmres capture stream");
  }
  hipError_t e = hipMemcpyAsync(sig, sigma, sizeof(double) * nsys, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && copy_io) e = hipMemcpyAsync(X, x, sizeof(R) * n * nsys, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && copy_io) e = hipMemcpyAsync(B, b, sizeof(R) * n * nsys, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return c->hip_fail(e, "gmres inputs");
  const R* base = base_of<R>(c);
  const R* bdata = bdata_of<R>(c);
  const int* act = &st->t.active;
  Batch bb;                       // basis operations
  bb.nsys = nsys;
  bb.vec = sv;
  bb.res = GS_DOUBLES;
  bb.act = GS_INTS;
  Batch bn = bb;                  // vectors one after another (b, x)
  bn.vec = n;
  Batch bx = bb;                  // x += Z y: basis stride for Z, n for x
  bx.wvec = n;

  const int* upd = &st->t.have_update;
  // r = b - (J - sigma I) x -> V_s[:,0]; with LGMRES the image of the last
  // correction, A dx = r_prev - r; beta, convergence and budget tests
  // zero_x: x is known to be zero (the first cycle of an x0_zero solve): the
  // residual is b, no operator product
  auto start_cycle = [&](hipStream_t q, int naug, bool zero_x = false) -> hipError_t {
    if (!zero_x) {
      hipError_t r =
          launch_jv_batch<R>(c->op, base, bdata, X, T, nsys, n, n, sigma, sig, nullptr, 0, q, c->variant_of<R>());
      if (r != hipSuccess) return r;
    }
    bl.residual(n, B, zero_x ? nullptr : T, V, &st->t.rnorm2, nullptr, q, bb, n, n);
    if (k) bl.lincomb(n, nsys, RPREV, n, 1.0, V, sv, -1.0, AUGA, sa, upd, GS_INTS, q);
    gstate_cycle_start(st, nsys, q, naug, zero_x ? 0 : 1);
    return hipGetLastError();
  };
  // one Arnoldi step on direction zj (null: the step's w is already in place)
  auto arnoldi_step = [&](hipStream_t q, int j, const R* zj) -> hipError_t {
    R* w = V + (long long)(j + 1) * n;
    if (zj) {
      hipError_t r = launch_jv_batch<R>(c->op, base, bdata, zj, w, nsys, sv, sv, sigma, sig, act, GS_INTS, q,
                                        c->variant_of<R>());
      if (r != hipSuccess) return r;
    }
    // CGS pass 1: d1 = V[0..j]^T w and ||w||^2
    bl.multidot(n, V, n, j + 2, w, st->d1, false, act, q, bb);
    // pass 2: w -= V d1, d2 = V^T w
    bl.update(n, V, n, j + 1, st->d1, -1.0, w, w, 1, st->d2, false, act, q, bb);
    // pass 3: w -= V d2, wn2 = ||w||^2, then the Givens step (fused when
    // the reduction finishes inside the kernel)
    if (!bl.update(n, V, n, j + 1, st->d2, -1.0, w, w, 2, &st->wn2, false, act, q, bb, st, j))
      gstate_step(st, nsys, j, q);
    bl.scale(n, w, w, &st->t.inv, act, q, bb);
    return hipGetLastError();
  };
  // m Krylov steps, naug augmentation steps, the least-squares solve and
  // x += Z y (+ AUG y_aug); LGMRES then stores the correction
  auto arnoldi_cycle = [&](hipStream_t q, int naug) -> hipError_t {
    if (k) bl.lincomb(n, nsys, V, sv, 1.0, V, sv, 0.0, RPREV, n, act, GS_INTS, q);
    bl.scale(n, V, V, &st->t.inv, act, q, bb);
    for (int j = 0; j < m; ++j) {
      R* vj = V + (long long)j * n;
      const R* zj = vj;
      if (pc) {
        R* zz = Z + (long long)j * n;
        hipError_t r = precond_apply<R>(c, pc_shift0, nsys, vj, zz, act, 1, sv, GS_INTS, q);
        if (r != hipSuccess) return r;
        zj = zz;
      }
      hipError_t r = arnoldi_step(q, j, zj);
      if (r != hipSuccess) return r;
    }
    for (int i = 0; i < naug; ++i) {
      // direction: correction i; its image is stored, so w needs no product
      bl.lincomb(n, nsys, AUGA + (long long)i * n, sa, 1.0, AUGA + (long long)i * n, sa, 0.0,
                 V + (long long)(m + i + 1) * n, sv, act, GS_INTS, q);
      hipError_t r = arnoldi_step(q, m + i, nullptr);
      if (r != hipSuccess) return r;
    }
    gstate_finish(st, nsys, q);
    if (k) bl.lincomb(n, nsys, X, n, 1.0, X, n, 0.0, XOLD, n, upd, GS_INTS, q);
    // x += Z y  (Z = V without preconditioning)
    bl.update(n, Z, n, m, st->y, 1.0, X, X, 0, nullptr, false, upd, q, bx);
    if (naug) {
      Batch ba = bx;
      ba.vec = sa;
      bl.update(n, AUG, n, naug, st->y + m, 1.0, X, X, 0, nullptr, false, upd, q, ba);
    }
    if (k) {
      // keep the newest k corrections: shift, then AUG_0 = x - x_old
      for (int i = naug < k ? naug : k - 1; i >= 1; --i) {
        bl.lincomb(n, nsys, AUG + (long long)(i - 1) * n, sa, 1.0, AUG + (long long)(i - 1) * n, sa, 0.0,
                   AUG + (long long)i * n, sa, upd, GS_INTS, q);
        bl.lincomb(n, nsys, AUGA + (long long)(i - 1) * n, sa, 1.0, AUGA + (long long)(i - 1) * n, sa, 0.0,
                   AUGA + (long long)i * n, sa, upd, GS_INTS, q);
      }
      bl.lincomb(n, nsys, X, n, 1.0, XOLD, n, -1.0, AUG, sa, upd, GS_INTS, q);
    }
    return hipGetLastError();
  };

  // one graph = one cycle followed by the next cycle's start; with LGMRES
  // the cycle's shape depends on the corrections already stored (naug)
  auto get_graph = [&](int naug, hipGraphExec_t& exec) -> int {
    exec = nullptr;
    std::vector<unsigned char> key;
    put(key, (int)sizeof(R));
    put(key, nsys);
    put(key, m);
    put(key, k);
    put(key, naug);
    put(key, pc_shift0);
    put(key, n);
    put(key, c->variant_of<R>());
    for (const void* ptr : {(const void*)V, (const void*)Z, (const void*)T, (const void*)st, (const void*)sig,
                            (const void*)bl.partial, (const void*)bl.ticket, (const void*)X, (const void*)B, (const void*)base,
                            (const void*)bdata, (const void*)c->pc_lu, (const void*)c->pc_perm})
      put(key, ptr);
    for (const void* ptr : {(const void*)AUG, (const void*)AUGA, (const void*)RPREV, (const void*)XOLD}) put(key, ptr);
    put(key, c->pc_kind);
    for (const void* ptr : {(const void*)c->fp_U, (const void*)c->fp_L, (const void*)c->fp_piv,
                            (const void*)c->fp_specA64, (const void*)c->fp_specB64, (const void*)c->fp_specA32,
                            (const void*)c->fp_specB32})
      put(key, ptr);
    for (int i = 0; i < nsys; ++i) put(key, sigma[i]);
    exec = find_graph(c, key);
    if (!exec) {
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return c->hip_fail(e, "gmres begin capture");
      hipError_t ec = arnoldi_cycle(c->cap_stream, naug);
      if (ec == hipSuccess) ec = start_cycle(c->cap_stream, naug < k ? naug + 1 : k);
      e = hipStreamEndCapture(c->cap_stream, &g);
      if (ec != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return c->hip_fail(ec, "gmres capture");
      }
      if (e != hipSuccess) return c->hip_fail(e, "gmres end capture");
      e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) return c->hip_fail(e, "gmres graph instantiate");
      if (c->graphs.size() >= MAX_GRAPHS) {
        hipStreamSynchronize(s);
        hipGraphExecDestroy(c->graphs.front().exec);
        c->graphs.erase(c->graphs.begin());
      }
      c->graphs.push_back(CycleGraph{key, exec});
    }
    return SA_OK;
  };

  for (int i = 0; i < nsys; ++i) info[i] = sa_gmres_info{};
  gstate_init(st, nsys, o.tol, m, o.max_matvec, s);
  bl.nrm2sq(n, B, &st->t.bnorm2, nullptr, s, bn);
  gstate_set_bnorm(st, nsys, s);
  e = start_cycle(s, 0, x0_zero);
  if (e != hipSuccess) return c->hip_fail(e, "gmres residual");
  std::vector<GTail> h;
  int cycles = 0;
  for (;;) {
    e = read_tails(st, nsys, h, s);
    if (e != hipSuccess) return c->hip_fail(e, "gmres status");
    bool any_active = false;
    for (int i = 0; i < nsys; ++i) {
      info[i].iters = h[i].iters;
      info[i].matvecs = h[i].matvecs;
      info[i].cycles = cycles;
      info[i].relres = h[i].relres;
      info[i].precond_applies = pc ? h[i].krylov : 0;
      if (h[i].nonfinite) {
        info[i].status = SA_ENONFINITE;
        return c->fail(SA_ENONFINITE, "gmres: non-finite residual (system %d)", i);
      }
      info[i].status = h[i].converged ? SA_OK : SA_NOT_CONVERGED;
      any_active = any_active || h[i].active;
    }
    if (!any_active) break;
    const int naug = cycles < k ? cycles : k;   // corrections stored so far
    if (graph) {
      hipGraphExec_t exec;
      const int rc = get_graph(naug, exec);
      if (rc != SA_OK) return rc;
      e = hipGraphLaunch(exec, s);
      if (e != hipSuccess) return c->hip_fail(e, "gmres graph launch");
    } else {
      e = arnoldi_cycle(s, naug);
      if (e == hipSuccess) e = start_cycle(s, naug < k ? naug + 1 : k);
      if (e != hipSuccess) return c->hip_fail(e, "gmres cycle");
    }
    ++cycles;
  }
  if (copy_io) {
    e = hipMemcpyAsync(x, X, sizeof(R) * n * nsys, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return c->hip_fail(e, "gmres solution");
  }
  bool all = true;
  for (int i = 0; i < nsys; ++i) all = all && info[i].status == SA_OK;
  return all ? SA_OK : SA_NOT_CONVERGED;
}

template int solve_gmres<double>(Ctx*, const sa_gmres_opts&, int, const double*, const double*, double*, int,
                                 sa_gmres_info*, const std::string&, bool, bool);
template int solve_gmres<float>(Ctx*, const sa_gmres_opts&, int, const double*, const float*, float*, int,
                                sa_gmres_info*, const std::string&, bool, bool);

size_t gmres_workspace_bytes(const Ctx* c, const sa_gmres_opts& o, int nshift) {
  auto r = [](size_t b) -> size_t { return (b + 255) / 256 * 256; };
  const size_t n = (size_t)c->n;
  // the buffers solve_gmres names, without the copies of b and x that only
  // captured cycles use
  auto gm = [&](size_t es, size_t nsys, size_t m, size_t k, bool pc) -> size_t {
    const size_t sv = n * (m + k + 1);
    size_t t = r(es * sv * nsys);                                   // V
    if (pc) t += r(es * sv * nsys);                                 // Z
    if (k) t += 2 * r(es * n * k * nsys) + 2 * r(es * n * nsys);   // aug, augA, rprev, xold
    t += r(es * n * nsys);                                          // T
    t += r(sizeof(GState) * nsys) + r(sizeof(double) * nsys);       // state, sigma
    t += r(sizeof(double) * RED_BLOCKS * PARTIAL_LD * nsys) + r(sizeof(int) * nsys);   // partial, ticket
    return t;
  };
  const bool pc = o.use_precond != 0;
  if (o.prec == SA_F64) return gm(sizeof(double), nshift, o.restart, o.augment, pc);
  if (o.prec == SA_F32) return gm(sizeof(float), nshift, o.restart, o.augment, pc);
  // refinement: one shift at a time, its FP64 buffers plus one FP32 solve
  return 2 * r(sizeof(double) * n) + 2 * r(sizeof(float) * n) + r(sizeof(GState)) +
         r(sizeof(double) * RED_BLOCKS * PARTIAL_LD) + r(sizeof(int)) + gm(sizeof(float), 1, o.restart, o.augment, pc);
}

// Iterative refinement: FP64 residual and update, FP32 GMRES on the scaled
// residual equation r/||r||, solved to inner_tol relative, or only as far as
// the outer tolerance still requires (so the last sweep does not overshoot).
int solve_ir(Ctx* c, const sa_gmres_opts& o, double sigma, const double* b, double* x, int pc_shift,
             sa_gmres_info* info, bool x0_zero) {
  hipStream_t s = c->stream;
  const long long n = c->n;
  double* r = (double*)c->buffer("ir_r", sizeof(double) * n);
  double* y = (double*)c->buffer("ir_y", sizeof(double) * n);
  float* r32 = (float*)c->buffer("ir_r32", sizeof(float) * n);
  float* d32 = (float*)c->buffer("ir_d32", sizeof(float) * n);
  GState* st = (GState*)c->buffer("ir_state", sizeof(GState));
  Blas<double> bl;
  bl.partial = (double*)c->buffer("ir_partial", sizeof(double) * RED_BLOCKS * PARTIAL_LD);
  bl.ticket = (int*)c->buffer("ir_ticket", sizeof(int));
  Blas<float> bl32;
  bl32.partial = bl.partial;
  bl32.ticket = bl.ticket;
  if (!r || !y || !r32 || !d32 || !st || !bl.partial || !bl.ticket)
    return c->fail(SA_ENOMEM, "ir: out of device memory");
  *info = sa_gmres_info{};
  // the outer state only tracks ||b||, ||r|| and the tolerance; no budget
  gstate_init(st, 1, o.tol, 1, (long long)1 << 62, s);
  bl.nrm2sq(n, b, &st->t.bnorm2, nullptr, s);
  gstate_set_bnorm(st, 1, s);
  sa_gmres_opts in = o;
  in.prec = SA_F32;
  in.tol = o.inner_tol;
  long long inner_mv = 0, inner_it = 0, inner_pc = 0;
  int inner_cycles = 0;
  hipError_t e;
  std::vector<GTail> h;
  for (int outer = 0;; ++outer) {
    const bool zero_x = x0_zero && outer == 0;   // r = b, no product
    if (!zero_x) {
      e = c->jv<double>(x, y, 1, sigma, nullptr);
      if (e != hipSuccess) return c->hip_fail(e, "ir residual");
    }
    bl.residual(n, b, zero_x ? nullptr : y, r, &st->t.rnorm2, nullptr, s);
    gstate_cycle_start(st, 1, s, 0, zero_x ? 0 : 1);  // beta = ||r||, inv = 1/||r||, converged flag
    e = read_tails(st, 1, h, s);
    if (e != hipSuccess) return c->hip_fail(e, "ir status");
    info->outer = outer;
    info->relres = h[0].relres;
    info->iters = inner_it;
    info->matvecs = inner_mv + h[0].matvecs;
    info->cycles = inner_cycles;
    info->precond_applies = inner_pc;
    if (h[0].nonfinite) {
      info->status = SA_ENONFINITE;
      return c->fail(SA_ENONFINITE, "ir: non-finite residual");
    }
    if (h[0].converged) {
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
    // the last sweeps need only close the remaining gap: ask the inner solve
    // for max(inner_tol, tol ||b|| / (2 ||r||)), never looser than 1/2
    in.tol = std::min(0.5, std::max(o.inner_tol, 0.5 * o.tol / h[0].relres));
    int rc = solve_gmres<float>(c, in, 1, &sigma, r32, d32, pc_shift, &ii, "ir32", true, true);
    if (rc < 0) return rc;
    inner_mv += ii.matvecs;
    inner_it += ii.iters;
    inner_pc += ii.precond_applies;
    inner_cycles += ii.cycles;
    // x += ||r|| d
    axpy_f2d(n, d32, x, &st->t.beta, s);
  }
}

}  // namespace sa
