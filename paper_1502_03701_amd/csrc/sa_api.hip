// C ABI of libsa: context, base state, operator application and the GMRES
// solvers of the Cayley systems.  Host code only orchestrates: every
// arithmetic step runs in the kernels of jv.hip, blas.hip, gmres_small.hip,
// arnoldi_small.hip and bjac.hip.
#include "sa_runtime.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>

using namespace sa;

namespace sa {

int Ctx::fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  err = buf;
  return code;
}

int Ctx::hip_fail(hipError_t e, const char* where) {
  return fail(e == hipErrorOutOfMemory ? SA_ENOMEM : SA_EDEVICE, "%s: %s", where,
              hipGetErrorString(e));
}

void* Ctx::buffer(const std::string& name, size_t bytes, bool zero) {
  if (arena) {
    auto at = arena->bufs.find(name);
    if (at != arena->bufs.end() && at->second.bytes >= bytes) return at->second.ptr;
    const size_t need = (bytes + 255) / 256 * 256;
    if (need > arena->cap - arena->used) return nullptr;
    void* p = arena->base + arena->used;
    arena->used += need;
    if (zero) zero_fill(p, need, stream);
    arena->bufs[name] = Buf{p, need};
    return p;
  }
  auto it = bufs.find(name);
  if (it != bufs.end() && it->second.bytes >= bytes) return it->second.ptr;
  if (it != bufs.end()) {
    drop_graphs();   // a cached graph may reference the old address
    hipStreamSynchronize(stream);
    hipFree(it->second.ptr);
    bufs.erase(it);
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes == 0 ? 256 : bytes) != hipSuccess) return nullptr;
  if (zero) hipMemsetAsync(p, 0, bytes, stream);
  bufs[name] = Buf{p, bytes};
  return p;
}

void Ctx::drop_graphs() {
  if (graphs.empty()) return;
  hipStreamSynchronize(stream);
  for (auto& g : graphs) hipGraphExecDestroy(g.exec);
  graphs.clear();
}

// Detect a base state of uniform thermodynamic state (p0 and s0 equal at
// every point, compared exactly) and classify the base-data fields the iso
// kernels read; fill the context's IsoBase records and op.iso.
static int setup_iso(Ctx* c) {
  OpParams& op = c->op;
  op.iso[0] = op.iso[1] = nullptr;
  c->iso = false;
  const int nd = op.ndim, nv = c->nv;
  const int nf = iso_fields(nd);
  // the iso kernels index the base data with 32-bit offsets
  if ((long long)(iso_fidx(nd, nf - 1) + 1) * op.npts >= (1LL << 31)) return SA_OK;
  int fidx[ISO_MAXF];
  for (int q = 0; q < nf; ++q) fidx[q] = iso_fidx(nd, q);
  int* flags = (int*)c->buffer("iso_flags", 3 * sizeof(int), false);
  if (!flags) return c->fail(SA_ENOMEM, "sa_base_set: out of device memory");
  hipError_t e = hipMemsetAsync(flags, 0, 3 * sizeof(int), c->stream);
  if (e == hipSuccess) e = launch_iso_classify(op, c->base64, c->bdata64, fidx, nf, flags, c->stream);
  int hf[3] = {0, 0, 0};
  double h[5] = {0, 0, 0, 0, 0};   // p0, s0, T0, T_p, T_s at point 0
  const long long np = op.npts;
  const long long off[5] = {0, (long long)(nv - 1) * np, (long long)nv * np, (long long)(nv + 1) * np,
                            (long long)(nv + 2) * np};
  if (e == hipSuccess) e = hipMemcpyAsync(hf, flags, sizeof hf, hipMemcpyDeviceToHost, c->stream);
  for (int q = 0; q < 5 && e == hipSuccess; ++q)
    e = hipMemcpyAsync(&h[q], c->base64 + off[q], sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "sa_base_set classify");
  if (hf[0]) return SA_OK;   // p0 or s0 varies: general kernels only
  const double p0 = h[0], T0 = h[2];
  const double S = op.suth;
  const double rho = p0 / (op.R * T0);
  const double mu0 = op.mu_ref * T0 * std::sqrt(T0) * (1.0 + S) / (T0 + S);
  const double muT = mu0 * (1.5 / T0 - 1.0 / (T0 + S));
  auto fill = [&](auto& ib, auto* bd) {
    using R = std::remove_reference_t<decltype(ib.Tp)>;
    ib.bd = bd;
    ib.gmask = ib.pmask = 0;
    for (int q = 0; q < nf; ++q) {
      if (!(hf[1] >> q & 1)) continue;           // identically zero
      if (hf[2] >> q & 1)
        ib.gmask |= 1u << q;
      else
        ib.pmask |= 1u << q;
    }
    ib.Tp = R(h[3]);
    ib.Ts = R(h[4]);
    ib.p0 = R(p0);
    ib.ip0 = R(1.0 / p0);
    ib.T0 = R(T0);
    ib.rho = R(rho);
    ib.irho = R(1.0 / rho);
    ib.irT = R(1.0 / (rho * T0));
    ib.mu0 = R(mu0);
    ib.muT = R(muT);
    ib.lam0 = R(op.cp / op.pr * mu0);
    ib.igam = R(1.0 / op.gamma);
    ib.icp = R(1.0 / op.cp);
  };
  fill(c->iso64, c->bdata64);
  fill(c->iso32, c->bdata32);
  c->iso = true;
  op.iso[0] = &c->iso64;
  op.iso[1] = &c->iso32;
  return SA_OK;
}

// Time each operator kernel variant on this problem (one warm-up and three
// timed launches, HIP events on the context's stream) and keep the fastest
// per precision.  Inputs are the base fields themselves (finite values of
// the right size); the output goes to a scratch buffer.
static int autotune_jv(Ctx* c) {
  if (std::getenv("SA_JV_AUTOTUNE") && std::strcmp(std::getenv("SA_JV_AUTOTUNE"), "0") == 0)
    return SA_OK;
  hipEvent_t ev0, ev1;
  if (hipEventCreate(&ev0) != hipSuccess) return c->fail(SA_EDEVICE, "autotune: event");
  if (hipEventCreate(&ev1) != hipSuccess) {
    hipEventDestroy(ev0);
    return c->fail(SA_EDEVICE, "autotune: event");
  }
  void* y = c->buffer("tune_y", sizeof(double) * c->n, false);
  int rc = y ? SA_OK : c->fail(SA_ENOMEM, "autotune: out of device memory");
  for (int pr = 0; pr < 2 && rc == SA_OK; ++pr) {
    if (c->jv_pinned[pr]) continue;
    float best = 0.0f;
    int best_v = -1;
    for (int v = 0; v < JV_NVARIANTS && rc == SA_OK; ++v) {
      if (jv_variant_is_iso(v) && !c->iso) {
        c->jv_tune_us[pr][v] = 0.0f;
        continue;
      }
      auto launch = [&]() -> hipError_t {
        if (pr == 0)
          return launch_jv<double>(c->op, c->base64, c->bdata64, c->base64, (double*)y, 1, 0.0, nullptr, c->stream, v);
        return launch_jv<float>(c->op, c->base32, c->bdata32, c->base32, (float*)y, 1, 0.0f, nullptr, c->stream, v);
      };
      hipError_t e = launch();
      if (e == hipSuccess) e = hipEventRecord(ev0, c->stream);
      for (int it = 0; it < 3 && e == hipSuccess; ++it) e = launch();
      if (e == hipSuccess) e = hipEventRecord(ev1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(ev1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
      if (e != hipSuccess) {
        rc = c->hip_fail(e, "autotune");
        break;
      }
      c->jv_tune_us[pr][v] = ms * 1000.0f / 3.0f;
      if (best_v < 0 || ms < best) {
        best = ms;
        best_v = v;
      }
    }
    if (rc == SA_OK) c->jv_variant[pr] = best_v;
  }
  hipEventDestroy(ev0);
  hipEventDestroy(ev1);
  return rc;
}

Ctx::~Ctx() {
  hipStreamSynchronize(stream);
  drop_graphs();
  if (cap_stream) hipStreamDestroy(cap_stream);
  for (auto& kv : bufs) hipFree(kv.second.ptr);
}

int gmres_check(Ctx* c, const sa_gmres_opts* o, int nshift, const double* sigma_host, const void* b_dev,
                const void* x_dev, const sa_gmres_info* info, const char* who) {
  if (!c->has_base) return c->fail(SA_ESTATE, "%s: call sa_base_set first", who);
  if (!o || !sigma_host || !b_dev || !x_dev || !info || nshift < 1)
    return c->fail(SA_EINVAL, "%s: null argument or nshift < 1", who);
  if (o->restart < 1 || o->restart > GMAX) return c->fail(SA_EINVAL, "%s: restart must be 1..%d", who, GMAX);
  if (o->augment < 0 || o->restart + o->augment > GMAX)
    return c->fail(SA_EINVAL, "%s: need augment >= 0 and restart + augment <= %d", who, GMAX);
  if (!(o->tol > 0) || o->max_matvec < 1) return c->fail(SA_EINVAL, "%s: bad tol or max_matvec", who);
  if (o->use_precond) {
    if (!c->has_precond) return c->fail(SA_ESTATE, "%s: preconditioner not set up", who);
    if (nshift != c->pc_nshift)
      return c->fail(SA_EINVAL, "%s: nshift must equal the preconditioner's shift count", who);
  }
  if (o->prec == SA_MIXED && (!(o->inner_tol > 0) || o->max_outer < 1))
    return c->fail(SA_EINVAL, "%s: MIXED needs inner_tol > 0 and max_outer >= 1", who);
  if (o->prec != SA_F64 && o->prec != SA_F32 && o->prec != SA_MIXED) return c->fail(SA_EINVAL, "%s: bad precision", who);
  return SA_OK;
}

int gmres_dispatch(Ctx* c, const sa_gmres_opts& o, int nshift, const double* sigma_host, const void* b_dev,
                   void* x_dev, sa_gmres_info* info) {
  // FP64 / FP32: all shifts advance in lockstep in the same launches
  if (o.prec == SA_F64)
    return solve_gmres<double>(c, o, nshift, sigma_host, (const double*)b_dev, (double*)x_dev,
                               o.use_precond ? 0 : -1, info);
  if (o.prec == SA_F32)
    return solve_gmres<float>(c, o, nshift, sigma_host, (const float*)b_dev, (float*)x_dev,
                              o.use_precond ? 0 : -1, info);
  int rc_all = SA_OK;
  for (int s = 0; s < nshift; ++s) {
    const long long off = (long long)s * c->n;
    const int rc = solve_ir(c, o, sigma_host[s], (const double*)b_dev + off, (double*)x_dev + off,
                            o.use_precond ? s : -1, &info[s]);
    if (rc < 0) return rc;
    if (rc > 0) rc_all = rc;
  }
  return rc_all;
}

}  // namespace sa

extern "C" {

const char* sa_version(void) { return "sa-mi355x 0.1 (gfx950)"; }

int sa_create(sa_ctx** out, void* hip_stream) {
  if (!out) return SA_EINVAL;
  *out = nullptr;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SA_EDEVICE;
  scratch_init(dev);
  auto* c = new (std::nothrow) sa_ctx();
  if (!c) return SA_ENOMEM;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->device = dev;
  *out = c;
  return SA_OK;
}

void sa_destroy(sa_ctx* ctx) { delete ctx; }

const char* sa_last_error(const sa_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int sa_base_set(sa_ctx* c, const sa_problem* pb, const double* q0_dev) {
  if (!c) return SA_EINVAL;
  if (!pb || !q0_dev) return c->fail(SA_EINVAL, "sa_base_set: null argument");
  if (pb->ndim != 2 && pb->ndim != 3) return c->fail(SA_EINVAL, "sa_base_set: ndim must be 2 or 3");
  const int nz = pb->ndim == 2 ? 1 : pb->n[2];
  if (pb->n[0] < 7 || pb->n[1] < 7 || (pb->ndim == 3 && nz < 7))
    return c->fail(SA_EINVAL, "sa_base_set: every axis needs at least 7 points");
  if (pb->ndim == 2 && pb->n[2] != 1) return c->fail(SA_EINVAL, "sa_base_set: 2D needs n[2] == 1");
  if (pb->bc_y != SA_BC_PERIODIC && pb->bc_y != SA_BC_WALL)
    return c->fail(SA_EINVAL, "sa_base_set: bad bc_y");
  if (pb->scheme != SA_SCHEME_EXPLICIT && pb->scheme != SA_SCHEME_COMPACT)
    return c->fail(SA_EINVAL, "sa_base_set: bad scheme");
  if (!(pb->mach > 0) || !(pb->gamma > 1) || !(pb->pr > 0) || !(pb->sutherland > 0))
    return c->fail(SA_EINVAL, "sa_base_set: mach, gamma, pr, sutherland must be positive (gamma > 1)");
  for (int a = 0; a < pb->ndim; ++a)
    if (!(pb->len[a] > 0)) return c->fail(SA_EINVAL, "sa_base_set: lengths must be positive");
  if (!(pb->stretch >= 0.0 && pb->stretch <= 20.0))
    return c->fail(SA_EINVAL, "sa_base_set: stretch must be in [0, 20]");
  if (pb->stretch > 0.0 && pb->bc_y != SA_BC_WALL)
    return c->fail(SA_EINVAL, "sa_base_set: grid stretching needs walls in y");
  OpParams& op = c->op;
  op.ndim = pb->ndim;
  op.nx = pb->n[0];
  op.ny = pb->n[1];
  op.nz = nz;
  op.bcy = pb->bc_y;
  op.npts = (long long)op.nx * op.ny * op.nz;
  op.ihx = op.nx / pb->len[0];
  op.ihy = (pb->bc_y == SA_BC_WALL ? (op.ny - 1) : op.ny) / pb->len[1];
  op.ihz = pb->ndim == 3 ? op.nz / pb->len[2] : 1.0;
  op.gamma = pb->gamma;
  op.R = 1.0 / (pb->gamma * pb->mach * pb->mach);
  op.p_ref = op.R;
  op.cp = pb->gamma * op.R / (pb->gamma - 1.0);
  op.mu_ref = pb->re > 0 ? 1.0 / pb->re : 0.0;
  op.suth = pb->sutherland;
  op.pr = pb->pr;
  op.scheme = pb->scheme;
  op.stretch = pb->stretch;
  op.cwork = nullptr;
  op.ctab64 = nullptr;
  op.ctab32 = nullptr;
  c->prob = *pb;
  c->nv = pb->ndim + 2;
  c->n = (long long)c->nv * op.npts;
  const size_t nf = (size_t)(c->nv + 3) * op.npts;
  c->has_base = false;
  c->has_precond = false;
  c->iso = false;
  op.iso[0] = op.iso[1] = nullptr;
  c->drop_graphs();
  c->base64 = (double*)c->buffer("base64", nf * sizeof(double));
  c->base32 = (float*)c->buffer("base32", nf * sizeof(float));
  const size_t nbd = (size_t)base_data_fields(op.ndim) * op.npts;
  c->bdata64 = (double*)c->buffer("bdata64", nbd * sizeof(double));
  c->bdata32 = (float*)c->buffer("bdata32", nbd * sizeof(float));
  if (!c->bdata64 || !c->bdata32) return c->fail(SA_ENOMEM, "sa_base_set: out of device memory");
  int* flag = (int*)c->buffer("flag", sizeof(int));
  if (!c->base64 || !c->base32 || !flag) return c->fail(SA_ENOMEM, "sa_base_set: out of device memory");
  hipError_t e = hipMemcpyAsync(c->base64, q0_dev, (size_t)c->n * sizeof(double), hipMemcpyDeviceToDevice,
                                c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "sa_base_set copy");
  hipMemsetAsync(flag, 0, sizeof(int), c->stream);
  e = launch_base_derive(op, c->base64, c->base32, flag, c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "sa_base_set derive");
  int hflag = 0;
  hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "sa_base_set sync");
  if (hflag) return c->fail(SA_ENONFINITE, "sa_base_set: q0 has NaN/Inf or non-positive pressure");
  {
    // per-row y metric [m1 | m2 | m4] (see OpParams), double and float
    double* y64 = (double*)c->buffer("ymet64", sizeof(double) * 3 * op.ny, false);
    float* y32 = (float*)c->buffer("ymet32", sizeof(float) * 3 * op.ny, false);
    if (!y64 || !y32) return c->fail(SA_ENOMEM, "sa_base_set: out of device memory");
    std::vector<double> h(3 * (size_t)op.ny);
    const int ny = op.ny;
    for (int j = 0; j < ny; ++j) {
      if (op.stretch > 0.0) {
        // y(eta) = (Ly/2) sinh(beta eta)/sinh(beta), eta_j = -1 + 2 j/(ny-1)
        const double b = op.stretch, eta = -1.0 + 2.0 * j / (ny - 1), heta = 2.0 / (ny - 1);
        const double half = 0.5 * pb->len[1] / std::sinh(b);
        const double yp = half * b * std::cosh(b * eta), ypp = half * b * b * std::sinh(b * eta);
        h[j] = 1.0 / (heta * yp);
        h[ny + j] = h[j] * h[j];
        h[2 * ny + j] = -ypp / (yp * yp);
      } else {
        h[j] = op.ihy;
        h[ny + j] = op.ihy * op.ihy;
        h[2 * ny + j] = 0.0;
      }
    }
    std::vector<float> h32(h.begin(), h.end());
    e = hipMemcpy(y64, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(y32, h32.data(), sizeof(float) * h32.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return c->hip_fail(e, "sa_base_set y metric");
    op.ym64 = y64;
    op.ym32 = y32;
  }
  if (op.scheme == SA_SCHEME_COMPACT) {
    // workspace (one system) and Thomas tables of the compact derivatives
    const size_t nt = compact_table_elems(op);
    op.cwork = c->buffer("cwork", sizeof(double) * compact_work_elems(op.ndim, op.npts), false);
    double* t64 = (double*)c->buffer("ctab64", sizeof(double) * nt, false);
    float* t32 = (float*)c->buffer("ctab32", sizeof(float) * nt, false);
    if (!op.cwork || !t64 || !t32) return c->fail(SA_ENOMEM, "sa_base_set: out of device memory");
    std::vector<double> h64;
    compact_tables(op, h64);
    std::vector<float> h32(h64.begin(), h64.end());
    e = hipMemcpy(t64, h64.data(), sizeof(double) * nt, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t32, h32.data(), sizeof(float) * nt, hipMemcpyHostToDevice);
    if (e != hipSuccess) return c->hip_fail(e, "sa_base_set tables");
    op.ctab64 = t64;
    op.ctab32 = t32;
  }
  // discrete derivatives of the base state, once per base state
  e = op.scheme == SA_SCHEME_COMPACT ? launch_base_data_compact(op, c->base64, c->bdata64, c->stream)
                                     : launch_base_data(op, c->base64, c->bdata64, c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "sa_base_set base data");
  cast_d2f((long long)nbd, c->bdata64, c->bdata32, nullptr, c->stream);
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "sa_base_set base data sync");
  // the uniform-state and autotuned kernels are explicit-difference kernels
  if (op.scheme == SA_SCHEME_EXPLICIT) {
    int rc = op.stretch > 0.0 ? SA_OK : setup_iso(c);   // the uniform-state kernels take uniform rows
    if (rc != SA_OK) return rc;
    rc = autotune_jv(c);
    if (rc != SA_OK) return rc;
  } else {
    for (int pr = 0; pr < 2; ++pr)
      for (int v = 0; v < JV_NVARIANTS; ++v) c->jv_tune_us[pr][v] = 0.0f;
  }
  c->has_base = true;
  return SA_OK;
}

int sa_set_jv_variant(sa_ctx* c, sa_prec prec, int variant) {
  if (!c) return SA_EINVAL;
  if (prec != SA_F64 && prec != SA_F32) return c->fail(SA_EINVAL, "sa_set_jv_variant: precision must be F64 or F32");
  if (variant < -1 || variant >= JV_NVARIANTS) return c->fail(SA_EINVAL, "sa_set_jv_variant: bad variant %d", variant);
  const int pr = prec == SA_F64 ? 0 : 1;
  c->drop_graphs();
  c->jv_variant[pr] = variant;
  c->jv_pinned[pr] = variant >= 0;
  return SA_OK;
}

int sa_get_jv_variant(const sa_ctx* c, sa_prec prec, float* times_us) {
  if (!c || (prec != SA_F64 && prec != SA_F32)) return SA_EINVAL;
  const int pr = prec == SA_F64 ? 0 : 1;
  if (times_us)
    for (int v = 0; v < JV_NVARIANTS; ++v) times_us[v] = c->jv_tune_us[pr][v];
  return c->jv_variant[pr];
}

int sa_op_apply(sa_ctx* c, sa_prec prec, int nrhs, const void* x_dev, void* y_dev, double shift) {
  if (!c) return SA_EINVAL;
  if (!c->has_base) return c->fail(SA_ESTATE, "sa_op_apply: call sa_base_set first");
  if (nrhs < 1 || !x_dev || !y_dev) return c->fail(SA_EINVAL, "sa_op_apply: bad nrhs or null pointer");
  hipError_t e;
  if (prec == SA_F64)
    e = c->jv<double>((const double*)x_dev, (double*)y_dev, nrhs, shift, nullptr);
  else if (prec == SA_F32)
    e = c->jv<float>((const float*)x_dev, (float*)y_dev, nrhs, shift, nullptr);
  else
    return c->fail(SA_EINVAL, "sa_op_apply: precision must be SA_F64 or SA_F32");
  if (e != hipSuccess) return c->hip_fail(e, "sa_op_apply");
  return SA_OK;
}

int sa_gmres_solve(sa_ctx* c, const sa_gmres_opts* o, int nshift, const double* sigma_host,
                   const void* b_dev, void* x_dev, sa_gmres_info* info) {
  if (!c) return SA_EINVAL;
  const int rc = gmres_check(c, o, nshift, sigma_host, b_dev, x_dev, info, "sa_gmres_solve");
  if (rc != SA_OK) return rc;
  return gmres_dispatch(c, *o, nshift, sigma_host, b_dev, x_dev, info);
}

}  // extern "C"
