// Tangent-linear Navier-Stokes operator: y = (J(q0) - shift I) x.
//
// J is the exact derivative of the discrete right-hand side N(q) of the
// compressible Navier-Stokes equations in (p, u_i, s) form (Section
// "Governing equations", eq. navier_stokes), i.e. the operator N_lin that
// the Frechet quotient of eq. frechet approximates.  The discretisation:
//   * explicit central differences, 6th order in the interior, 4th and 2nd
//     order on the second and first rows next to a wall; mixed derivatives
//     are products of first differences;
//   * viscous terms in expanded form, d_j tau_ij = mu L u_i + mu/3 G_i +
//     mu'(T)[D_j T (D_j u_i + D_i u_j) - 2/3 D_i T D_k u_k] with
//     G_i = D2_i u_i + sum_{j!=i} D_i D_j u_j, heat flux lambda L T +
//     lambda'(T) |D T|^2, dissipation mu (2 s_ij s_ij - 2/3 s_kk^2);
//   * the pressure equation with the material derivative and the heat
//     terms (gamma-1)(Q+Phi); the entropy equation with +(Q+Phi)/(rho T);
//   * Sutherland viscosity, lambda = c_p mu/Pr, ideal gas.
// Linearisation: every product is differentiated by the product rule; the
// temperature perturbation T' = T_p p' + T_s s' is formed pointwise before
// it is differentiated; base-state derivatives are the discrete ones.
#include <cstdlib>
#include <cstring>

#include "jv_common.h"

namespace sa {
namespace {

// Field access around one point.  Variables 0..ND+1 are p, u_i, s; ND+2 is T.
// PERT: values come from the perturbation x (zero on wall rows), T' is formed
// from the base fields T_p, T_s.  !PERT: base fields, T from the T0 field.
template <typename R, int ND, bool PERT>
struct Acc {
  const R* base;
  const R* x;
  long long npts;
  int nx, ny, nz, bcy;
  int i, j, k;

  __device__ __forceinline__ long long at(int di, int dj, int dk, bool& wall) const {
    int ii = i + di;
    ii = ii < 0 ? ii + nx : (ii >= nx ? ii - nx : ii);
    int jj = j + dj;
    if (bcy == 0) {
      jj = jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj);
      wall = false;
    } else {
      jj = jj < 0 ? 0 : (jj >= ny ? ny - 1 : jj);   // clamped: coefficient is 0 there
      wall = (jj == 0 || jj == ny - 1);
    }
    int kk = 0;
    if (ND == 3) {
      kk = k + dk;
      kk = kk < 0 ? kk + nz : (kk >= nz ? kk - nz : kk);
    }
    return ((long long)kk * ny + jj) * nx + ii;
  }

  __device__ __forceinline__ R operator()(int f, int di, int dj, int dk) const {
    bool wall;
    long long id = at(di, dj, dk, wall);
    if (!PERT) return base[(long long)f * npts + id];
    if (wall) return R(0);
    if (f < ND + 2) return x[(long long)f * npts + id];
    // T' = T_p p' + T_s s'
    const R tp = base[(long long)(ND + 3) * npts + id];
    const R ts = base[(long long)(ND + 4) * npts + id];
    return tp * x[id] + ts * x[(long long)(ND + 1) * npts + id];
  }
};

template <typename R, int ND, bool PERT>
__device__ __forceinline__ R d1(const Acc<R, ND, PERT>& A, int f, int a, const Axis<R>& ax, R ih) {
  R acc = R(0);
#pragma unroll
  for (int m = 1; m <= 3; ++m) {
    const int dx = a == 0 ? m : 0, dy = a == 1 ? m : 0, dz = a == 2 ? m : 0;
    acc += ax.c1[m - 1] * (A(f, dx, dy, dz) - A(f, -dx, -dy, -dz));
  }
  return acc * ih;
}

template <typename R, int ND, bool PERT>
__device__ __forceinline__ R d2(const Acc<R, ND, PERT>& A, int f, int a, const Axis<R>& ax, R ih) {
  R acc = ax.c0 * A(f, 0, 0, 0);
#pragma unroll
  for (int m = 1; m <= 3; ++m) {
    const int dx = a == 0 ? m : 0, dy = a == 1 ? m : 0, dz = a == 2 ? m : 0;
    acc += ax.c2[m - 1] * (A(f, dx, dy, dz) + A(f, -dx, -dy, -dz));
  }
  return acc * (ih * ih);
}

// D_a D_b f (a != b) as the tensor product of the two first differences.
template <typename R, int ND, bool PERT>
__device__ __forceinline__ R dmix(const Acc<R, ND, PERT>& A, int f, int a, int b,
                                  const Axis<R>& axa, const Axis<R>& axb, R iha, R ihb) {
  R acc = R(0);
#pragma unroll
  for (int m = 1; m <= 3; ++m) {
    R inner = R(0);
#pragma unroll
    for (int n = 1; n <= 3; ++n) {
      int o1[3] = {0, 0, 0}, o2[3] = {0, 0, 0};
      o1[a] = m;
      o2[b] = n;
      const R pp = A(f, o1[0] + o2[0], o1[1] + o2[1], o1[2] + o2[2]);
      const R pm = A(f, o1[0] - o2[0], o1[1] - o2[1], o1[2] - o2[2]);
      const R mp = A(f, -o1[0] + o2[0], -o1[1] + o2[1], -o1[2] + o2[2]);
      const R mm = A(f, -o1[0] - o2[0], -o1[1] - o2[1], -o1[2] - o2[2]);
      inner += axb.c1[n - 1] * ((pp - pm) - (mp - mm));
    }
    acc += axa.c1[m - 1] * inner;
  }
  return acc * (iha * ihb);
}

template <typename R, int ND, bool PERT>
__device__ __forceinline__ void gather(Pt<R, ND>& P, const Acc<R, ND, PERT>& A, const Axis<R>* ax,
                                       const R* ih) {
#pragma unroll
  for (int f = 0; f < ND + 3; ++f) {
    P.q[f] = A(f, 0, 0, 0);
#pragma unroll
    for (int a = 0; a < ND; ++a) P.D[f][a] = d1(A, f, a, ax[a], ih[a]);
  }
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    R L = R(0);
    R d2ii = R(0);
#pragma unroll
    for (int a = 0; a < ND; ++a) {
      const R v = d2(A, 1 + i, a, ax[a], ih[a]);
      L += v;
      if (a == i) d2ii = v;
    }
    P.Lu[i] = L;
    R g = d2ii;
#pragma unroll
    for (int jv = 0; jv < ND; ++jv)
      if (jv != i) g += dmix(A, 1 + jv, i, jv, ax[i], ax[jv], ih[i], ih[jv]);
    P.G[i] = g;
  }
  R LT = R(0);
#pragma unroll
  for (int a = 0; a < ND; ++a) LT += d2(A, ND + 2, a, ax[a], ih[a]);
  P.LT = LT;
}

template <typename R, int ND>
__global__ void __launch_bounds__(256) jv_direct_kernel(OpParams op, const R* __restrict__ base,
                                                        const R* __restrict__ x, R* __restrict__ y,
                                                        int nrhs, R shift,
                                                        const int* __restrict__ active) {
  if (active && !*active) return;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= op.npts) return;
  const int i = (int)(id % op.nx);
  const int j = (int)((id / op.nx) % op.ny);
  const int k = ND == 3 ? (int)(id / ((long long)op.nx * op.ny)) : 0;
  const long long ndof = (long long)(ND + 2) * op.npts;
  const bool wall = op.bcy == 1 && (j == 0 || j == op.ny - 1);
  if (wall) {
    for (int r = 0; r < nrhs; ++r)
#pragma unroll
      for (int f = 0; f < ND + 2; ++f) y[r * ndof + (long long)f * op.npts + id] = R(0);
    return;
  }
  Axis<R> ax[3];
  ax[0] = axis_coefs<R>(6);
  ax[1] = axis_coefs<R>(wall_row_order(j, op.ny, op.bcy));
  ax[2] = axis_coefs<R>(6);
  const R ih[3] = {R(op.ihx), R(op.ihy), R(op.ihz)};

  Acc<R, ND, false> Ab{base, nullptr, op.npts, op.nx, op.ny, op.nz, op.bcy, i, j, k};
  Pt<R, ND> b;
  gather(b, Ab, ax, ih);

  for (int r = 0; r < nrhs; ++r) {
    const R* xr = x + r * ndof;
    Acc<R, ND, true> Av{base, xr, op.npts, op.nx, op.ny, op.nz, op.bcy, i, j, k};
    Pt<R, ND> v;
    gather(v, Av, ax, ih);
    R out[ND + 2];
    tangent_point<R, ND>(b, v, op, out);
#pragma unroll
    for (int f = 0; f < ND + 2; ++f) {
      const long long o = (long long)f * op.npts + id;
      y[r * ndof + o] = out[f] - shift * xr[o];
    }
  }
}

__global__ void base_derive_kernel(OpParams op, double* __restrict__ base, float* __restrict__ base32,
                                   int* __restrict__ flag) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= op.npts) return;
  const int nv = op.ndim + 2;
  const double p = base[id];
  const double s = base[(long long)(nv - 1) * op.npts + id];
  bool bad = !(p > 0.0) || !isfinite(p);
  for (int f = 0; f < nv; ++f) bad = bad || !isfinite(base[(long long)f * op.npts + id]);
  // rho = (p/p_ref)^(1/gamma) exp(-s/c_p), T = p/(rho R)
  const double rho = exp(log(p / op.p_ref) / op.gamma - s / op.cp);
  const double T = p / (rho * op.R);
  const double Tp = T / p * (1.0 - 1.0 / op.gamma);
  const double Ts = T / op.cp;
  base[(long long)nv * op.npts + id] = T;
  base[(long long)(nv + 1) * op.npts + id] = Tp;
  base[(long long)(nv + 2) * op.npts + id] = Ts;
  for (int f = 0; f < nv + 3; ++f)
    base32[(long long)f * op.npts + id] = (float)base[(long long)f * op.npts + id];
  if (bad) atomicOr(flag, 1);
}

// Exact classification of the base state (see launch_iso_classify).
struct IsoIdx {
  int q[ISO_MAXF];
};
__global__ void iso_classify_kernel(OpParams op, const double* __restrict__ base, const double* __restrict__ bdata,
                                    IsoIdx fi, int nf, int* __restrict__ flags) {
  __shared__ int sf[3];
  if (threadIdx.x < 3) sf[threadIdx.x] = 0;
  __syncthreads();
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < op.npts) {
    const int nv = op.ndim + 2;
    int nonuni = 0, nz = 0, var = 0;
    if (base[id] != base[0] || base[(long long)(nv - 1) * op.npts + id] != base[(long long)(nv - 1) * op.npts])
      nonuni = 1;
    const int j = (int)((id / op.nx) % op.ny);
    for (int q = 0; q < nf; ++q) {
      const double* f = bdata + (long long)fi.q[q] * op.npts;
      const double v = f[id];
      if (v != 0.0) nz |= 1 << q;
      if (v != f[(long long)j * op.nx]) var |= 1 << q;
    }
    if (nonuni) atomicOr(&sf[0], 1);
    if (nz) atomicOr(&sf[1], nz);
    if (var) atomicOr(&sf[2], var);
  }
  __syncthreads();
  if (threadIdx.x < 3 && sf[threadIdx.x]) atomicOr(&flags[threadIdx.x], sf[threadIdx.x]);
}

}  // namespace

hipError_t launch_iso_classify(const OpParams& p, const double* base, const double* bdata, const int* fidx, int nf,
                               int* flags, hipStream_t s) {
  if (nf > ISO_MAXF) return hipErrorInvalidValue;
  IsoIdx fi{};
  for (int q = 0; q < nf; ++q) fi.q[q] = fidx[q];
  const int threads = 256;
  const long long blocks = (p.npts + threads - 1) / threads;
  iso_classify_kernel<<<dim3((unsigned)blocks), dim3(threads), 0, s>>>(p, base, bdata, fi, nf, flags);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_jv_direct(const OpParams& p, const R* base, const R* x, R* y, int nrhs, R shift,
                            const int* active, hipStream_t s) {
  const int threads = 256;
  const long long blocks = (p.npts + threads - 1) / threads;
  if (p.ndim == 2)
    jv_direct_kernel<R, 2><<<dim3((unsigned)blocks), dim3(threads), 0, s>>>(p, base, x, y, nrhs, shift, active);
  else
    jv_direct_kernel<R, 3><<<dim3((unsigned)blocks), dim3(threads), 0, s>>>(p, base, x, y, nrhs, shift, active);
  return hipGetLastError();
}

template hipError_t launch_jv_direct<double>(const OpParams&, const double*, const double*, double*, int,
                                      double, const int*, hipStream_t);
template hipError_t launch_jv_direct<float>(const OpParams&, const float*, const float*, float*, int, float,
                                     const int*, hipStream_t);

hipError_t launch_base_derive(const OpParams& p, double* base, float* base32, int* flag,
                              hipStream_t s) {
  const int threads = 256;
  const long long blocks = (p.npts + threads - 1) / threads;
  base_derive_kernel<<<dim3((unsigned)blocks), dim3(threads), 0, s>>>(p, base, base32, flag);
  return hipGetLastError();
}

}  // namespace sa

namespace sa {

// 0: perturbation-only kernel of the precision, 1: tiled, base state
// differentiated on the fly, 2: reference, 3: tiled with precomputed base
// data, 4: prefetching perturbation-only kernel, 5: staging one
static int kernel_choice() {
  static const int k = [] {
    const char* e = std::getenv("SA_JV_KERNEL");
    if (!e) return 0;
    if (std::strcmp(e, "onthefly") == 0) return 1;
    if (std::strcmp(e, "reference") == 0) return 2;
    if (std::strcmp(e, "tiled") == 0) return 3;
    if (std::strcmp(e, "prefetch") == 0) return 4;
    if (std::strcmp(e, "stage") == 0) return 5;
    return 0;
  }();
  return k;
}

static bool pert_kernel(int k) { return k == 0 || k == 4 || k == 5; }

bool jv_kernel_forced() { return kernel_choice() != 0; }

template <typename R>
hipError_t launch_jv_pert(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                          const int* active, hipStream_t s, long long sX, long long sY, const double* shifts,
                          long long sA, int variant) {
  const int k = kernel_choice();
  if (k == 4) variant = 0;
  if (k == 5) variant = 2;
  if (variant < 0 || variant >= JV_NVARIANTS) variant = sizeof(R) == 8 ? 0 : 2;
  // kernel (0 prefetch, 1 stage) and z planes per workgroup of each variant
  // an iso variant on a base state outside that class: the default kernel
  const IsoBase<R>* ib = static_cast<const IsoBase<R>*>(p.iso[sizeof(R) == 8 ? 0 : 1]);
  if (jv_variant_is_iso(variant) && !ib) variant = sizeof(R) == 8 ? 0 : 2;
  static constexpr int kind[JV_NVARIANTS] = {0, 0, 1, 1, 0, 0, 1, 1, 2, 2, 2, 2};
  static constexpr int depth[JV_NVARIANTS] = {32, 16, 16, 32, 4, 1, 4, 1, 32, 16, 4, 1};
  const int nzc = depth[variant];
  if (kind[variant] == 2)
    return launch_jv_iso<R>(p, *ib, x, y, nrhs, shift, active, s, sX, sY, shifts, sA, nzc);
  if (kind[variant] == 0)
    return launch_jv_prefetch<R>(p, base, bdata, x, y, nrhs, shift, active, s, sX, sY, shifts, sA, nzc);
  return launch_jv_stage<R>(p, base, bdata, x, y, nrhs, shift, active, s, sX, sY, shifts, sA, nzc);
}

template <typename R>
hipError_t launch_jv(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                     const int* active, hipStream_t s, int variant) {
  const int k = kernel_choice();
  if (k == 2) return launch_jv_direct<R>(p, base, x, y, nrhs, shift, active, s);
  if (pert_kernel(k) && bdata)
    return launch_jv_pert<R>(p, base, bdata, x, y, nrhs, shift, active, s, 0, 0, nullptr, 0, variant);
  return launch_jv_tiled<R>(p, base, x, y, nrhs, shift, active, k == 1 ? nullptr : bdata, s);
}

template <typename R>
hipError_t launch_jv_batch(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nsys,
                           long long sX, long long sY, const double* shifts_host, const double* shifts_dev,
                           const int* active, long long sA, hipStream_t s, int variant) {
  if (pert_kernel(kernel_choice()) && bdata)
    return launch_jv_pert<R>(p, base, bdata, x, y, nsys, R(0), active, s, sX, sY, shifts_dev, sA, variant);
  for (int r = 0; r < nsys; ++r) {
    hipError_t e = launch_jv<R>(p, base, bdata, x + r * sX, y + r * sY, 1, R(shifts_host[r]),
                                active ? active + r * sA : nullptr, s, variant);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_jv_batch<double>(const OpParams&, const double*, const double*, const double*, double*,
                                            int, long long, long long, const double*, const double*, const int*,
                                            long long, hipStream_t, int);
template hipError_t launch_jv_batch<float>(const OpParams&, const float*, const float*, const float*, float*, int,
                                           long long, long long, const double*, const double*, const int*,
                                           long long, hipStream_t, int);

template hipError_t launch_jv<double>(const OpParams&, const double*, const double*, const double*, double*,
                                      int, double, const int*, hipStream_t, int);
template hipError_t launch_jv<float>(const OpParams&, const float*, const float*, const float*, float*, int,
                                     float, const int*, hipStream_t, int);

}  // namespace sa
