// Operator with compact first derivatives (Section "Governing equations",
// last paragraph: the paper differentiates its wave terms with the 6th-order
// compact scheme of Lele).  The discrete operator is the one of jv.hip with
// every first difference D_a replaced by the compact derivative
//   alpha f'_{i-1} + f'_i + alpha f'_{i+1}
//       = a (f_{i+1} - f_{i-1}) / (2h) + b (f_{i+2} - f_{i-2}) / (4h),
// alpha = 1/3, a = 14/9, b = 1/9 (cyclic on periodic axes); next to a wall
// the 4th-order Pade row (alpha = 1/4, a = 3/2, b = 0), at a wall the
// 3rd-order one-sided row f'_0 + 2 f'_1 = (-5/2 f_0 + 2 f_1 + 1/2 f_2)/h.
// Second derivatives stay the explicit ones.
//
// Compact derivatives couple whole grid lines, so the operator is computed
// derivative-first, per system, in a context workspace:
//   1. W = (p', u', s', T') with wall rows zero, T' = T_p p' + T_s s';
//   2. D_a W for every axis a: one thread per grid line, a Thomas sweep
//      whose right-hand side is formed on the fly from a 5-point window
//      (periodic lines: Sherman-Morrison on the cyclic system);
//   3. the mixed parts of G_i: M_x = D_y v + D_z w, M_y = D_x u + D_z w,
//      M_z = D_x u + D_y v, then D_x M_x, D_y M_y, D_z M_z;
//   4. per point: the explicit second differences of W, the base data, and
//      the pointwise tangent-linear algebra (jv_common.h).
// The base data (sa_base_set) come from the same steps on q0.
#include <cmath>
#include <vector>

#include "jv_common.h"

namespace sa {
namespace {

constexpr double C_ALPHA = 1.0 / 3.0, C_A = 14.0 / 9.0, C_B = 1.0 / 9.0;

// One axis of the grid as lines: n points, stride st between them; line L
// starts at (L % m1) s1 + (L / m1) s2; `lines` lines per field.
struct CAxis {
  int n, lines, periodic, m1;
  long long st, s1, s2;
  int tab;   // offset of the axis' tables (l, inv, c, q: n each) in the table array
  int sc;    // offset of its two scalars (1/(1 + v.q), v_{n-1})
};

CAxis axis_of(const OpParams& p, int a) {
  CAxis x{};
  const long long nx = p.nx, ny = p.ny, nz = p.nz;
  if (a == 0) {
    x.n = p.nx; x.st = 1; x.lines = (int)(ny * nz); x.m1 = 1 << 30; x.s1 = nx; x.s2 = 0; x.periodic = 1;
  } else if (a == 1) {
    x.n = p.ny; x.st = nx; x.lines = (int)(nx * nz); x.m1 = (int)nx; x.s1 = 1; x.s2 = nx * ny;
    x.periodic = p.bcy == 0;
  } else {
    x.n = p.nz; x.st = nx * ny; x.lines = (int)(nx * ny); x.m1 = 1 << 30; x.s1 = 1; x.s2 = 0; x.periodic = 1;
  }
  x.tab = a == 0 ? 0 : (a == 1 ? 4 * p.nx : 4 * (p.nx + p.ny));
  x.sc = 4 * (p.nx + p.ny + p.nz) + 2 * a;
  return x;
}

// compact derivative along one axis of nf fields: dst_f = D src_f, field f
// at src + f fs (dst + f fd); fields of one system.  rs (stretched rows,
// else null): the solution is scaled by rs[i] (the line's metric) after the
// solve, with ih = 1
template <typename R>
__global__ void __launch_bounds__(256) cd1_kernel(CAxis ax, const R* __restrict__ tab, R ih, const R* __restrict__ rs,
                                                  const R* __restrict__ src, long long fs, R* __restrict__ dst,
                                                  long long fd, int nf, const int* __restrict__ active, long long sA,
                                                  int sys) {
  if (active && !active[sys * sA]) return;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)ax.lines * nf) return;
  const int f = (int)(t / ax.lines), L = (int)(t % ax.lines);
  const long long start = (long long)(L % ax.m1) * ax.s1 + (long long)(L / ax.m1) * ax.s2;
  const R* g = src + f * fs + start;
  R* o = dst + f * fd + start;
  const int n = ax.n;
  const long long st = ax.st;
  const R* tl = tab + ax.tab;
  const R* tinv = tl + n;
  const R* tc = tinv + n;
  const R ha = R(C_A / 2.0) * ih, hb = R(C_B / 4.0) * ih;
  // forward sweep: d'_i = (r_i - l_i d'_{i-1}) inv_i, the right-hand side
  // from a window f[i-2 .. i+2] (wrapped on periodic lines, zero beyond the
  // ends of the others, where only the closure rows read near the ends)
  auto at = [&](int i) -> R {
    if (ax.periodic) return g[(long long)(i < 0 ? i + n : (i >= n ? i - n : i)) * st];
    return (i < 0 || i >= n) ? R(0) : g[(long long)i * st];
  };
  R w0 = at(-2), w1 = at(-1), w2 = at(0), w3 = at(1), w4 = at(2);
  R dp = R(0);
  for (int i = 0; i < n; ++i) {
    R r;
    if (ax.periodic || (i >= 2 && i <= n - 3)) {
      r = ha * (w3 - w1) + hb * (w4 - w0);
    } else if (i == 0) {
      r = (R(-2.5) * w2 + R(2) * w3 + R(0.5) * w4) * ih;
    } else if (i == 1 || i == n - 2) {
      r = R(0.75) * (w3 - w1) * ih;
    } else {   // i == n - 1
      r = (R(2.5) * w2 - R(2) * w1 - R(0.5) * w0) * ih;
    }
    dp = (r - tl[i] * dp) * tinv[i];
    o[(long long)i * st] = dp;
    w0 = w1;
    w1 = w2;
    w2 = w3;
    w3 = w4;
    w4 = at(i + 3);
  }
  // back substitution
  R x = o[(long long)(n - 1) * st];
  if (rs) o[(long long)(n - 1) * st] = x * rs[n - 1];
  for (int i = n - 2; i >= 0; --i) {
    x = o[(long long)i * st] - tc[i] * x;
    o[(long long)i * st] = rs ? x * rs[i] : x;
  }
  if (ax.periodic) {   // Sherman-Morrison correction of the cyclic system
    const R* tq = tc + n;
    const R fac = (o[0] + tab[ax.sc + 1] * o[(long long)(n - 1) * st]) * tab[ax.sc];
    for (int i = 0; i < n; ++i) o[(long long)i * st] -= fac * tq[i];
  }
}

// W = (p', u', s', T') of system sys with zero wall rows
template <typename R, int ND>
__global__ void __launch_bounds__(256) cstage_kernel(OpParams op, const R* __restrict__ base, const R* __restrict__ x, long long sX,
                              R* __restrict__ W, const int* __restrict__ active, long long sA, int sys) {
  if (active && !active[sys * sA]) return;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long np = op.npts;
  if (id >= np) return;
  constexpr int NV = ND + 2;
  const int j = (int)((id / op.nx) % op.ny);
  const bool wall = op.bcy == 1 && (j == 0 || j == op.ny - 1);
  const R* xs = x + sys * sX;
  R pp = R(0), sp = R(0);
#pragma unroll
  for (int f = 0; f < NV; ++f) {
    const R v = wall ? R(0) : xs[f * np + id];
    W[f * np + id] = v;
    if (f == 0) pp = v;
    if (f == NV - 1) sp = v;
  }
  W[NV * np + id] = base[(NV + 1) * np + id] * pp + base[(NV + 2) * np + id] * sp;   // T_p p' + T_s s'
}

// M_x = D_y v + D_z w, M_y = D_x u + D_z w, M_z = D_x u + D_y v (2D: D_y v, D_x u)
// from D (D[a][f] at D + (a NF + f) np, NF = ND + 3)
template <typename R, int ND>
__global__ void __launch_bounds__(256) cmix_kernel(OpParams op, const R* __restrict__ D, R* __restrict__ M, const int* __restrict__ active,
                            long long sA, int sys) {
  if (active && !active[sys * sA]) return;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long np = op.npts;
  if (id >= np) return;
  constexpr int NF = ND + 3;
  auto d = [&](int a, int f) { return D[(long long)(a * NF + f) * np + id]; };
  if (ND == 2) {
    M[id] = d(1, 2);
    M[np + id] = d(0, 1);
  } else {
    M[id] = d(1, 2) + d(2, 3);
    M[np + id] = d(0, 1) + d(2, 3);
    M[2 * np + id] = d(0, 1) + d(1, 2);
  }
}

// explicit second derivative along one axis of field f at point (i, j, k)
template <typename R>
__device__ __forceinline__ R d2_at(const OpParams& op, const R* __restrict__ F, int a, int i, int j, int k) {
  const long long nx = op.nx, ny = op.ny;
  int order = 6, n, c;
  if (a == 0) {
    n = op.nx;
    c = i;
  } else if (a == 1) {
    n = op.ny;
    c = j;
    order = wall_row_order(j, op.ny, op.bcy);
  } else {
    n = op.nz;
    c = k;
  }
  const Axis<R> A = axis_coefs<R>(order);
  const bool per = a != 1 || op.bcy == 0;
  auto at = [&](int cc) -> R {
    if (per) cc = cc < 0 ? cc + n : (cc >= n ? cc - n : cc);
    else cc = cc < 0 ? 0 : (cc >= n ? n - 1 : cc);   // only reached with zero coefficients
    const int ii = a == 0 ? cc : i, jj = a == 1 ? cc : j, kk = a == 2 ? cc : k;
    return F[((long long)kk * ny + jj) * nx + ii];
  };
  R acc = A.c0 * at(c);
#pragma unroll
  for (int m = 1; m <= 3; ++m) acc += A.c2[m - 1] * (at(c + m) + at(c - m));
  if (a == 1) return acc * ymet<R>(op)[op.ny + j];   // m2 of the row; fill_pt adds m4 D_y f
  const R ih = R(a == 0 ? op.ihx : op.ihz);
  return acc * ih * ih;
}

// the point's fields for the algebra: W values, compact D, explicit second
// differences and the compact mixed parts of G
template <typename R, int ND>
__device__ __forceinline__ void fill_pt(const OpParams& op, const R* __restrict__ W, const R* __restrict__ D,
                                        const R* __restrict__ GM, long long id, int i, int j, int k, Pt<R, ND>& P) {
  constexpr int NF = ND + 3;
  const long long np = op.npts;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    P.q[f] = W[f * np + id];
#pragma unroll
    for (int a = 0; a < ND; ++a) P.D[f][a] = D[(long long)(a * NF + f) * np + id];
  }
  const R m4 = ymet<R>(op)[2 * op.ny + j];   // -y''/y'^2 of the row (0 on uniform rows)
#pragma unroll
  for (int c = 0; c < ND; ++c) {
    const R* F = W + (long long)(1 + c) * np;
    R L = R(0), own = R(0);
#pragma unroll
    for (int a = 0; a < ND; ++a) {
      R d2 = d2_at<R>(op, F, a, i, j, k);
      if (a == 1) d2 += m4 * P.D[1 + c][1];
      L += d2;
      if (a == c) own = d2;
    }
    P.Lu[c] = L;
    P.G[c] = own + GM[(long long)c * np + id];
  }
  R LT = R(0);
#pragma unroll
  for (int a = 0; a < ND; ++a) LT += d2_at<R>(op, W + (long long)(ND + 2) * np, a, i, j, k);
  P.LT = LT + m4 * P.D[ND + 2][1];
}

// y = (J - shift I) x at every point of system sys
template <typename R, int ND>
__global__ void __launch_bounds__(256) cpoint_kernel(OpParams op, const R* __restrict__ bdata, const R* __restrict__ W,
                              const R* __restrict__ D, const R* __restrict__ GM, const R* __restrict__ x, R* __restrict__ y,
                              long long sX, long long sY, R shift, const double* __restrict__ shifts,
                              const int* __restrict__ active, long long sA, int sys) {
  if (active && !active[sys * sA]) return;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long np = op.npts;
  if (id >= np) return;
  const int i = (int)(id % op.nx), j = (int)((id / op.nx) % op.ny), k = (int)(id / ((long long)op.nx * op.ny));
  Pt<R, ND> v;
  fill_pt<R, ND>(op, W, D, GM, id, i, j, k, v);
  // base data: p0, u0_i, T0, D p0, D u0, D s0, D T0, L u0 + G0/3, L T0
  Pt<R, ND> b;
  int q = 0;
  auto get = [&]() { return bdata[(long long)(q++) * np + id]; };
  b.q[0] = get();
#pragma unroll
  for (int a = 0; a < ND; ++a) b.q[1 + a] = get();
  b.q[ND + 1] = R(0);
  b.q[ND + 2] = get();
#pragma unroll
  for (int a = 0; a < ND; ++a) b.D[0][a] = get();
#pragma unroll
  for (int c = 0; c < ND; ++c)
#pragma unroll
    for (int a = 0; a < ND; ++a) b.D[1 + c][a] = get();
#pragma unroll
  for (int a = 0; a < ND; ++a) b.D[ND + 1][a] = get();
#pragma unroll
  for (int a = 0; a < ND; ++a) b.D[ND + 2][a] = get();
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    b.Lu[a] = get();
    b.G[a] = R(0);
  }
  b.LT = get();
  R out[ND + 2];
  tangent_point<R, ND>(b, v, op, out);
  const R sh = shifts ? R(shifts[sys]) : shift;
  const bool wall = op.bcy == 1 && (j == 0 || j == op.ny - 1);
#pragma unroll
  for (int f = 0; f < ND + 2; ++f) {
    const R val = out[f] - sh * v.q[f];
    y[sys * sY + f * np + id] = wall ? R(0) : val;
  }
}

// base data of the compact operator from W = (p0, u0_i, s0, T0)
template <int ND>
__global__ void __launch_bounds__(256) cbase_kernel(OpParams op, const double* __restrict__ W, const double* __restrict__ D,
                             const double* __restrict__ GM, double* __restrict__ bdata) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long np = op.npts;
  if (id >= np) return;
  const int i = (int)(id % op.nx), j = (int)((id / op.nx) % op.ny), k = (int)(id / ((long long)op.nx * op.ny));
  Pt<double, ND> b;
  fill_pt<double, ND>(op, W, D, GM, id, i, j, k, b);
  int q = 0;
  auto put = [&](double v) { bdata[(long long)(q++) * np + id] = v; };
  put(b.q[0]);
  for (int a = 0; a < ND; ++a) put(b.q[1 + a]);
  put(b.q[ND + 2]);
  for (int a = 0; a < ND; ++a) put(b.D[0][a]);
  for (int c = 0; c < ND; ++c)
    for (int a = 0; a < ND; ++a) put(b.D[1 + c][a]);
  for (int a = 0; a < ND; ++a) put(b.D[ND + 1][a]);
  for (int a = 0; a < ND; ++a) put(b.D[ND + 2][a]);
  for (int a = 0; a < ND; ++a) put(b.Lu[a] + b.G[a] * (1.0 / 3.0));
  put(b.LT);
}

template <typename R>
const R* ymet_host(const OpParams& p) {
  if constexpr (sizeof(R) == 8) return p.ym64;
  else return p.ym32;
}

template <typename R>
const R* ctab(const OpParams& p);
template <>
const double* ctab<double>(const OpParams& p) {
  return p.ctab64;
}
template <>
const float* ctab<float>(const OpParams& p) {
  return p.ctab32;
}

inline unsigned blocks(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// steps 2-3 for one system: D of the NF fields of W along every axis, the
// mixed sums M and their derivatives GM
template <typename R, int ND>
hipError_t derivatives(const OpParams& p, const R* W, R* D, R* M, R* GM, const int* active, long long sA, int sys,
                       hipStream_t s) {
  constexpr int NF = ND + 3;
  const long long np = p.npts;
  const R* tab = ctab<R>(p);
  // stretched rows: the y solve runs with ih = 1 and scales its solution by
  // the row metric m1 (a row-dependent factor does not commute with A^-1)
  const bool st = p.stretch > 0.0;
  const R ih[3] = {R(p.ihx), st ? R(1) : R(p.ihy), R(p.ihz)};
  const R* rs[3] = {nullptr, st ? ymet_host<R>(p) : nullptr, nullptr};
  for (int a = 0; a < ND; ++a) {
    const CAxis ax = axis_of(p, a);
    cd1_kernel<R><<<blocks((long long)ax.lines * NF, 256), 256, 0, s>>>(ax, tab, ih[a], rs[a], W, np,
                                                                          D + (long long)a * NF * np, np, NF, active,
                                                                          sA, sys);
  }
  cmix_kernel<R, ND><<<blocks(np, 256), 256, 0, s>>>(p, D, M, active, sA, sys);
  for (int a = 0; a < ND; ++a) {
    const CAxis ax = axis_of(p, a);
    cd1_kernel<R><<<blocks(ax.lines, 256), 256, 0, s>>>(ax, tab, ih[a], rs[a], M + (long long)a * np, np,
                                                        GM + (long long)a * np, np, 1, active, sA, sys);
  }
  return hipGetLastError();
}

}  // namespace

size_t compact_work_elems(int ndim, long long npts) {
  const int nf = ndim + 3;
  return (size_t)(nf + ndim * nf + 2 * ndim) * (size_t)npts;
}

size_t compact_table_elems(const OpParams& p) { return (size_t)(4 * (p.nx + p.ny + p.nz) + 6); }

// Thomas tables of every axis (the cyclic ones for the Sherman-Morrison
// solve, with gamma = -1), in double and float.
void compact_tables(const OpParams& p, std::vector<double>& t64) {
  t64.assign(compact_table_elems(p), 0.0);
  for (int a = 0; a < 3; ++a) {
    const int n = a == 0 ? p.nx : (a == 1 ? p.ny : p.nz);
    if (a == 2 && p.ndim == 2) continue;
    const CAxis ax = axis_of(p, a);
    std::vector<double> lo(n, 0.0), di(n, 1.0), up(n, 0.0);
    if (ax.periodic) {
      for (int i = 0; i < n; ++i) {
        lo[i] = C_ALPHA;
        up[i] = C_ALPHA;
      }
      di[0] = 1.0 + 1.0;                    // A[0][0] - gamma
      di[n - 1] = 1.0 + C_ALPHA * C_ALPHA;  // A[n-1][n-1] - alpha * alpha / gamma
    } else {
      for (int i = 2; i <= n - 3; ++i) {
        lo[i] = C_ALPHA;
        up[i] = C_ALPHA;
      }
      lo[1] = up[1] = 0.25;
      lo[n - 2] = up[n - 2] = 0.25;
      up[0] = 2.0;
      lo[n - 1] = 2.0;
    }
    lo[0] = 0.0;
    up[n - 1] = 0.0;
    double* tl = t64.data() + ax.tab;
    double* tinv = tl + n;
    double* tc = tinv + n;
    double cprev = 0.0;
    for (int i = 0; i < n; ++i) {
      const double den = di[i] - lo[i] * cprev;
      tl[i] = lo[i];
      tinv[i] = 1.0 / den;
      tc[i] = up[i] / den;
      cprev = tc[i];
    }
    if (ax.periodic) {
      // q = A'^{-1} u, u = (gamma, 0, .., 0, alpha); v = (1, 0, .., 0, alpha/gamma)
      double* tq = tc + n;
      std::vector<double> dp(n);
      double prev = 0.0;
      for (int i = 0; i < n; ++i) {
        const double r = i == 0 ? -1.0 : (i == n - 1 ? C_ALPHA : 0.0);
        prev = (r - tl[i] * prev) * tinv[i];
        dp[i] = prev;
      }
      double xx = dp[n - 1];
      tq[n - 1] = xx;
      for (int i = n - 2; i >= 0; --i) {
        xx = dp[i] - tc[i] * xx;
        tq[i] = xx;
      }
      const double vlast = C_ALPHA / -1.0;
      t64[ax.sc] = 1.0 / (1.0 + tq[0] + vlast * tq[n - 1]);
      t64[ax.sc + 1] = vlast;
    }
  }
}

template <typename R>
hipError_t launch_jv_compact(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                             const int* active, hipStream_t s, long long sX, long long sY, const double* shifts,
                             long long sA) {
  const long long np = p.npts;
  const int nd = p.ndim;
  const int nf = nd + 3;
  R* W = static_cast<R*>(p.cwork);
  R* D = W + (long long)nf * np;
  R* M = D + (long long)nd * nf * np;
  R* GM = M + (long long)nd * np;
  if (!W || !ctab<R>(p)) return hipErrorInvalidValue;
  const long long nvn = (long long)(nd + 2) * np;
  if (sX == 0) sX = nvn;
  if (sY == 0) sY = nvn;
  for (int sys = 0; sys < nrhs; ++sys) {
    hipError_t e;
    if (nd == 2) {
      cstage_kernel<R, 2><<<blocks(np, 256), 256, 0, s>>>(p, base, x, sX, W, active, sA, sys);
      e = derivatives<R, 2>(p, W, D, M, GM, active, sA, sys, s);
      if (e == hipSuccess)
        cpoint_kernel<R, 2><<<blocks(np, 256), 256, 0, s>>>(p, bdata, W, D, GM, x, y, sX, sY, shift, shifts, active,
                                                             sA, sys);
    } else {
      cstage_kernel<R, 3><<<blocks(np, 256), 256, 0, s>>>(p, base, x, sX, W, active, sA, sys);
      e = derivatives<R, 3>(p, W, D, M, GM, active, sA, sys, s);
      if (e == hipSuccess)
        cpoint_kernel<R, 3><<<blocks(np, 256), 256, 0, s>>>(p, bdata, W, D, GM, x, y, sX, sY, shift, shifts, active,
                                                             sA, sys);
    }
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}
template hipError_t launch_jv_compact<double>(const OpParams&, const double*, const double*, const double*, double*,
                                              int, double, const int*, hipStream_t, long long, long long,
                                              const double*, long long);
template hipError_t launch_jv_compact<float>(const OpParams&, const float*, const float*, const float*, float*, int,
                                             float, const int*, hipStream_t, long long, long long, const double*,
                                             long long);

hipError_t launch_base_data_compact(const OpParams& p, const double* base, double* bdata, hipStream_t s) {
  const long long np = p.npts;
  const int nd = p.ndim;
  const int nf = nd + 3;
  double* W = static_cast<double*>(p.cwork);
  if (!W || !p.ctab64) return hipErrorInvalidValue;
  double* D = W + (long long)nf * np;
  double* M = D + (long long)nd * nf * np;
  double* GM = M + (long long)nd * np;
  // W = (p0, u0_i, s0, T0): the base array's first nv + 1 fields
  hipError_t e = hipMemcpyAsync(W, base, sizeof(double) * nf * np, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  if (nd == 2) {
    e = derivatives<double, 2>(p, W, D, M, GM, nullptr, 0, 0, s);
    if (e == hipSuccess) cbase_kernel<2><<<blocks(np, 256), 256, 0, s>>>(p, W, D, GM, bdata);
  } else {
    e = derivatives<double, 3>(p, W, D, M, GM, nullptr, 0, 0, s);
    if (e == hipSuccess) cbase_kernel<3><<<blocks(np, 256), 256, 0, s>>>(p, W, D, GM, bdata);
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace sa
