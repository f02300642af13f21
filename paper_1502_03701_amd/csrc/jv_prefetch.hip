// Perturbation-only operator kernel y = (J(q0) - shift I) x (prefetching
// variant, the FP64 default), used once the base state's derivative data exist (sa_base_set computes them
// with the tiled kernel of jv_tiled.hip).  Same discrete operator and the
// same pointwise algebra (jv_common.h); organised for throughput on CDNA:
//   * a workgroup owns a TX x TY column tile and marches over NZC planes;
//   * each thread keeps its own column's perturbation values of planes
//     k-3 .. k+2 in a register queue and loads plane k+3, so every plane is
//     read once per tile for the z-derivatives;
//   * the centre plane with a 3-point xy halo is staged in LDS: the interior
//     comes from the queue, only the halo positions are loaded;
//   * mixed derivatives are first differences of staged first derivatives
//     (G_x = D2_x u + D_x(D_y v + D_z w), G_y = D2_y v + D_y(D_x u + D_z w),
//     G_z = D2_z w + D_x(D_z u) + D_y(D_z v)); the z-derivatives on the halo
//     strips come from direct loads, one halo position per thread;
//   * the global loads of plane k+1 (halo, halo z-taps, plane k+4) are
//     issued before the pointwise algebra of plane k, unconditionally and
//     with no arithmetic on them (T' and the wall rows are formed when plane
//     k+1 is staged), so the wave does not wait for them before the algebra;
//     the base data of a point are loaded before the plane's first barrier;
//     in FP64 the kernel runs at one wave per SIMD and this memory-level
//     parallelism is what keeps HBM busy;
//   * workgroups are numbered so that tiles adjacent in x run on the same
//     XCD (and share its L2), which serves the halo re-reads from cache;
//   * loads are branch-free (wall rows are clamped and masked), indices are
//     32-bit within a field.
#include "jv_common.h"

namespace sa {
namespace {

constexpr int TX = 16;
constexpr int TY = 16;
constexpr int PW = TX + 6;
constexpr int PH = TY + 6;
constexpr int NT = TX * TY;
constexpr int NHALO = PW * PH - NT;   // staged halo positions of a plane
constexpr int NXH = 6 * TY;           // x-strip positions needing D_z
constexpr int NYH = 6 * TX;           // y-strip positions needing D_z
static_assert(NHALO <= NT && NXH + NYH <= NT, "one halo position per thread");
constexpr int NXCD = 8;

// Periodic index of a in [-n, 2n).  Indices beyond n + 3 only feed points
// outside the grid (tiles are padded), so they are clamped into range.
__device__ __forceinline__ int wrapc(int a, int n) { return a < 0 ? a + n : (a >= n ? min(a - n, n - 1) : a); }

template <int ND>
constexpr int nbdata() { return 1 + ND + 1 + ND + ND * ND + ND + ND + ND + 1; }

// A batch of systems shares one launch: system sys (from the logical z block
// index sys * zchunks + chunk) reads x + sys*strideX, writes y + sys*strideY,
// uses shifts[sys] (or the scalar shift) and the flag active[sys*sA].
// FULL: the tiles cover the grid exactly (nx, ny multiples of 16): every
// thread owns a grid point and no branch surrounds the algebra and stores.
template <typename R, int ND, int NZC, bool FULL>
__global__ void __launch_bounds__(NT) jv_prefetch_kernel(OpParams op, const R* __restrict__ base,
                                                     const R* __restrict__ bdata, const R* __restrict__ x,
                                                     R* __restrict__ y, R shift, const int* __restrict__ active,
                                                     long long strideX, long long strideY,
                                                     const double* __restrict__ shifts, long long sA, int zchunks,
                                                     int gx, int gy, int ntot) {
  // XCD-aware numbering: hardware block L runs on XCD L % 8; each XCD gets a
  // contiguous range of logical tiles (x fastest).
  int lb;
  {
    const int L = blockIdx.x;
    const int per = ntot / NXCD, rem = ntot % NXCD;
    const int xcd = L % NXCD, idx = L / NXCD;
    lb = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  }
  const int bx = lb % gx;
  const int by = (lb / gx) % gy;
  const int bz = lb / (gx * gy);
  const int sys = bz / zchunks;
  const int zc = bz % zchunks;
  if (active && !active[sys * sA]) return;
  x += sys * strideX;
  y += sys * strideY;
  if (shifts) shift = R(shifts[sys]);
  constexpr int NF = ND + 3;   // p, u_i, s, T'
  constexpr int NB = nbdata<ND>();
  __shared__ R sP[NF][PH][PW];
  __shared__ R sX[2][TY][PW];  // D_y v + D_z w, D_z u  (x halo)
  __shared__ R sY[2][PH][TX];  // D_x u + D_z w, D_z v  (y halo)

  const int tid = threadIdx.x;
  const int ti = tid % TX, tj = tid / TX;
  const int nx = op.nx, ny = op.ny, nz = op.nz;
  const int i0 = bx * TX, j0 = by * TY;
  const int i = i0 + ti, j = j0 + tj;
  const int plane = nx * ny;
  const int npts = (int)op.npts;
  const bool inside = FULL || (i < nx && j < ny);
  const bool wallbc = op.bcy == 1;
  const R ihx = R(op.ihx), ihz = R(op.ihz);
  // y metric of the own row (uniform or stretched rows)
  const R* ymt = ymet<R>(op);
  const int jm = j < ny ? j : ny - 1;
  const R my1 = ymt[jm], my2 = ymt[ny + jm], my4 = ymt[2 * ny + jm];
  const Axis<R> ax = axis_coefs<R>(6);
  const Axis<R> ayc = axis_coefs<R>(wall_row_order(j < ny ? j : ny - 1, ny, op.bcy));
  const Axis<R> az = axis_coefs<R>(6);
  const R* Tp = base + (long long)(ND + 3) * npts;
  const R* Ts = base + (long long)(ND + 4) * npts;

  auto grow = [&](int jj) -> int {   // global row of a staged row
    const int g = j0 - 3 + jj;
    if (!wallbc) return wrapc(g, ny);
    return g < 0 ? 0 : (g > ny - 1 ? ny - 1 : g);
  };
  auto is_wall = [&](int g) -> bool { return wallbc && (g == 0 || g == ny - 1); };
  // the NF staged fields at flat index p (T' = T_p p' + T_s s'), zero on walls
  auto load_point = [&](int p, bool wall, R v[NF]) {
#pragma unroll
    for (int f = 0; f < ND + 2; ++f) v[f] = x[f * npts + p];
    const R tp = Tp[p], ts = Ts[p];
    v[ND + 2] = tp * v[0] + ts * v[ND + 1];
    if (wall) {
#pragma unroll
      for (int f = 0; f < NF; ++f) v[f] = R(0);
    }
  };
  // The same in two halves for the loads of the next plane: the raw values
  // (x fields, then T_p, T_s) are loaded before the algebra of this plane
  // and combined only when the next plane is staged, so that no arithmetic
  // on them (which would make the wave wait for them) precedes the algebra.
  auto load_raw = [&](int p, R v[NF + 1]) {
#pragma unroll
    for (int f = 0; f < ND + 2; ++f) v[f] = x[f * npts + p];
    v[ND + 2] = Tp[p];
    v[ND + 3] = Ts[p];
  };
  auto finish_raw = [&](bool wall, R v[NF + 1]) {
    v[ND + 2] = v[ND + 2] * v[0] + v[ND + 3] * v[ND + 1];
    if (wall) {
#pragma unroll
      for (int f = 0; f < NF; ++f) v[f] = R(0);
    }
  };

  // own column
  const int col_own = grow(tj + 3) * nx + wrapc(i, nx);
  const bool wall_own = is_wall(grow(tj + 3));
  // staged halo position of this thread: rows 0-2 and PH-3..PH-1 in full,
  // then columns 0-2 and PW-3..PW-1 of the rows in between
  const bool has_h = tid < NHALO;
  int hii = 0, hjj = 0;
  if (tid < 6 * PW) {
    const int r = tid / PW;
    hii = tid % PW;
    hjj = r < 3 ? r : PH - 6 + r;
  } else if (has_h) {
    const int t2 = tid - 6 * PW;
    const int c = t2 % 6;
    hjj = 3 + t2 / 6;
    hii = c < 3 ? c : TX + c;
  }
  const int col_h = grow(hjj) * nx + wrapc(i0 - 3 + hii, nx);
  const bool wall_h = is_wall(grow(hjj));
  // halo position of this thread for the z-derivatives of the mixed terms:
  // x strips (D_z w, D_z u) for tid < NXH, y strips (D_z w, D_z v) after
  const bool has_d = tid < NXH + NYH;
  const bool dxs = tid < NXH;
  int dr, dc;   // x strip: row dr of sX, column dc; y strip: row dr of sY, column dc
  if (dxs) {
    const int c = tid % 6;
    dr = tid / 6;
    dc = c < 3 ? c : TX + c;
  } else {
    const int t2 = has_d ? tid - NXH : 0;
    const int r = t2 / TX;
    dc = t2 % TX;
    dr = r < 3 ? r : TY + r;
  }
  const int gj_d = dxs ? grow(dr + 3) : grow(dr);
  const int col_d = gj_d * nx + wrapc(dxs ? i0 - 3 + dc : i0 + dc, nx);
  const bool wall_d = is_wall(gj_d);
  const int fb = dxs ? 1 : 2;   // u on x strips, v on y strips (w on both)
  const Axis<R> ayd = axis_coefs<R>(wall_row_order(gj_d, ny, op.bcy));

  const int kbeg = ND == 3 ? zc * NZC : 0;
  const int kend = ND == 3 ? min(nz, kbeg + NZC) : 1;

  // register queue: zq[f][m] = field f at plane k - 3 + m, m = 0..5
  R zq[NF][6];
  if (ND == 3) {
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      R v[NF];
      load_point(wrapc(kbeg - 3 + m, nz) * plane + col_own, wall_own, v);
#pragma unroll
      for (int f = 0; f < NF; ++f) zq[f][m] = v[f];
    }
  }

  // global loads of one plane: halo, halo z-taps, plane k+3 at the own column
  R hv[NF + 1], dzw[6], dzb[6], qn[NF + 1], bq[NB];   // hv, qn: raw until finish_raw
  auto load_plane = [&](int k) {
    // unconditional: threads without a halo position load a valid one and
    // drop it (a load under a divergent branch is merged by a register copy,
    // which waits for it)
    load_raw(k * plane + col_h, hv);
    if (ND == 3) {
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        const int p = wrapc(k - 3 + m + (m >= 3 ? 1 : 0), nz) * plane + col_d;
        dzw[m] = x[3 * npts + p];
        dzb[m] = x[fb * npts + p];
      }
    }
    load_raw((ND == 3 ? wrapc(k + 3, nz) * plane : 0) + col_own, qn);
  };
  auto load_bdata = [&](int k) {
#pragma unroll
    // streamed once: nontemporal, so they do not push the reused x halos out of L2
    for (int q = 0; q < NB; ++q) bq[q] = __builtin_nontemporal_load(bdata + (q * npts + k * plane + col_own));
  };
  load_plane(kbeg);

  for (int k = kbeg; k < kend; ++k) {
    const int pown = k * plane + col_own;   // the output index for inside points
    load_bdata(k);
    finish_raw(wall_h, hv);
    finish_raw(wall_own, qn);
    __syncthreads();
    // ---- stage plane k: interior from the queue, halo from the loads ----
#pragma unroll
    for (int f = 0; f < NF; ++f) sP[f][tj + 3][ti + 3] = ND == 3 ? zq[f][3] : qn[f];
    if (has_h) {
#pragma unroll
      for (int f = 0; f < NF; ++f) sP[f][hjj][hii] = hv[f];
    }
    __syncthreads();
    // ---- staged first-derivative fields on the halo strips ----
    if (has_d) {
      R dzwv = R(0), dzbv = R(0);
      if (ND == 3 && !wall_d) {
#pragma unroll
        for (int m = 1; m <= 3; ++m) {
          dzwv += az.c1[m - 1] * (dzw[2 + m] - dzw[3 - m]);
          dzbv += az.c1[m - 1] * (dzb[2 + m] - dzb[3 - m]);
        }
        dzwv *= ihz;
        dzbv *= ihz;
      }
      if (dxs) {
        R dyv = R(0);
#pragma unroll
        for (int m = 1; m <= 3; ++m) dyv += ayd.c1[m - 1] * (sP[2][dr + 3 + m][dc] - sP[2][dr + 3 - m][dc]);
        sX[0][dr][dc] = dyv * ymt[gj_d] + dzwv;
        sX[1][dr][dc] = dzbv;
      } else {
        R dxu = R(0);
#pragma unroll
        for (int m = 1; m <= 3; ++m) dxu += ax.c1[m - 1] * (sP[1][dr][dc + 3 + m] - sP[1][dr][dc + 3 - m]);
        sY[0][dr][dc] = dxu * ihx + dzwv;
        sY[1][dr][dc] = dzbv;
      }
    }
    // ---- own point: derivatives from LDS (x, y) and from the queue (z) ----
    Pt<R, ND> P;
    const int cx = ti + 3, cy = tj + 3;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const R c0 = sP[f][cy][cx];
      R a1x = R(0), a2x = R(0), a1y = R(0), a2y = R(0), a1z = R(0), a2z = R(0);
#pragma unroll
      for (int m = 1; m <= 3; ++m) {
        const R xp = sP[f][cy][cx + m], xm = sP[f][cy][cx - m];
        const R yp = sP[f][cy + m][cx], ym = sP[f][cy - m][cx];
        a1x += ax.c1[m - 1] * (xp - xm);
        a2x += ax.c2[m - 1] * (xp + xm);
        a1y += ayc.c1[m - 1] * (yp - ym);
        a2y += ayc.c2[m - 1] * (yp + ym);
        if (ND == 3) {
          const R zp = m == 3 ? qn[f] : zq[f][3 + m], zm = zq[f][3 - m];
          a1z += az.c1[m - 1] * (zp - zm);
          a2z += az.c2[m - 1] * (zp + zm);
        }
      }
      P.q[f] = c0;
      P.D[f][0] = a1x * ihx;
      P.D[f][1] = a1y * my1;
      if (ND == 3) P.D[f][2] = a1z * ihz;
      if ((f >= 1 && f <= ND) || f == ND + 2) {
        const R d2x = (ax.c0 * c0 + a2x) * (ihx * ihx);
        const R d2y = (ayc.c0 * c0 + a2y) * my2 + P.D[f][1] * my4;
        const R d2z = ND == 3 ? (az.c0 * c0 + a2z) * (ihz * ihz) : R(0);
        const R L = d2x + d2y + d2z;
        if (f == ND + 2) {
          P.LT = L;
        } else {
          P.Lu[f - 1] = L;
          P.G[f - 1] = f == 1 ? d2x : (f == 2 ? d2y : d2z);
        }
      }
    }
    sX[0][tj][cx] = P.D[2][1] + (ND == 3 ? P.D[3][ND - 1] : R(0));
    sY[0][cy][ti] = P.D[1][0] + (ND == 3 ? P.D[3][ND - 1] : R(0));
    if (ND == 3) {
      sX[1][tj][cx] = P.D[1][ND - 1];
      sY[1][cy][ti] = P.D[2][ND - 1];
    }
    __syncthreads();
    {
      R gxs = R(0), gys = R(0), gz1 = R(0), gz2 = R(0);
#pragma unroll
      for (int m = 1; m <= 3; ++m) {
        gxs += ax.c1[m - 1] * (sX[0][tj][cx + m] - sX[0][tj][cx - m]);
        gys += ayc.c1[m - 1] * (sY[0][cy + m][ti] - sY[0][cy - m][ti]);
        if (ND == 3) {
          gz1 += ax.c1[m - 1] * (sX[1][tj][cx + m] - sX[1][tj][cx - m]);
          gz2 += ayc.c1[m - 1] * (sY[1][cy + m][ti] - sY[1][cy - m][ti]);
        }
      }
      P.G[0] += gxs * ihx;
      P.G[1] += gys * my1;
      if (ND == 3) P.G[2] += gz1 * ihx + gz2 * my1;
    }
    // the queue takes plane k+3; then the next plane's loads fly during the algebra
    if (ND == 3) {
#pragma unroll
      for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int m = 0; m < 5; ++m) zq[f][m] = zq[f][m + 1];
        zq[f][5] = qn[f];
      }
    }
    const int knext = min(k + 1, kend - 1);
    load_plane(knext);
    R* bk = bq;
    if (inside) {
      const bool wallrow = wallbc && (j == 0 || j == ny - 1);
      R out[ND + 2];
      {
        Pt<R, ND> b;
        int q = 0;
        b.q[0] = bk[q++];
#pragma unroll
        for (int a = 0; a < ND; ++a) b.q[1 + a] = bk[q++];
        b.q[ND + 2] = bk[q++];
        b.q[ND + 1] = R(0);
#pragma unroll
        for (int a = 0; a < ND; ++a) b.D[0][a] = bk[q++];
#pragma unroll
        for (int c2 = 0; c2 < ND; ++c2)
#pragma unroll
          for (int a = 0; a < ND; ++a) b.D[1 + c2][a] = bk[q++];
#pragma unroll
        for (int a = 0; a < ND; ++a) b.D[ND + 1][a] = bk[q++];
#pragma unroll
        for (int a = 0; a < ND; ++a) b.D[ND + 2][a] = bk[q++];
#pragma unroll
        for (int a = 0; a < ND; ++a) {
          b.Lu[a] = bk[q++];
          b.G[a] = R(0);
        }
        b.LT = bk[q++];
        tangent_point<R, ND>(b, P, op, out);
      }
#pragma unroll
      for (int f = 0; f < ND + 2; ++f)   // written once, read by another kernel: nontemporal
        __builtin_nontemporal_store(zero_on(wallrow, out[f] - shift * P.q[f]), y + (f * npts + pown));
    }
  }
}

}  // namespace

template <typename R>
hipError_t launch_jv_prefetch(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                          const int* active, hipStream_t s, long long sX, long long sY, const double* shifts,
                          long long sA, int nzc) {
  const long long ndof = (long long)(p.ndim + 2) * p.npts;
  // 32-bit indices within the base data (the widest per-point array)
  if ((long long)base_data_fields(p.ndim) * p.npts >= (1LL << 31)) return hipErrorInvalidValue;
  if (nzc != 1 && nzc != 4 && nzc != 16 && nzc != 32) return hipErrorInvalidValue;
  const int zchunks = p.ndim == 3 ? (p.nz + nzc - 1) / nzc : 1;
  if (sX == 0) sX = ndof;   // right-hand sides one after another
  if (sY == 0) sY = ndof;
  const int gx = (p.nx + TX - 1) / TX, gy = (p.ny + TY - 1) / TY;
  const long long ntot = (long long)gx * gy * zchunks * nrhs;
  if (ntot >= (1LL << 31)) return hipErrorInvalidValue;
  dim3 grid((unsigned)ntot);
#define SA_LAUNCH(ND_, NZ_, F_)                                                                                   \
  jv_prefetch_kernel<R, ND_, NZ_, F_><<<grid, NT, 0, s>>>(p, base, bdata, x, y, shift, active, sX, sY, shifts, sA, \
                                                        zchunks, gx, gy, (int)ntot)
  const bool full = p.nx % TX == 0 && p.ny % TY == 0;
  if (p.ndim == 2) {
    SA_LAUNCH(2, 16, false);   // one plane: the chunk depth is irrelevant
  } else if (nzc == 1) {
    if (full) SA_LAUNCH(3, 1, true); else SA_LAUNCH(3, 1, false);
  } else if (nzc == 4) {
    if (full) SA_LAUNCH(3, 4, true); else SA_LAUNCH(3, 4, false);
  } else if (nzc == 16) {
    if (full) SA_LAUNCH(3, 16, true); else SA_LAUNCH(3, 16, false);
  } else {
    if (full) SA_LAUNCH(3, 32, true); else SA_LAUNCH(3, 32, false);
  }
#undef SA_LAUNCH
  return hipGetLastError();
}

template hipError_t launch_jv_prefetch<double>(const OpParams&, const double*, const double*, const double*, double*,
                                           int, double, const int*, hipStream_t, long long, long long,
                                           const double*, long long, int);
template hipError_t launch_jv_prefetch<float>(const OpParams&, const float*, const float*, const float*, float*, int,
                                          float, const int*, hipStream_t, long long, long long, const double*,
                                          long long, int);

}  // namespace sa
