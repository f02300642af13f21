// Small dense steps of the implicitly restarted Arnoldi method (Algorithm 1)
// on one 64-lane workgroup: Ritz pairs of H_m (complex Schur form by shifted
// QR with Wilkinson shifts, eigenvectors by back substitution), ordering by
// decreasing |theta|, the Ritz-estimate test of eq. ritz_estimate, and the
// p exact-shift QR steps H <- Q^T H Q with Q accumulated (a conjugate pair of
// shifts is one real double-shift step, (H - s)(H - conj s) = QR).
#include <cfloat>

#include "arnoldi_small.h"

namespace sa {
namespace {

constexpr double EPS = 2.220446049250313e-16;   // 2^-52
constexpr int LD = MMAX;
// Largest m whose four m x m working matrices of the restart (T and Z, then
// H_m, M, HQ and Q) fit in 64 KB of LDS with leading dimension m; larger
// Arnoldi dimensions work in the state's global arrays.
constexpr int RESTART_LDS_M = 44;

__device__ __forceinline__ double cabs2(double r, double i) { return hypot(r, i); }

// complex Schur form T = Z^H H Z of the real m x m matrix in st->Hm, into
// (Tr, Ti) and (Zr, Zi), column-major with leading dimension LDT (LDS or the
// state's arrays).  All 64 lanes take part; lane 0 decides, every lane
// applies rotations to the row/column it owns.  Returns 0 on success.
template <int LDT>
__device__ int complex_schur(IState* st, int m, double* Tr, double* Ti, double* Zr, double* Zi) {
  const int lane = threadIdx.x;
  for (int j = 0; j < m; ++j) {
    if (lane < m) {
      Tr[j * LDT + lane] = st->Hm[j * MMAX + lane];
      Ti[j * LDT + lane] = 0.0;
      Zr[j * LDT + lane] = lane == j ? 1.0 : 0.0;
      Zi[j * LDT + lane] = 0.0;
    }
  }
  __shared__ int s_hi, s_l, s_stop, s_iter;
  __shared__ double s_mr, s_mi, s_c, s_sr, s_si;
  if (lane == 0) {
    s_hi = m - 1;
    s_iter = 0;
    s_stop = 0;
  }
  __syncthreads();
  int total = 0;
  while (true) {
    if (lane == 0) {
      const int hi = s_hi;
      int l = hi;
      while (l > 0) {
        const double sub = cabs2(Tr[(l - 1) * LDT + l], Ti[(l - 1) * LDT + l]);
        double d = cabs2(Tr[(l - 1) * LDT + l - 1], Ti[(l - 1) * LDT + l - 1]) +
                   cabs2(Tr[l * LDT + l], Ti[l * LDT + l]);
        if (d == 0.0) d = st->hnorm;
        if (sub <= EPS * d) {
          Tr[(l - 1) * LDT + l] = 0.0;
          Ti[(l - 1) * LDT + l] = 0.0;
          break;
        }
        --l;
      }
      s_l = l;
      if (hi <= 0) {
        s_stop = 1;
      } else if (l == hi) {
        s_hi = hi - 1;
        s_iter = 0;
        s_stop = 2;   // deflated one eigenvalue, no sweep
      } else {
        s_stop = 0;
        // Wilkinson shift from the trailing 2x2 block
        const double ar = Tr[(hi - 1) * LDT + hi - 1], ai = Ti[(hi - 1) * LDT + hi - 1];
        const double br = Tr[hi * LDT + hi - 1], bi = Ti[hi * LDT + hi - 1];
        const double cr = Tr[(hi - 1) * LDT + hi], ci = Ti[(hi - 1) * LDT + hi];
        const double dr = Tr[hi * LDT + hi], di = Ti[hi * LDT + hi];
        // eigenvalues of [[a b][c d]]: t/2 +- sqrt((a-d)^2/4 + b c)
        const double hr = 0.5 * (ar - dr), hi_ = 0.5 * (ai - di);
        const double qr = hr * hr - hi_ * hi_ + (br * cr - bi * ci);
        const double qi = 2.0 * hr * hi_ + (br * ci + bi * cr);
        // complex sqrt
        const double mod = hypot(qr, qi);
        double sr = sqrt(0.5 * (mod + qr));
        double si = sqrt(fmax(0.0, 0.5 * (mod - qr)));
        if (qi < 0) si = -si;
        const double tr = 0.5 * (ar + dr), ti = 0.5 * (ai + di);
        const double m1r = tr + sr, m1i = ti + si, m2r = tr - sr, m2i = ti - si;
        const double d1 = hypot(m1r - dr, m1i - di), d2 = hypot(m2r - dr, m2i - di);
        double mr = d1 < d2 ? m1r : m2r, mi = d1 < d2 ? m1i : m2i;
        ++s_iter;
        if (s_iter % 11 == 10) {   // exceptional shift
          const double sub = cabs2(Tr[(hi - 1) * LDT + hi], Ti[(hi - 1) * LDT + hi]);
          mr = dr + 0.75 * sub;
          mi = di;
        }
        s_mr = mr;
        s_mi = mi;
      }
    }
    __syncthreads();
    const int stop = s_stop;
    if (stop == 1) break;
    if (stop == 2) {
      __syncthreads();
      continue;
    }
    if (++total > 60 * m) return 1;
    const int l = s_l, hi = s_hi;
    for (int k = l; k < hi; ++k) {
      if (lane == 0) {
        double xr, xi, yr, yi;
        if (k == l) {
          xr = Tr[l * LDT + l] - s_mr;
          xi = Ti[l * LDT + l] - s_mi;
          yr = Tr[l * LDT + l + 1];
          yi = Ti[l * LDT + l + 1];
        } else {
          xr = Tr[(k - 1) * LDT + k];
          xi = Ti[(k - 1) * LDT + k];
          yr = Tr[(k - 1) * LDT + k + 1];
          yi = Ti[(k - 1) * LDT + k + 1];
        }
        const double ax = hypot(xr, xi), ay = hypot(yr, yi);
        const double nrm = hypot(ax, ay);
        double c, sr, si;
        if (nrm == 0.0) {
          c = 1.0; sr = 0.0; si = 0.0;
        } else if (ax == 0.0) {
          c = 0.0; sr = 1.0; si = 0.0;
        } else {
          c = ax / nrm;
          // s = (x/|x|) conj(y) / nrm
          const double ur = xr / ax, ui = xi / ax;
          sr = (ur * yr + ui * yi) / nrm;
          si = (ui * yr - ur * yi) / nrm;
        }
        s_c = c;
        s_sr = sr;
        s_si = si;
      }
      __syncthreads();
      const double c = s_c, sr = s_sr, si = s_si;
      // rows k, k+1: T <- G T, G = [[c, s], [-conj(s), c]], columns >= max(k-1, 0)
      {
        const int j = lane;
        if (j < m && j >= (k > 0 ? k - 1 : 0)) {
          const double t1r = Tr[j * LDT + k], t1i = Ti[j * LDT + k];
          const double t2r = Tr[j * LDT + k + 1], t2i = Ti[j * LDT + k + 1];
          Tr[j * LDT + k] = c * t1r + (sr * t2r - si * t2i);
          Ti[j * LDT + k] = c * t1i + (sr * t2i + si * t2r);
          // -conj(s) t1 + c t2
          Tr[j * LDT + k + 1] = -(sr * t1r + si * t1i) + c * t2r;
          Ti[j * LDT + k + 1] = -(sr * t1i - si * t1r) + c * t2i;
        }
      }
      __syncthreads();
      // columns k, k+1: T <- T G^H, rows 0..min(k+2, hi)
      {
        const int i = lane;
        const int imax = k + 2 < hi ? k + 2 : hi;
        if (i <= imax) {
          const double t1r = Tr[k * LDT + i], t1i = Ti[k * LDT + i];
          const double t2r = Tr[(k + 1) * LDT + i], t2i = Ti[(k + 1) * LDT + i];
          // t1 c + t2 conj(s) ; -t1 s + t2 c
          Tr[k * LDT + i] = t1r * c + (t2r * sr + t2i * si);
          Ti[k * LDT + i] = t1i * c + (t2i * sr - t2r * si);
          Tr[(k + 1) * LDT + i] = -(t1r * sr - t1i * si) + t2r * c;
          Ti[(k + 1) * LDT + i] = -(t1r * si + t1i * sr) + t2i * c;
        }
        if (i < m) {
          const double z1r = Zr[k * LDT + i], z1i = Zi[k * LDT + i];
          const double z2r = Zr[(k + 1) * LDT + i], z2i = Zi[(k + 1) * LDT + i];
          Zr[k * LDT + i] = z1r * c + (z2r * sr + z2i * si);
          Zi[k * LDT + i] = z1i * c + (z2i * sr - z2r * si);
          Zr[(k + 1) * LDT + i] = -(z1r * sr - z1i * si) + z2r * c;
          Zi[(k + 1) * LDT + i] = -(z1r * si + z1i * sr) + z2i * c;
        }
      }
      __syncthreads();
    }
  }
  return 0;
}

// Unit eigenvector of T for eigenvalue p (lane p), mapped by Z: stored in
// (Yr, Yi) column p (unsorted order, later permuted).
template <int LDT>
__device__ void schur_eigvec(IState* st, int m, int p, const double* Tr, const double* Ti, double* xr,
                             double* xi) {
  const double lr = Tr[p * LDT + p], li = Ti[p * LDT + p];
  const double smin = fmax(EPS * st->hnorm, DBL_MIN * 1e10);
  for (int i = 0; i < m; ++i) {
    xr[i] = 0.0;
    xi[i] = 0.0;
  }
  xr[p] = 1.0;
  for (int i = p - 1; i >= 0; --i) {
    double sr = 0.0, si = 0.0;
    for (int j = i + 1; j <= p; ++j) {
      const double ar = Tr[j * LDT + i], ai = Ti[j * LDT + i];
      sr += ar * xr[j] - ai * xi[j];
      si += ar * xi[j] + ai * xr[j];
    }
    double dr = Tr[i * LDT + i] - lr, di = Ti[i * LDT + i] - li;
    if (hypot(dr, di) < smin) {
      dr = smin;
      di = 0.0;
    }
    // x_i = -s / d
    const double den = dr * dr + di * di;
    xr[i] = -(sr * dr + si * di) / den;
    xi[i] = -(si * dr - sr * di) / den;
  }
}

// USE_LDS: the working matrices live in LDS with leading dimension
// RESTART_LDS_M (dynamic LDS of 4 RESTART_LDS_M m doubles); else in the
// state's arrays.
template <bool USE_LDS>
__global__ void restart_kernel(IState* st) {
  constexpr int L = USE_LDS ? RESTART_LDS_M : LD;
  extern __shared__ double lds[];
  const int lane = threadIdx.x;
  const int m = st->m;
  if (USE_LDS && m > RESTART_LDS_M) {   // launched for a smaller m: refuse
    if (lane == 0) {
      st->fail = 1;
      st->done = 1;
    }
    return;
  }
  const int ms = USE_LDS ? L * m : 0;   // LDS words per matrix
  double* Tr = USE_LDS ? lds : st->Tr;
  double* Ti = USE_LDS ? lds + ms : st->Ti;
  double* Zr = USE_LDS ? lds + 2 * ms : st->Zr;
  double* Zi = USE_LDS ? lds + 3 * ms : st->Zi;
  // H_m and the norms
  for (int j = 0; j < m; ++j)
    if (lane < m) st->Hm[j * LD + lane] = st->H[j * (MMAX + 1) + lane];
  __syncthreads();
  if (lane == 0) {
    double s = 0.0;
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) s += st->Hm[j * LD + i] * st->Hm[j * LD + i];
    st->hnorm = sqrt(s);
    st->fnorm = fabs(st->H[(m - 1) * (MMAX + 1) + m]);
    st->fail = 0;
  }
  __syncthreads();
  if (complex_schur<L>(st, m, Tr, Ti, Zr, Zi)) {
    if (lane == 0) {
      st->fail = 1;
      st->done = 1;
    }
    return;
  }
  __syncthreads();
  // eigenvalues and unit eigenvectors (lane p -> eigenvalue p), into M/HQ
  // as temporaries (x in M/HQ columns, y = Z x into er/ei later)
  if (lane < m) {
    st->er[lane] = Tr[lane * L + lane];
    st->ei[lane] = Ti[lane * L + lane];
    double* xr = st->M + lane * LD;
    double* xi = st->HQ + lane * LD;
    schur_eigvec<L>(st, m, lane, Tr, Ti, xr, xi);
  }
  __syncthreads();
  // y_p = Z x_p, normalised; store unsorted into Yr/Yi
  if (lane < m) {
    const int p = lane;
    const double* xr = st->M + p * LD;
    const double* xi = st->HQ + p * LD;
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) {
      double yr = 0.0, yi = 0.0;
      for (int j = 0; j <= p; ++j) {
        const double zr = Zr[j * L + i], zi = Zi[j * L + i];
        yr += zr * xr[j] - zi * xi[j];
        yi += zr * xi[j] + zi * xr[j];
      }
      st->Yr[p * LD + i] = yr;
      st->Yi[p * LD + i] = yi;
      nrm += yr * yr + yi * yi;
    }
    nrm = 1.0 / sqrt(nrm);
    for (int i = 0; i < m; ++i) {
      st->Yr[p * LD + i] *= nrm;
      st->Yi[p * LD + i] *= nrm;
    }
  }
  __syncthreads();
  // classification, pairing and ordering (lane 0)
  if (lane == 0) {
    const double imtol = 1e-12 * st->hnorm;
    for (int p = 0; p < m; ++p) st->partner[p] = -2;   // -2 unassigned, -1 real
    for (int p = 0; p < m; ++p)
      if (fabs(st->ei[p]) <= imtol) st->partner[p] = -1;
    for (int p = 0; p < m; ++p) {
      if (st->partner[p] != -2 || st->ei[p] < 0) continue;
      int best = -1;
      double bd = 0.0;
      for (int q = 0; q < m; ++q) {
        if (q == p || st->partner[q] != -2 || st->ei[q] > 0) continue;
        const double d = hypot(st->er[q] - st->er[p], st->ei[q] + st->ei[p]);
        if (best < 0 || d < bd) {
          best = q;
          bd = d;
        }
      }
      if (best >= 0) {
        st->partner[p] = best;
        st->partner[best] = p;
      } else {
        st->partner[p] = -1;
      }
    }
    for (int p = 0; p < m; ++p)
      if (st->partner[p] == -2) st->partner[p] = -1;   // unmatched: treat as real
    // groups: real eigenvalue, or (positive-imaginary member, partner)
    int gidx[MMAX];
    double gkey[MMAX];
    int ng = 0;
    for (int p = 0; p < m; ++p) {
      if (st->partner[p] >= 0 && st->ei[p] < 0) continue;
      gidx[ng] = p;
      gkey[ng] = hypot(st->er[p], st->partner[p] >= 0 ? st->ei[p] : 0.0);
      ++ng;
    }
    // stable selection sort by decreasing |theta|, ties by larger real part
    for (int a = 0; a < ng; ++a) {
      int best = a;
      for (int b = a + 1; b < ng; ++b) {
        const bool better = gkey[b] > gkey[best] ||
                            (gkey[b] == gkey[best] && st->er[gidx[b]] > st->er[gidx[best]]);
        if (better) best = b;
      }
      const int ti = gidx[a];
      gidx[a] = gidx[best];
      gidx[best] = ti;
      const double tk = gkey[a];
      gkey[a] = gkey[best];
      gkey[best] = tk;
    }
    int pos = 0;
    for (int g = 0; g < ng; ++g) {
      const int p = gidx[g];
      st->order[pos++] = p;
      if (st->partner[p] >= 0) st->order[pos++] = -1 - p;   // conjugate of p
    }
    for (int o = 0; o < m; ++o) {
      const int code = st->order[o];
      const int p = code >= 0 ? code : -1 - code;
      const bool cplx = st->partner[p] >= 0;
      st->wr[o] = st->er[p];
      st->wi[o] = cplx ? (code >= 0 ? st->ei[p] : -st->ei[p]) : 0.0;
    }
  }
  __syncthreads();
  // sorted eigenvectors into Tr/Ti (free now): column o
  if (lane < m) {
    const int o = lane;
    const int code = st->order[o];
    const int p = code >= 0 ? code : -1 - code;
    const double sgn = code >= 0 ? 1.0 : -1.0;
    for (int i = 0; i < m; ++i) {
      st->Tr[o * LD + i] = st->Yr[p * LD + i];
      st->Ti[o * LD + i] = sgn * st->Yi[p * LD + i];
    }
  }
  __syncthreads();
  for (int j = 0; j < m; ++j)
    if (lane < m) {
      st->Yr[j * LD + lane] = st->Tr[j * LD + lane];
      st->Yi[j * LD + lane] = st->Ti[j * LD + lane];
    }
  __syncthreads();
  // Ritz estimates and the convergence test (eq. ritz_estimate)
  __shared__ int s_done, s_k;
  if (lane == 0) {
    int nconv = 0;
    for (int o = 0; o < m; ++o) {
      const double e = st->fnorm * hypot(st->Yr[o * LD + m - 1], st->Yi[o * LD + m - 1]);
      st->est[o] = e;
      const double th = hypot(st->wr[o], st->wi[o]);
      if (o < st->nev && e <= fmax(EPS * st->hnorm, st->tol * th)) ++nconv;
    }
    st->nconv = nconv;
    for (int o = 0; o < st->nev; ++o) {
      // lambda = (sigma theta - mu)/(theta - 1)
      const double tr = st->wr[o], ti = st->wi[o];
      const double nr = st->sigma * tr - st->mu, ni = st->sigma * ti;
      const double dr = tr - 1.0, di = ti;
      const double den = dr * dr + di * di;
      st->lam_r[o] = (nr * dr + ni * di) / den;
      st->lam_i[o] = (ni * dr - nr * di) / den;
    }
    int done = (nconv >= st->nev || st->restarts >= st->max_restarts) ? 1 : 0;
    int k = st->nev;
    if (k < m && st->wi[k - 1] != 0.0 && st->wi[k] != 0.0 && st->wi[k - 1] > 0.0) ++k;   // keep pairs whole
    if (k >= m) done = 1;
    st->done = done;
    st->k = k;
    s_done = done;
    s_k = k;
  }
  __syncthreads();
  if (s_done) return;
  const int k = s_k;
  // the shift steps work on H_m, M, HQ and Q (in LDS: where T and Z were)
  double* Hm = USE_LDS ? lds : st->Hm;
  double* Mw = USE_LDS ? lds + ms : st->M;
  double* HQ = USE_LDS ? lds + 2 * ms : st->HQ;
  double* Q = USE_LDS ? lds + 3 * ms : st->Q;
  // Q = I
  for (int j = 0; j < m; ++j)
    if (lane < m) {
      Q[j * L + lane] = lane == j ? 1.0 : 0.0;
      if (USE_LDS) Hm[j * L + lane] = st->Hm[j * LD + lane];
    }
  __syncthreads();
  __shared__ double s_v[MMAX];
  __shared__ double s_mu[2];
  __shared__ int s_pair;
  for (int o = k; o < m;) {
    if (lane == 0) {
      s_mu[0] = st->wr[o];
      s_mu[1] = st->wi[o];
      s_pair = (st->wi[o] > 0.0 && o + 1 < m && st->wi[o + 1] < 0.0) ? 1 : 0;
    }
    __syncthreads();
    const double mr = s_mu[0], mi = s_mu[1];
    const int pair = s_pair;
    // M = H - mr I, or H^2 - 2 mr H + |mu|^2 I ; lane owns column j
    if (lane < m) {
      const int j = lane;
      for (int i = 0; i < m; ++i) {
        double v;
        if (pair) {
          double hh = 0.0;
          for (int r = 0; r < m; ++r) hh += Hm[r * L + i] * Hm[j * L + r];
          v = hh - 2.0 * mr * Hm[j * L + i] + (i == j ? mr * mr + mi * mi : 0.0);
        } else {
          v = Hm[j * L + i] - (i == j ? mr : 0.0);
        }
        Mw[j * L + i] = v;
      }
      for (int i = 0; i < m; ++i) HQ[j * L + i] = i == j ? 1.0 : 0.0;   // Qj = I
    }
    __syncthreads();
    // Householder QR of M; Qj accumulated in HQ (Qj <- Qj P)
    for (int c = 0; c < m - 1; ++c) {
      if (lane == 0) {
        double nrm = 0.0;
        for (int i = c; i < m; ++i) nrm += Mw[c * L + i] * Mw[c * L + i];
        nrm = sqrt(nrm);
        const double x0 = Mw[c * L + c];
        const double alpha = x0 >= 0 ? -nrm : nrm;
        for (int i = 0; i < m; ++i) s_v[i] = 0.0;
        if (nrm > 0.0) {
          s_v[c] = x0 - alpha;
          for (int i = c + 1; i < m; ++i) s_v[i] = Mw[c * L + i];
          double vn = 0.0;
          for (int i = c; i < m; ++i) vn += s_v[i] * s_v[i];
          vn = sqrt(vn);
          if (vn > 0.0)
            for (int i = c; i < m; ++i) s_v[i] /= vn;
          else
            for (int i = c; i < m; ++i) s_v[i] = 0.0;
        }
      }
      __syncthreads();
      if (lane < m) {
        // M <- P M on column lane (columns >= c)
        const int j = lane;
        if (j >= c) {
          double d = 0.0;
          for (int i = c; i < m; ++i) d += s_v[i] * Mw[j * L + i];
          for (int i = c; i < m; ++i) Mw[j * L + i] -= 2.0 * d * s_v[i];
        }
        // Qj <- Qj P on row lane
        const int i = lane;
        double d = 0.0;
        for (int r = c; r < m; ++r) d += HQ[r * L + i] * s_v[r];
        for (int r = c; r < m; ++r) HQ[r * L + i] -= 2.0 * d * s_v[r];
      }
      __syncthreads();
    }
    // H <- Qj^T H Qj : first M = H Qj (lane owns row i), then H = Qj^T M (lane owns column j)
    if (lane < m) {
      const int i = lane;
      for (int j = 0; j < m; ++j) {
        double s = 0.0;
        for (int r = 0; r < m; ++r) s += Hm[r * L + i] * HQ[j * L + r];
        Mw[j * L + i] = s;
      }
    }
    __syncthreads();
    if (lane < m) {
      const int j = lane;
      for (int i = 0; i < m; ++i) {
        double s = 0.0;
        for (int r = 0; r < m; ++r) s += HQ[i * L + r] * Mw[j * L + r];
        Hm[j * L + i] = (i > j + 1) ? 0.0 : s;   // Hessenberg up to rounding
      }
    }
    __syncthreads();
    // Q <- Q Qj (lane owns row i); M as temporary
    if (lane < m) {
      const int i = lane;
      for (int j = 0; j < m; ++j) {
        double s = 0.0;
        for (int r = 0; r < m; ++r) s += Q[r * L + i] * HQ[j * L + r];
        Mw[j * L + i] = s;
      }
    }
    __syncthreads();
    if (lane < m)
      for (int j = 0; j < m; ++j) Q[j * L + lane] = Mw[j * L + lane];
    __syncthreads();
    o += pair ? 2 : 1;
  }
  // k-step update data; H <- [H_k 0; 0 0]
  if (lane == 0) {
    st->coef[0] = Hm[(k - 1) * L + k];                       // beta_hat = H(k+1, k)
    st->coef[1] = Q[(k - 1) * L + m - 1] * st->H[(m - 1) * (MMAX + 1) + m];   // Q(m,k) ||f_m||
    st->restarts += 1;
  }
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    for (int i = lane; i <= m; i += blockDim.x) {
      const double v = (j < k && i < k) ? Hm[j * L + i] : 0.0;
      st->H[j * (MMAX + 1) + i] = v;
    }
    if (USE_LDS && lane < m) st->Q[j * LD + lane] = Q[j * L + lane];   // read by the k-step update
  }
}

__global__ void column_kernel(IState* st, int j) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i <= j; ++i) st->H[j * (MMAX + 1) + i] = st->d1[i] + st->d2[i];
  const double h = sqrt(st->wn2);
  st->H[j * (MMAX + 1) + j + 1] = h;
  st->inv = h > 0.0 ? 1.0 / h : 0.0;
}

__global__ void set_fk_kernel(IState* st) {
  if (threadIdx.x != 0) return;
  const int k = st->k;
  const double h = sqrt(st->wn2);
  st->H[(k - 1) * (MMAX + 1) + k] = h;
  st->inv = h > 0.0 ? 1.0 / h : 0.0;
}

__global__ void inv_norm_kernel(IState* st) {
  if (threadIdx.x != 0) return;
  const double h = sqrt(st->wn2);
  st->inv = h > 0.0 ? 1.0 / h : 0.0;
}

__global__ void init_kernel(IState* st, int m, int nev, double tol, double sigma, double mu,
                            int max_restarts) {
  const int lane = threadIdx.x;
  for (int j = 0; j < m; ++j)
    for (int i = lane; i <= m; i += blockDim.x) st->H[j * (MMAX + 1) + i] = 0.0;
  if (lane == 0) {
    st->m = m;
    st->nev = nev;
    st->tol = tol;
    st->sigma = sigma;
    st->mu = mu;
    st->max_restarts = max_restarts;
    st->restarts = 0;
    st->done = 0;
    st->fail = 0;
    st->nconv = 0;
    st->k = 0;
  }
}

// out[:, c] = sum_r V[:, r] C[r + c*ldc]
template <int MAXR>
__global__ void __launch_bounds__(256) gemm_tall_kernel(long long n, const double* __restrict__ V,
                                                        long long ldv, int nrow,
                                                        const double* __restrict__ C, int ldc, int ncol,
                                                        double* __restrict__ out, long long ldo) {
  __shared__ double sC[MMAX * MMAX];
  for (int t = threadIdx.x; t < nrow * ncol; t += blockDim.x) {
    const int r = t % nrow, c = t / nrow;
    sC[c * MMAX + r] = C[r + (long long)c * ldc];
  }
  __syncthreads();
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double v[MAXR];
#pragma unroll
    for (int r = 0; r < MAXR; ++r) v[r] = r < nrow ? V[(long long)r * ldv + i] : 0.0;
    for (int c = 0; c < ncol; ++c) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < MAXR; ++r)
        if (r < nrow) s += v[r] * sC[c * MMAX + r];
      out[(long long)c * ldo + i] = s;
    }
  }
}

__global__ void combine2_kernel(long long n, const double* __restrict__ x1, const double* __restrict__ x2,
                                const double* __restrict__ a, double* __restrict__ y) {
  const double a0 = a[0], a1 = a[1];
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    y[i] = a0 * x1[i] + a1 * x2[i];
}

__global__ void eig_resid_kernel(long long n, const double* __restrict__ Jxr, const double* __restrict__ Jxi,
                                 const double* __restrict__ xr, const double* __restrict__ xi, double lr,
                                 double li, double* __restrict__ partial) {
  __shared__ double red[2][4];
  double a = 0.0, b = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double rr = Jxr[i] - (lr * xr[i] - li * xi[i]);
    const double ri = Jxi[i] - (lr * xi[i] + li * xr[i]);
    a += rr * rr + ri * ri;
    b += xr[i] * xr[i] + xi[i] * xi[i];
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = a;
    red[1][w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int k = 0; k < (int)(blockDim.x / 64); ++k) {
      sa += red[0][k];
      sb += red[1][k];
    }
    partial[2 * blockIdx.x] = sa;
    partial[2 * blockIdx.x + 1] = sb;
  }
}

__global__ void eig_resid_reduce(const double* __restrict__ partial, int nb, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < nb; ++k) {
    a += partial[2 * k];
    b += partial[2 * k + 1];
  }
  out[0] = a;
  out[1] = b;
}

inline unsigned grid_for(long long n) {
  long long b = (n + 255) / 256;
  if (b > RED_BLOCKS) b = RED_BLOCKS;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

void iram_column(IState* st, int j, hipStream_t s) { column_kernel<<<1, 64, 0, s>>>(st, j); }
void iram_restart(IState* st, int m, hipStream_t s) {
  if (m <= RESTART_LDS_M)
    restart_kernel<true><<<1, 64, sizeof(double) * 4 * RESTART_LDS_M * m, s>>>(st);
  else
    restart_kernel<false><<<1, 64, 0, s>>>(st);
}
void iram_set_fk(IState* st, hipStream_t s) { set_fk_kernel<<<1, 64, 0, s>>>(st); }
void iram_inv_norm(IState* st, hipStream_t s) { inv_norm_kernel<<<1, 64, 0, s>>>(st); }
void iram_init(IState* st, int m, int nev, double tol, double sigma, double mu, int max_restarts,
               hipStream_t s) {
  init_kernel<<<1, 64, 0, s>>>(st, m, nev, tol, sigma, mu, max_restarts);
}

void gemm_tall(long long n, const double* V, long long ldv, int nrow, const double* C, int ldc, int ncol,
               double* out, long long ldo, hipStream_t s) {
  if (nrow <= 16)
    gemm_tall_kernel<16><<<grid_for(n), 256, 0, s>>>(n, V, ldv, nrow, C, ldc, ncol, out, ldo);
  else if (nrow <= 32)
    gemm_tall_kernel<32><<<grid_for(n), 256, 0, s>>>(n, V, ldv, nrow, C, ldc, ncol, out, ldo);
  else
    gemm_tall_kernel<64><<<grid_for(n), 256, 0, s>>>(n, V, ldv, nrow, C, ldc, ncol, out, ldo);
}

void combine2(long long n, const double* x1, const double* x2, const double* a, double* y, hipStream_t s) {
  combine2_kernel<<<grid_for(n), 256, 0, s>>>(n, x1, x2, a, y);
}

void eig_residual(long long n, const double* Jxr, const double* Jxi, const double* xr, const double* xi,
                  double lr, double li, double* partial, double* out, hipStream_t s) {
  const unsigned nb = grid_for(n);
  eig_resid_kernel<<<nb, 256, 0, s>>>(n, Jxr, Jxi, xr, xi, lr, li, partial);
  eig_resid_reduce<<<1, 64, 0, s>>>(partial, (int)nb, out);
}

}  // namespace sa
