// Mean-flow preconditioner (Section "Preconditioning"; the Conclusions'
// direction of a cheaper approximate operator): M(s) = P (J(q_bar) - s I) P,
// the operator of the base state averaged over the periodic axes,
// q_bar(y) = mean over x (and z) of q0, solved exactly.
//
// For q_bar the discrete operator commutes with shifts along x and z, so it
// is block diagonal in their Fourier modes; each mode's block couples y rows
// only within the stencil reach (3), i.e. it is banded with kl = ku =
// 4 nv - 1 in the unknown order u = (j-1) nv + v (interior rows j = 1 ..
// ny-2).  Setup:
//   * q_bar and its base-derivative data (the same kernels as sa_base_set);
//   * the operator's columns by probing: 7 y-colours x nv variables, each
//     probe a unit at (x = 0, z = 0) on every interior row of its colour
//     (rows 7 apart, beyond the reach), nv probes per operator launch; the
//     responses at x, z offsets -3..3 give every band entry's stencil
//     coefficients S[u][b][dz][dx];
//   * per (mode, shift) one wavefront builds the mode's rows on the fly,
//     A_k[u][u'] = sum_{dx,dz} S[u][b][dz][dx] e^{-i(kx dx 2pi/nx + kz dz 2pi/nz)}
//     - s delta, and factors them by banded LU with partial pivoting in a
//     sliding (kl+1) x (kl+ku+1) window in LDS: U rows (kl+ku+1 entries),
//     L multipliers (kl) and pivot offsets are written per step.
// Apply z = M(s)^{-1} r: real-to-complex FFT along x (two real lines packed
// into one complex transform) and a complex FFT along z, one wavefront per
// (mode, system) for the banded forward and back substitutions, the inverse
// transforms, and zero wall rows.  The FFTs are self-sorting mixed-radix
// (Stockham) transforms in LDS for any length: radix 4, then 2, then the odd
// prime factors, each stage a direct sum over its radix.
#include <cmath>
#include <vector>

#include "sa_runtime.h"

namespace sa {
namespace {

template <typename T>
struct cx {
  T re, im;
};

constexpr int REACH = 3;
constexpr int NOFF = 2 * REACH + 1;   // offsets -3 .. 3
constexpr int NCOL = 7;               // y colours of the probes (> 2 REACH)
constexpr size_t LDS_CAP = 65536;     // dynamic LDS a launch of this file may take
constexpr int BS_GROUP = 16;          // forward steps per prefetch group of the banded solve
constexpr int BS_GROUP_BACK = 8;      // back-substitution steps per group (KU + 16 <= 64)
constexpr int BS_GROUP_BACK_WIDE = 16;   // the same when the packed U leaves room: KU + 32 <= 64
constexpr int FFT_THREADS = 512;      // threads per FFT workgroup (8 waves: LDS-bound occupancy)
// LDS a workgroup of the x and z FFTs batches its lines in. The x lines are
// contiguous in memory, so a 32 KB batch (four workgroups per CU to hide LDS
// latency) still reads whole rows; a z workgroup gathers its ub lines as runs
// of ub consecutive complex values per plane, and in FP64 the longer runs of
// a 64 KB batch pay more than the extra occupancy.
template <typename R> constexpr size_t fft_x_lds() { return 32768; }
template <typename R> constexpr size_t fft_z_lds() { return sizeof(R) == 8 ? 65536 : 32768; }

struct FGeom {
  int nd, nv, nx, ny, nz;
  int mx, mz, nmodes;   // modes: kx = 0 .. mx-1 (real DFT), kz = 0 .. mz-1
  int N, kl, ku, KW;    // unknowns per mode, bandwidths, window width
  int KU;               // column length of the packed U (set up: <= KW)
  long long npts, n;
};

FGeom geom_of(const Ctx* c) {
  FGeom g{};
  g.nd = c->op.ndim;
  g.nv = c->nv;
  g.nx = c->op.nx;
  g.ny = c->op.ny;
  g.nz = c->op.nz;
  g.mx = g.nx / 2 + 1;
  g.mz = g.nd == 3 ? g.nz : 1;
  g.nmodes = g.mx * g.mz;
  g.N = (g.ny - 2) * g.nv;
  g.kl = g.ku = REACH * g.nv + g.nv - 1;
  g.KW = g.kl + g.ku + 1;
  g.KU = c->fp_ku > 0 ? c->fp_ku : g.KW;
  g.npts = c->op.npts;
  g.n = c->n;
  return g;
}

// ---------------------------------------------------------------- setup ----

// q_bar: one workgroup per (variable, row) sums q0 over x and z in a fixed
// order and writes the mean to every point of that (variable, row)
__global__ void __launch_bounds__(256) mean_base_kernel(FGeom g, const double* __restrict__ q0,
                                                        double* __restrict__ qbar) {
  const int v = blockIdx.x / g.ny, j = blockIdx.x % g.ny;
  const int nxz = g.nx * g.nz;
  __shared__ double red[256];
  double acc = 0.0;
  for (int t = threadIdx.x; t < nxz; t += 256) {
    const int k = t / g.nx, i = t % g.nx;
    acc += q0[(((long long)v * g.nz + k) * g.ny + j) * g.nx + i];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double mean = red[0] / (double)nxz;
  for (int t = threadIdx.x; t < nxz; t += 256) {
    const int k = t / g.nx, i = t % g.nx;
    qbar[(((long long)v * g.nz + k) * g.ny + j) * g.nx + i] = mean;
  }
}

// probes of colour c: vector v' has 1 at (x = 0, z = 0, row j, variable v')
// for every interior row j = c (mod 7)
__global__ void probe_kernel(FGeom g, int c, double* __restrict__ P) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nrow = g.ny - 2;
  if (t >= g.nv * nrow) return;
  const int vp = t / nrow, j = 1 + t % nrow;
  if (j % NCOL != c) return;
  P[(long long)vp * g.n + (((long long)vp * g.nz + 0) * g.ny + j) * g.nx + 0] = 1.0;
}

// stencil coefficients S[u][b][dz][dx] of the band entries whose column row
// j' has colour c, from the responses Y[v'] of that colour's probes
__global__ void gather_kernel(FGeom g, int c, const double* __restrict__ Y, double* __restrict__ S) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)g.N * g.KW * NOFF * NOFF;
  if (t >= tot) return;
  const int dx = (int)(t % NOFF) - REACH;
  const int dz = (int)((t / NOFF) % NOFF) - REACH;
  const int b = (int)((t / (NOFF * NOFF)) % g.KW);
  const int u = (int)(t / ((long long)NOFF * NOFF * g.KW));
  const int up = u - g.kl + b;
  if (up < 0 || up >= g.N) {
    if (c == 0) S[t] = 0.0;   // outside the matrix: written once
    return;
  }
  const int j = 1 + u / g.nv, v = u % g.nv;
  const int jp = 1 + up / g.nv, vp = up % g.nv;
  if (jp % NCOL != c) return;
  double val = 0.0;
  const bool zok = g.nd == 3 || dz == 0;
  if (zok && abs(j - jp) <= REACH) {
    const int ii = (dx + g.nx) % g.nx, kk = g.nd == 3 ? (dz + g.nz) % g.nz : 0;
    val = Y[(long long)vp * g.n + (((long long)v * g.nz + kk) * g.ny + j) * g.nx + ii];
  }
  S[t] = val;
}

// Band LU with partial pivoting of A_k - s I for one (mode, shift) per
// wavefront.  Window W: logical row i (matrix row col + i) at physical row
// (r0 + i) % KH, logical column jj (matrix column col + jj) at physical
// column (c0 + jj) % KW.  Factor layout per (shift, mode), each row of it
// what one substitution step reads: Ut[c][0] = 1 / U(c, c) and Ut[c][d] =
// U(c - d, c) for d = 1 .. KW-1 (column c of U upwards from the diagonal;
// u_pack_kernel turns it into the layout the back substitution reads);
// L[u][0 .. kl), the multiplier of row u + 1 + d at step u; piv[u] in
// [0, kl], row u exchanged with row u + piv[u].
template <typename F>
__global__ void __launch_bounds__(64) band_lu_kernel(FGeom g, const double* __restrict__ S,
                                                     const double* __restrict__ shifts, cx<F>* __restrict__ Uo,
                                                     cx<F>* __restrict__ Lo, int* __restrict__ pivo,
                                                     int* __restrict__ singular) {
  constexpr int MAXKH = 4 * 5;        // kl + 1 <= 4 nv <= 20
  constexpr int MAXKW = 2 * 4 * 5 - 1;   // kl + ku + 1 <= 39
  __shared__ cx<F> W[MAXKH][MAXKW];
  __shared__ cx<F> lw[MAXKH];
  const int lane = threadIdx.x;
  const int m = blockIdx.x % g.nmodes, s = blockIdx.x / g.nmodes;
  const int kx = m % g.mx, kz = m / g.mx;
  const double sig = shifts[s];
  const int kl = g.kl, KW = g.KW, KH = g.kl + 1, N = g.N;
  // twiddles e^{-i theta d}, d = -3 .. 3
  double exr[NOFF], exi[NOFF], ezr[NOFF], ezi[NOFF];
#pragma unroll
  for (int d = 0; d < NOFF; ++d) {
    const double ax = -2.0 * M_PI * (double)kx * (double)(d - REACH) / (double)g.nx;
    exr[d] = cos(ax);
    exi[d] = sin(ax);
    const double az = g.nd == 3 ? -2.0 * M_PI * (double)kz * (double)(d - REACH) / (double)g.nz : 0.0;
    ezr[d] = cos(az);
    ezi[d] = sin(az);
  }
  const long long fo = (long long)s * g.nmodes + m;
  cx<F>* U = Uo + fo * ((long long)N * KW + 1);
  cx<F>* L = Lo + fo * ((long long)N * kl + 1);
  int* piv = pivo + fo * (long long)N;
  // entry (u, col + jj) of A_k - s I into physical W[pr][(c0 + jj) % KW], one column per lane
  auto gen_row = [&](int u, int col, int pr, int c0) {
    for (int jj = lane; jj < KW; jj += 64) {
      const int b = col + jj - u + kl;
      const int up = col + jj;
      double vr = 0.0, vi = 0.0;
      if (u < N && up < N && b >= 0 && b < KW) {
        const double* Sb = S + ((long long)u * KW + b) * NOFF * NOFF;
        const int z0 = g.nd == 3 ? 0 : REACH, z1 = g.nd == 3 ? NOFF : REACH + 1;
        for (int dz = z0; dz < z1; ++dz) {
          double sr = 0.0, si = 0.0;
#pragma unroll
          for (int dx = 0; dx < NOFF; ++dx) {
            const double c = Sb[dz * NOFF + dx];
            sr += c * exr[dx];
            si += c * exi[dx];
          }
          vr += sr * ezr[dz] - si * ezi[dz];
          vi += sr * ezi[dz] + si * ezr[dz];
        }
        if (b == kl) vr -= sig;
      }
      W[pr][(c0 + jj) % KW] = cx<F>{(F)vr, (F)vi};
    }
  };
  // entries Ut[c][d] with d > c (above row 0) are no matrix entries: zero;
  // so are the slots after each factor, which the solve's idle lanes read
  if (lane == 0) {
    U[(long long)N * KW] = cx<F>{F(0), F(0)};
    L[(long long)N * kl] = cx<F>{F(0), F(0)};
  }
  for (int e = lane; e < KW * KW; e += 64) {
    const int c = e / KW, d = e - c * KW;
    if (c < N && d > c) U[(long long)c * KW + d] = cx<F>{F(0), F(0)};
  }
  int r0 = 0, c0 = 0;
  for (int i = 0; i < KH; ++i) gen_row(i, 0, i, 0);
  __syncthreads();
  bool sing = false;
  for (int col = 0; col < N; ++col) {
    const int imax = min(kl, N - 1 - col);
    // pivot: first largest |re| + |im| among the window's first column
    F best = F(-1);
    int bi = 0;
    if (lane <= imax) {
      const cx<F> a = W[(r0 + lane) % KH][c0];
      best = fabs(a.re) + fabs(a.im);
      bi = lane;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const F ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    const int p = bi;
    if (!(best > F(0))) sing = true;
    // exchange logical rows 0 and p
    if (p != 0) {
      for (int jj = lane; jj < KW; jj += 64) {
        const int pc = (c0 + jj) % KW;
        const cx<F> t0 = W[r0 % KH][pc];
        W[r0 % KH][pc] = W[(r0 + p) % KH][pc];
        W[(r0 + p) % KH][pc] = t0;
      }
    }
    __syncthreads();
    const cx<F> pv = W[r0 % KH][c0];
    const F den = pv.re * pv.re + pv.im * pv.im;
    // multipliers l_i = a_i0 / pivot, and the U row
    if (lane >= 1 && lane <= kl) {
      cx<F> l{F(0), F(0)};
      if (lane <= imax && den > F(0)) {
        const cx<F> a = W[(r0 + lane) % KH][c0];
        l.re = (a.re * pv.re + a.im * pv.im) / den;
        l.im = (a.im * pv.re - a.re * pv.im) / den;
      }
      lw[lane] = l;
      L[(long long)col * kl + lane - 1] = l;
    }
    for (int jj = lane; jj < KW; jj += 64) {
      cx<F> val = W[r0 % KH][(c0 + jj) % KW];
      if (jj == 0) val = den > F(0) ? cx<F>{pv.re / den, -pv.im / den} : cx<F>{F(0), F(0)};
      if (col + jj < N) U[(long long)(col + jj) * KW + jj] = val;
    }
    if (lane == 0) piv[col] = p;
    __syncthreads();
    // trailing update of the window: W[i][jj] -= l_i W[0][jj]
    const int nupd = kl * (KW - 1);
    for (int e = lane; e < nupd; e += 64) {
      const int i = 1 + e / (KW - 1), jj = 1 + e % (KW - 1);
      const int pc = (c0 + jj) % KW;
      const cx<F> u0 = W[r0 % KH][pc];
      const cx<F> l = lw[i];
      cx<F>& w = W[(r0 + i) % KH][pc];
      w.re -= l.re * u0.re - l.im * u0.im;
      w.im -= l.re * u0.im + l.im * u0.re;
    }
    __syncthreads();
    // slide: the consumed column becomes the last one (zero for the rows
    // already in the window) and the pivot row's slot takes row col+kl+1
    const int oldc = c0, oldr = r0 % KH;
    c0 = (c0 + 1) % KW;
    r0 = r0 + 1;
    if (lane < kl) W[(r0 + lane) % KH][oldc] = cx<F>{F(0), F(0)};
    gen_row(col + 1 + kl, col + 1, oldr, c0);
    __syncthreads();
  }
  if (sing && lane == 0) atomicOr(singular, 1);
}

// Row exchanges reach only a few rows, so U's columns stay far inside the
// kl + ku band the factorisation allows (at C2 about 22 of 39 entries): the
// back substitution reads columns of the exact common length KU.
// ext = max over every (shift, mode) block and column of the largest d with
// U(c - d, c) != 0.  Grid: x over a block's N KW entries, y strides blocks
// (a few y rows: one atomic per wavefront, not per entry).
template <typename F>
__global__ void __launch_bounds__(256) u_extent_kernel(FGeom g, long long nblk, const cx<F>* __restrict__ U,
                                                       int* __restrict__ ext) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int nU = g.N * g.KW;
  int e = 0;
  if (r < nU) {
    const int d = r % g.KW;
    for (long long b = blockIdx.y; b < nblk; b += gridDim.y) {
      const cx<F> u = U[b * ((long long)nU + 1) + r];
      if (d > e && (u.re != F(0) || u.im != F(0))) e = d;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e = max(e, __shfl_xor(e, off, 64));
  if ((threadIdx.x & 63) == 0 && e > 0) atomicMax(ext, e);
}

// The layout the back substitution reads, KU entries per column: Uc[c][d] =
// U(c - d, c) / U(c, c) for d = 1 .. KU-1 and Uc[c][0] = 1 - 1 / U(c, c), so
// one multiply-add form serves every lane of a step (lane 0 turns r_0 into
// r_0 / U(c, c)); a zero slot after each block.
template <typename F>
__global__ void __launch_bounds__(256) u_pack_kernel(FGeom g, long long nblk, int KU, const cx<F>* __restrict__ U,
                                                     cx<F>* __restrict__ Uc) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int nc = g.N * KU;
  if (r > nc) return;
  const int c = r / KU, d = r - c * KU;
  for (long long b = blockIdx.y; b < nblk; b += gridDim.y) {
    cx<F> out{F(0), F(0)};
    if (r < nc) {
      const cx<F>* col = U + b * ((long long)g.N * g.KW + 1) + (long long)c * g.KW;
      const cx<F> iv = col[0];
      if (d == 0) {
        out = cx<F>{F(1) - iv.re, -iv.im};
      } else {
        const cx<F> u = col[d];
        out = cx<F>{u.re * iv.re - u.im * iv.im, u.re * iv.im + u.im * iv.re};
      }
    }
    Uc[b * ((long long)nc + 1) + r] = out;
  }
}

// FP32 factors in step pairs: the rows a sweep uses at two consecutive steps
// side by side (16 bytes a lane, one load serves two steps): Out[q][w] =
// (In[a][w], In[b][w]) with rows (a, b) = (2q, 2q + 1) for the forward sweep,
// (N-1-2q, N-2-2q) for the back substitution (rev), zero where a row is
// outside 0 .. N-1; a zero pair after each block.  In: rows of width W with
// a zero slot after each block of N rows.
__global__ void __launch_bounds__(256) pair_rows_kernel(int N, int W, int rev, long long nblk,
                                                        const cx<float>* __restrict__ In, cx<float>* __restrict__ Out) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int NP = (N + 1) / 2, np = NP * W;
  if (r > np) return;
  const int q = r / W, w = r - q * W;
  const int ra = rev ? N - 1 - 2 * q : 2 * q, rb = rev ? N - 2 - 2 * q : 2 * q + 1;
  for (long long b = blockIdx.y; b < nblk; b += gridDim.y) {
    cx<float> o0{0.0f, 0.0f}, o1{0.0f, 0.0f};
    if (r < np) {
      const cx<float>* in = In + b * ((long long)N * W + 1);
      if (ra >= 0 && ra < N) o0 = in[(long long)ra * W + w];
      if (rb >= 0 && rb < N) o1 = in[(long long)rb * W + w];
    }
    cx<float>* out = Out + 2 * (b * ((long long)np + 1) + r);
    out[0] = o0;
    out[1] = o1;
  }
}

// ---------------------------------------------------------------- apply ----

// Division by a small runtime divisor d with a multiply-high: for a d < 2^32,
// floor(a / d) = umulhi(a, floor(2^32 / d) + 1).  Magic 0 stands for d = 1.
unsigned magic_of(int d) { return d <= 1 ? 0u : (unsigned)((1ull << 32) / (unsigned)d + 1ull); }
__device__ __forceinline__ int fdiv(int a, unsigned m) { return m ? (int)__umulhi((unsigned)a, m) : a; }

// Radices of a length-n transform, in the order they are applied, with each
// stage's m' = n / (L p) and L (the product of the earlier radices) and
// their division magics.
constexpr int FMAX_STAGES = 24;
struct FPlan {
  int n, ns;
  unsigned nm;
  int rad[FMAX_STAGES], mp[FMAX_STAGES], L[FMAX_STAGES];
  unsigned mpm[FMAX_STAGES], Lm[FMAX_STAGES], bm[FMAX_STAGES];   // bm: magic of n / p
};

FPlan plan_of(int n) {
  FPlan p{};
  p.n = n;
  p.nm = magic_of(n);
  int m = n;
  while (m % 4 == 0) { p.rad[p.ns++] = 4; m /= 4; }
  while (m % 2 == 0) { p.rad[p.ns++] = 2; m /= 2; }
  for (int f = 3; f * f <= m; f += 2)
    while (m % f == 0) { p.rad[p.ns++] = f; m /= f; }
  if (m > 1) p.rad[p.ns++] = m;
  int L = 1;
  for (int t = 0; t < p.ns; ++t) {
    p.L[t] = L;
    p.Lm[t] = magic_of(L);
    p.mp[t] = n / (L * p.rad[t]);
    p.mpm[t] = magic_of(p.mp[t]);
    p.bm[t] = magic_of(n / p.rad[t]);
    L *= p.rad[t];
  }
  return p;
}

// one output of a stage of radix P_ (0: the runtime radix p)
template <typename R, int P_>
__device__ __forceinline__ cx<R> stage_out(const cx<R>* src, int mp, int p, int step, int n, const cx<R>* tw,
                                           bool inverse) {
  const int pr = P_ ? P_ : p;
  R ar = R(0), ai = R(0);
  int q = 0;
#pragma unroll
  for (int r = 0; r < (P_ ? P_ : 64); ++r) {
    if (!P_ && r >= pr) break;
    const cx<R> x = src[mp * r];
    const cx<R> w = tw[q];
    const R wi = inverse ? -w.im : w.im;
    ar += x.re * w.re - x.im * wi;
    ai += x.re * wi + x.im * w.re;
    q += step;
    if (q >= n) q -= n;
  }
  return cx<R>{ar, ai};
}

// Self-sorting FFT of P sequences of length n held one after another in a
// (LDS), with b as the second buffer; returns the buffer with the result.
// After the stages of radices p_0 .. p_{t-1} (product L), entry j + (n/L) k
// of a holds the length-L DFT, at frequency k, of the subsequence that
// starts at j with stride n/L; a stage of radix p combines p of them:
//   A'[j', k'] = sum_r e^{-2 pi i r k' / (L p)} A[j' + m' r, k' mod L],  m' = n/(L p).
// inverse: conjugate twiddles (unscaled).  Every thread of the block calls it.
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> x, cx<R> w, bool conj) {
  const R wi = conj ? -w.im : w.im;
  return cx<R>{x.re * w.re - x.im * wi, x.re * wi + x.im * w.re};
}

// Radix-4 and radix-2 stages as butterflies: the p outputs A'[j', kk + L q]
// (q = 0 .. p-1) share the inputs A[j' + m' r, kk]; each input is twiddled
// by e^{-2 pi i r kk / (L p)} and a p-point DFT gives the outputs.
template <typename R, int RP>
__device__ __forceinline__ void butterflies(const FPlan& pl, int t, const cx<R>* a, cx<R>* b, int P,
                                            const cx<R>* __restrict__ tw, bool inverse) {
  const int n = pl.n, mp = pl.mp[t], L = pl.L[t];
  const int nbf = n / RP;
  const int m = mp * RP;
  for (int o = threadIdx.x; o < P * nbf; o += blockDim.x) {
    const int sq = fdiv(o, pl.bm[t]), bi = o - sq * nbf;
    const int kk = fdiv(bi, pl.mpm[t]), jp = bi - kk * mp;
    const cx<R>* src = a + sq * n + jp + m * kk;
    cx<R> x[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      x[r] = src[mp * r];
      if (r > 0) x[r] = cmul(x[r], tw[r * kk * mp], inverse);   // r kk m' < n
    }
    cx<R>* dst = b + sq * n + jp + mp * kk;
    const long long sL = (long long)mp * L;   // output stride of q
    if (RP == 2) {
      dst[0] = cx<R>{x[0].re + x[1].re, x[0].im + x[1].im};
      dst[sL] = cx<R>{x[0].re - x[1].re, x[0].im - x[1].im};
    } else {
      // forward W_4 = -i, inverse +i: x1 * (-+i) = (+- x1.im, -+ x1.re)
      const cx<R> s02{x[0].re + x[2].re, x[0].im + x[2].im}, d02{x[0].re - x[2].re, x[0].im - x[2].im};
      const cx<R> s13{x[1].re + x[3].re, x[1].im + x[3].im}, d13{x[1].re - x[3].re, x[1].im - x[3].im};
      const cx<R> jd13 = inverse ? cx<R>{-d13.im, d13.re} : cx<R>{d13.im, -d13.re};   // W_4 (x1 - x3)
      dst[0] = cx<R>{s02.re + s13.re, s02.im + s13.im};
      dst[sL] = cx<R>{d02.re + jd13.re, d02.im + jd13.im};
      dst[2 * sL] = cx<R>{s02.re - s13.re, s02.im - s13.im};
      dst[3 * sL] = cx<R>{d02.re - jd13.re, d02.im - jd13.im};
    }
  }
}

template <typename R>
__device__ cx<R>* stockham(const FPlan& pl, cx<R>* a, cx<R>* b, int P, const cx<R>* __restrict__ tw, bool inverse) {
  const int n = pl.n;
  for (int t = 0; t < pl.ns; ++t) {
    const int p = pl.rad[t], mp = pl.mp[t], L = pl.L[t];
    const unsigned mpm = pl.mpm[t], Lm = pl.Lm[t];
    const int m = mp * p;
    if (p == 4 || p == 2) {
      if (p == 4) butterflies<R, 4>(pl, t, a, b, P, tw, inverse);
      else butterflies<R, 2>(pl, t, a, b, P, tw, inverse);
      __syncthreads();
      cx<R>* t2 = a;
      a = b;
      b = t2;
      continue;
    }
    for (int o = threadIdx.x; o < P * n; o += blockDim.x) {
      const int sq = fdiv(o, pl.nm), idx = o - sq * n;
      const int kp = fdiv(idx, mpm), jp = idx - kp * mp;
      const int kk = kp - fdiv(kp, Lm) * L;
      const cx<R>* src = a + sq * n + jp + m * kk;
      const int step = kp * mp;   // < n
      b[o] = p == 4   ? stage_out<R, 4>(src, mp, p, step, n, tw, inverse)
             : p == 2 ? stage_out<R, 2>(src, mp, p, step, n, tw, inverse)
                      : stage_out<R, 0>(src, mp, p, step, n, tw, inverse);
    }
    __syncthreads();
    cx<R>* t2 = a;
    a = b;
    b = t2;
  }
  return a;
}

// address of interior line lid = k N + u (u = (j-1) nv + v) within a system,
// and the offset of its spectrum in [k][kx][u] (add kx N)
__device__ __forceinline__ long long line_off(const FGeom& g, int lid) {
  const int k = lid / g.N, u = lid - k * g.N;
  const int jr = u / g.nv, v = u - jr * g.nv;
  return (((long long)v * g.nz + k) * g.ny + jr + 1) * g.nx;
}
__device__ __forceinline__ long long spec_off(const FGeom& g, int lid) {
  const int k = lid / g.N, u = lid - k * g.N;
  return (long long)k * g.mx * g.N + u;
}

constexpr int XMAX_PAIRS = 16;   // line pairs per workgroup of the x transforms

// the workgroup's lines 2 pair0 .. 2 pair0 + 2P - 1: vector and spectrum
// offsets (-1 past the last line), computed once into LDS
__device__ __forceinline__ void line_table(const FGeom& g, int pair0, int P, long long* s_in, long long* s_sp) {
  const int nl = g.nz * g.N;
  if (threadIdx.x < 2 * P) {
    const int lid = 2 * pair0 + threadIdx.x;
    s_in[threadIdx.x] = lid < nl ? line_off(g, lid) : -1;
    s_sp[threadIdx.x] = lid < nl ? spec_off(g, lid) : -1;
  }
}

// Forward real FFT along x of the interior lines, two lines (a, b) per
// complex transform z = a + i b: A_k = (Z_k + conj Z_{n-k}) / 2,
// B_k = -i (Z_k - conj Z_{n-k}) / 2.  P line pairs per workgroup;
// out[sys][k][kx][u] for kx = 0 .. nx/2.
template <typename R>
__global__ void __launch_bounds__(FFT_THREADS) fft_x_fwd(FGeom g, FPlan pl, int P, unsigned Pm, const R* __restrict__ r,
                                                         long long sV, const cx<R>* __restrict__ tw,
                                                         cx<R>* __restrict__ out, const int* __restrict__ active,
                                                         long long sA) {
  extern __shared__ unsigned char smem[];
  __shared__ long long s_in[2 * XMAX_PAIRS], s_sp[2 * XMAX_PAIRS];
  const int n = g.nx;
  cx<R>* stw = reinterpret_cast<cx<R>*>(smem);
  cx<R>* b0 = stw + n;
  cx<R>* b1 = b0 + P * n;
  const int sys = blockIdx.y;
  if (active && !active[sys * sA]) return;
  const int pair0 = blockIdx.x * P;
  const R* src = r + (long long)sys * sV;
  line_table(g, pair0, P, s_in, s_sp);
  for (int t = threadIdx.x; t < n; t += FFT_THREADS) stw[t] = tw[t];
  __syncthreads();
  for (int t = threadIdx.x; t < P * n; t += FFT_THREADS) {
    const int sq = fdiv(t, pl.nm), i = t - sq * n;
    const long long oa = s_in[2 * sq], ob = s_in[2 * sq + 1];
    const R a = oa >= 0 ? src[oa + i] : R(0);
    const R b = ob >= 0 ? src[ob + i] : R(0);
    b0[t] = cx<R>{a, b};
  }
  __syncthreads();
  const cx<R>* Z = stockham<R>(pl, b0, b1, P, stw, false);
  cx<R>* dst = out + (long long)sys * g.nz * g.mx * g.N;
  const long long kxs = g.N;
  for (int t = threadIdx.x; t < P * g.mx; t += FFT_THREADS) {
    const int kx = fdiv(t, Pm), sq = t - kx * P;   // consecutive threads: consecutive lines
    const long long sa = s_sp[2 * sq], sb = s_sp[2 * sq + 1];
    if (sa < 0) continue;
    const cx<R> zk = Z[sq * n + kx], zn = Z[sq * n + (kx == 0 ? 0 : n - kx)];
    const R h = R(0.5);
    dst[sa + kx * kxs] = cx<R>{h * (zk.re + zn.re), h * (zk.im - zn.im)};
    if (sb >= 0) dst[sb + kx * kxs] = cx<R>{h * (zk.im + zn.im), -h * (zk.re - zn.re)};
  }
}

// Complex FFT along z between in[sys][k][kx][u] and out[sys][kz][kx][u],
// a workgroup per (kx, ub consecutive u): the ub sequences in LDS.
template <typename R>
__global__ void __launch_bounds__(FFT_THREADS) fft_z(FGeom g, FPlan pl, int ub, unsigned ubm,
                                                     const cx<R>* __restrict__ in, const cx<R>* __restrict__ tw,
                                                     int inverse, cx<R>* __restrict__ out,
                                                     const int* __restrict__ active, long long sA) {
  extern __shared__ unsigned char smem[];
  const int n = g.nz;
  cx<R>* stw = reinterpret_cast<cx<R>*>(smem);
  cx<R>* b0 = stw + n;
  cx<R>* b1 = b0 + ub * n;
  const int sys = blockIdx.y;
  if (active && !active[sys * sA]) return;
  const int nub = (g.N + ub - 1) / ub;
  const int kx = blockIdx.x / nub;
  const int u0 = (blockIdx.x - kx * nub) * ub;
  const long long plane = (long long)g.mx * g.N;
  const cx<R>* src = in + (long long)sys * n * plane + (long long)kx * g.N + u0;
  cx<R>* dst = out + (long long)sys * n * plane + (long long)kx * g.N + u0;
  for (int t = threadIdx.x; t < n; t += FFT_THREADS) stw[t] = tw[t];
  for (int t = threadIdx.x; t < ub * n; t += FFT_THREADS) {
    const int k = fdiv(t, ubm), uu = t - k * ub;
    b0[uu * n + k] = u0 + uu < g.N ? src[(long long)k * plane + uu] : cx<R>{R(0), R(0)};
  }
  __syncthreads();
  const cx<R>* Z = stockham<R>(pl, b0, b1, ub, stw, inverse != 0);
  for (int t = threadIdx.x; t < ub * n; t += FFT_THREADS) {
    const int k = fdiv(t, ubm), uu = t - k * ub;
    if (u0 + uu < g.N) dst[(long long)k * plane + uu] = Z[uu * n + k];
  }
}

// Inverse real FFT along x (two lines per complex transform: Z = A + i B
// over the full circle from the Hermitian halves, imaginary parts of the
// k = 0 and Nyquist terms dropped) into the SoA vector, scaled by
// 1/(nx nz).  Wall rows of z are written 0 by zero_walls.
template <typename R>
__global__ void __launch_bounds__(FFT_THREADS) fft_x_inv(FGeom g, FPlan pl, int P, unsigned Pm,
                                                         const cx<R>* __restrict__ in, const cx<R>* __restrict__ tw,
                                                         R* __restrict__ z, long long sV,
                                                         const int* __restrict__ active, long long sA) {
  extern __shared__ unsigned char smem[];
  __shared__ long long s_in[2 * XMAX_PAIRS], s_sp[2 * XMAX_PAIRS];
  const int n = g.nx;
  cx<R>* stw = reinterpret_cast<cx<R>*>(smem);
  cx<R>* b0 = stw + n;
  cx<R>* b1 = b0 + P * n;
  const int sys = blockIdx.y;
  if (active && !active[sys * sA]) return;
  const int pair0 = blockIdx.x * P;
  const cx<R>* src = in + (long long)sys * g.nz * g.mx * g.N;
  line_table(g, pair0, P, s_in, s_sp);
  for (int t = threadIdx.x; t < n; t += FFT_THREADS) stw[t] = tw[t];
  __syncthreads();
  const bool even = n % 2 == 0;
  const long long kxs = g.N;
  for (int t = threadIdx.x; t < P * g.mx; t += FFT_THREADS) {
    const int kx = fdiv(t, Pm), sq = t - kx * P;
    const long long sa = s_sp[2 * sq], sb = s_sp[2 * sq + 1];
    cx<R> A = sa >= 0 ? src[sa + kx * kxs] : cx<R>{R(0), R(0)};
    cx<R> B = sb >= 0 ? src[sb + kx * kxs] : cx<R>{R(0), R(0)};
    if (kx == 0 || (even && kx == n / 2)) {
      A.im = R(0);
      B.im = R(0);
    }
    b0[sq * n + kx] = cx<R>{A.re - B.im, A.im + B.re};                 // A_k + i B_k
    if (kx != 0 && !(even && kx == n / 2))
      b0[sq * n + n - kx] = cx<R>{A.re + B.im, B.re - A.im};           // conj A_k + i conj B_k
  }
  __syncthreads();
  const cx<R>* Z = stockham<R>(pl, b0, b1, P, stw, true);
  const R scale = R(1) / (R(g.nx) * R(g.nz));
  R* dst = z + (long long)sys * sV;
  for (int t = threadIdx.x; t < P * n; t += FFT_THREADS) {
    const int sq = fdiv(t, pl.nm), i = t - sq * n;
    const long long oa = s_in[2 * sq], ob = s_in[2 * sq + 1];
    const cx<R> v = Z[t];
    if (oa >= 0) dst[oa + i] = v.re * scale;
    if (ob >= 0) dst[ob + i] = v.im * scale;
  }
}

template <typename R>
__global__ void zero_walls(FGeom g, R* __restrict__ z, long long sV, const int* __restrict__ active, long long sA) {
  const int sys = blockIdx.y;
  if (active && !active[sys * sA]) return;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)g.nv * g.nz * 2 * g.nx;
  if (t >= per) return;
  const int i = (int)(t % g.nx);
  const int w = (int)((t / g.nx) % 2);
  const long long vk = t / (2LL * g.nx);   // v * nz + k
  const int j = w ? g.ny - 1 : 0;
  z[(long long)sys * sV + (vk * g.ny + j) * g.nx + i] = R(0);
}

__device__ __forceinline__ float rdlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double rdlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename R>
__device__ __forceinline__ cx<R> rdlane(cx<R> v, int l) {
  return cx<R>{rdlane(v.re, l), rdlane(v.im, l)};
}

// whole-wavefront rotation: lane i receives lane (i + 1) mod 64 (DPP
// wave_rol:1; every lane has a source, so no old value is needed)
__device__ __forceinline__ float rol1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x134, 0xf, 0xf, false));
}
__device__ __forceinline__ double rol1(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0x134, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x134, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename R>
__device__ __forceinline__ cx<R> rol1(cx<R> v) {
  return cx<R>{rol1(v.re), rol1(v.im)};
}
// z - l b in four fused multiply-adds (b wave-uniform)
template <typename R>
__device__ __forceinline__ cx<R> cfms(cx<R> z, R lr, R li, cx<R> b) {
  R re = fma(-lr, b.re, z.re);
  re = fma(li, b.im, re);
  R im = fma(-lr, b.im, z.im);
  im = fma(-li, b.re, im);
  return cx<R>{re, im};
}

// Banded forward and back substitution of one (mode, system) per wavefront,
// in place on the mode's vector.  The moving window sits in registers with
// lane k holding row col + k (forward) or col - k (back), so a step's factor
// row is lane-aligned (one load at a uniform address), the finished row is
// read from lane 0 with readlane, every window lane updates its own row with
// four fused multiply-adds (in the back substitution lane 0 too: the packed
// U makes its update the division by the pivot), and
// the wavefront then rotates by one lane: the next rows move down and the
// finished row moves to lane 63, where the rows a group finishes collect
// for one store at the group's end.  The G rows a group brings into the
// window are loaded, with its factor rows and pivots, while the previous
// group runs (two register sets used in turn) and placed above the window
// at the group's start (window + entering + finished rows fit in 64 lanes).
// System sys uses the factors of shift shift0 + sys * shift_step.
// PAIR (FP32 factors): L and U in the step-pair layout of pair_rows_kernel.
template <typename F, typename R, int GB, bool PAIR>
__global__ void __launch_bounds__(64) band_solve_kernel(FGeom g, const cx<F>* __restrict__ Lo,
                                                        const cx<F>* __restrict__ Uo, const int* __restrict__ pivo,
                                                        int shift0, int shift_step, cx<R>* __restrict__ spec,
                                                        const int* __restrict__ active, long long sA) {
  constexpr int GF = BS_GROUP;
  const int m = blockIdx.x, sys = blockIdx.y;
  if (active && !active[sys * sA]) return;
  const int lane = threadIdx.x;
  const int N = g.N, kl = g.kl;
  const long long fo = (long long)(shift0 + sys * shift_step) * g.nmodes + m;
  const int KU = g.KU;
  const int NP = (N + 1) / 2;   // step pairs (PAIR)
  const cx<F>* L = Lo + (PAIR ? 2 * fo * ((long long)NP * kl + 1) : fo * ((long long)N * kl + 1));
  const cx<F>* Ut = Uo + (PAIR ? 2 * fo * ((long long)NP * KU + 1) : fo * ((long long)N * KU + 1));
  const int* piv = pivo + fo * (long long)N;
  cx<R>* vec = spec + ((long long)sys * g.nmodes + m) * N;   // mode m = kz mx + kx
  // loads are unconditional and need no select after them (idle lanes read
  // the zero slot after the factor; rows past the matrix read a clamped row,
  // which only rows past the matrix use), so the next group's stay in flight
  auto ldv = [&](bool ok, long long i) {
    const cx<R> v = vec[ok ? i : 0];
    return cx<R>{ok ? v.re : R(0), ok ? v.im : R(0)};
  };
  // ---- forward: P, then L; lanes 0 .. kl hold rows col .. col + kl
  const bool lmul = lane >= 1 && lane <= kl;         // lanes with a multiplier
  const bool fent = lane > kl && lane <= kl + GF;    // lanes of a group's entering rows
  const long long lzero = (long long)N * kl;         // the zero slot
  cx<R> z = ldv(lane <= kl && lane < N, lane);
  struct FwdSet {
    cx<F> l[GF];
    cx<R> ent;
    int pv[GF];   // pivot offsets of columns c0 .. c0 + GF - 1 (uniform: scalar loads)
  };
  // a factor row at a uniform base address plus a per-lane 32-bit byte
  // offset (one select per load): lane - 1 for the multiplier lanes, the
  // zero slot for the others
  const unsigned lmoff = (unsigned)(lane - 1) * (unsigned)sizeof(cx<F>);
  auto load_fwd = [&](int c0, FwdSet& f) {
    if constexpr (PAIR) {
      // c0 is even: steps c0 + s and c0 + s + 1 are pair (c0 + s) / 2
      const long long pzero = (long long)NP * kl;
#pragma unroll
      for (int s = 0; s < GF; s += 2) {
        const int q = min((c0 + s) >> 1, NP - 1);   // pairs past the end: the last pair
        const long long rb = (long long)q * kl;
        const unsigned off = lmul ? (unsigned)(lane - 1) * 16u : (unsigned)((pzero - rb) * 16);
        const float4 v = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(L) + rb * 16 + off);
        f.l[s] = cx<F>{v.x, v.y};
        f.l[s + 1] = cx<F>{v.z, v.w};
      }
    } else {
#pragma unroll
      for (int s = 0; s < GF; ++s) {
        const int col = min(c0 + s, N - 1);   // steps past the end run on row N-1's multipliers
        const long long rb = (long long)col * kl;
        const unsigned off = lmul ? lmoff : (unsigned)((lzero - rb) * (long long)sizeof(cx<F>));
        f.l[s] = *reinterpret_cast<const cx<F>*>(reinterpret_cast<const char*>(L + rb) + off);
      }
    }
    f.ent = vec[min(c0 + lane, N - 1)];
#pragma unroll
    for (int s = 0; s < GF; ++s) f.pv[s] = piv[min(c0 + s, N - 1)];
  };
  auto fwd_group = [&](int c0, const FwdSet& f) {
    if (fent) z = f.ent;
#pragma unroll
    for (int s = 0; s < GF; ++s) {
      const int p = f.pv[s];
      const cx<R> b = rdlane(z, p);
      if (p != 0) {   // uniform: exchange rows col and col + p
        const cx<R> a = rdlane(z, 0);
        z.re = lane == p ? a.re : (lane == 0 ? b.re : z.re);
        z.im = lane == p ? a.im : (lane == 0 ? b.im : z.im);
      }
      z = rol1(cfms(z, (R)f.l[s].re, (R)f.l[s].im, b));
    }
    const int o = lane - (64 - GF);   // lane 64 - GF + s holds row c0 + s
    if (o >= 0 && c0 + o < N) vec[c0 + o] = z;
  };
  FwdSet fa, fb;
  load_fwd(0, fa);
  for (int c0 = 0; c0 < N; c0 += 2 * GF) {
    load_fwd(c0 + GF, fb);
    fwd_group(c0, fa);
    load_fwd(c0 + 2 * GF, fa);
    fwd_group(c0 + GF, fb);
  }
  __syncthreads();   // the back substitution reads rows other lanes stored
  // ---- back: U by columns; lanes 0 .. KU-1 hold rows col .. col - KU + 1
  const bool umul = lane < KU;
  const bool bent = lane >= KU && lane < KU + GB;
  const long long uzero = (long long)N * KU;
  cx<R> r = ldv(umul && N - 1 - lane >= 0, (long long)N - 1 - lane);
  struct BwdSet {
    cx<F> u[GB];
    cx<R> ent;
  };
  const unsigned umoff = (unsigned)lane * (unsigned)sizeof(cx<F>);
  auto load_bwd = [&](int c0, BwdSet& b) {
    if constexpr (PAIR) {
      // N - 1 - c0 is a multiple of the (even) group: steps c0 - s and
      // c0 - s - 1 are pair (N - 1 - c0 + s) / 2
      const long long pzero = (long long)NP * KU;
#pragma unroll
      for (int s = 0; s < GB; s += 2) {
        const int q = min((N - 1 - c0 + s) >> 1, NP - 1);   // pairs past the start: the last pair
        const long long cb = (long long)q * KU;
        const unsigned off = umul ? (unsigned)lane * 16u : (unsigned)((pzero - cb) * 16);
        const float4 v = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(Ut) + cb * 16 + off);
        b.u[s] = cx<F>{v.x, v.y};
        b.u[s + 1] = cx<F>{v.z, v.w};
      }
    } else {
#pragma unroll
      for (int s = 0; s < GB; ++s) {
        const int col = max(c0 - s, 0);   // steps past the start run on row 0's column
        const long long cb = (long long)col * KU;
        const unsigned off = umul ? umoff : (unsigned)((uzero - cb) * (long long)sizeof(cx<F>));
        b.u[s] = *reinterpret_cast<const cx<F>*>(reinterpret_cast<const char*>(Ut + cb) + off);
      }
    }
    b.ent = vec[max(c0 - lane, 0)];
  };
  auto bwd_group = [&](int c0, const BwdSet& b) {
    if (bent) r = b.ent;
#pragma unroll
    for (int s = 0; s < GB; ++s) {
      // lane d >= 1: r_d - (U(col-d, col) / U(col, col)) r_0; lane 0:
      // r_0 - (1 - 1/U(col, col)) r_0 = r_0 / U(col, col), the unknown
      r = rol1(cfms(r, (R)b.u[s].re, (R)b.u[s].im, rdlane(r, 0)));
    }
    const int o = lane - (64 - GB);   // lane 64 - GB + s holds row c0 - s
    if (o >= 0 && c0 - o >= 0) vec[c0 - o] = r;
  };
  BwdSet ba, bb;
  load_bwd(N - 1, ba);
  for (int c0 = N - 1; c0 >= 0; c0 -= 2 * GB) {
    load_bwd(c0 - GB, bb);
    bwd_group(c0, ba);
    load_bwd(c0 - 2 * GB, ba);
    bwd_group(c0 - GB, bb);
  }
}

template <typename R>
const cx<R>* twx_of(const Ctx* c);
template <>
const cx<double>* twx_of<double>(const Ctx* c) {
  return reinterpret_cast<const cx<double>*>(c->fp_twx64);
}
template <>
const cx<float>* twx_of<float>(const Ctx* c) {
  return reinterpret_cast<const cx<float>*>(c->fp_twx32);
}
template <typename R>
const cx<R>* twz_of(const Ctx* c);
template <>
const cx<double>* twz_of<double>(const Ctx* c) {
  return reinterpret_cast<const cx<double>*>(c->fp_twz64);
}
template <>
const cx<float>* twz_of<float>(const Ctx* c) {
  return reinterpret_cast<const cx<float>*>(c->fp_twz32);
}

}  // namespace

// Workspace of the apply for nrhs systems: the spectrum and, in 3D, the
// x-transformed planes (complex, precision R).
size_t fourier_spec_bytes(const Ctx* c, int nrhs, size_t es) {
  const FGeom g = geom_of(c);
  return (size_t)nrhs * g.nz * g.mx * g.N * 2 * es;
}

// line pairs per workgroup of the x transforms (two LDS buffers of P n
// complex values and the twiddles within the x budget), and sequences per
// workgroup of the z transforms (within the z budget)
template <typename R>
int x_pairs(int n) {
  const int cap = (int)(fft_x_lds<R>() / sizeof(cx<R>));
  int P = (cap - n) / (2 * n);
  if (P > XMAX_PAIRS) P = XMAX_PAIRS;
  return P < 1 ? 1 : P;
}
template <typename R>
int z_seqs(int n) {
  const int cap = (int)(fft_z_lds<R>() / sizeof(cx<R>));
  int ub = (cap - n) / (2 * n);
  if (ub > 32) ub = 32;
  return ub < 1 ? 1 : ub;
}

template <typename R>
hipError_t fourier_apply(Ctx* c, int ishift, int nrhs, const R* r, R* z, const int* active, int shift_step,
                         long long sV, long long sA, hipStream_t s) {
  const FGeom g = geom_of(c);
  if (sV == 0) sV = c->n;
  const size_t es = sizeof(R);
  if (nrhs > c->fp_nrhs_cap) return hipErrorInvalidValue;
  cx<R>* A = reinterpret_cast<cx<R>*>(es == 8 ? c->fp_specA64 : c->fp_specA32);
  cx<R>* B = reinterpret_cast<cx<R>*>(es == 8 ? c->fp_specB64 : c->fp_specB32);
  const cx<R>* tx = twx_of<R>(c);
  const cx<R>* tz = twz_of<R>(c);
  const FPlan px = plan_of(g.nx), pz = plan_of(g.nz);
  const int P = x_pairs<R>(g.nx);
  const unsigned Pm = magic_of(P);
  const int npair = (g.nz * g.N + 1) / 2;
  const dim3 gx((unsigned)((npair + P - 1) / P), (unsigned)nrhs);
  const size_t xlds = (size_t)(g.nx + 2 * P * g.nx) * sizeof(cx<R>);
  const int ub = z_seqs<R>(g.nz);
  const unsigned ubm = magic_of(ub);
  const dim3 gz((unsigned)(g.mx * ((g.N + ub - 1) / ub)), (unsigned)nrhs);
  const size_t zlds = (size_t)(g.nz + 2 * ub * g.nz) * sizeof(cx<R>);
  // forward: x (into A), then z (A -> B) in 3D
  fft_x_fwd<R><<<gx, FFT_THREADS, xlds, s>>>(g, px, P, Pm, r, sV, tx, A, active, sA);
  cx<R>* spec = A;
  if (g.nd == 3) {
    fft_z<R><<<gz, FFT_THREADS, zlds, s>>>(g, pz, ub, ubm, A, tz, 0, B, active, sA);
    spec = B;
  }
  // longer back-substitution groups (more factor bytes in flight per
  // wavefront) when the packed U leaves the lanes for them
  const bool wide = g.KU + 2 * BS_GROUP_BACK_WIDE <= 64;
  const dim3 gb((unsigned)g.nmodes, (unsigned)nrhs);
  const cx<double>* L64 = (const cx<double>*)c->fp_L;
  const cx<double>* U64 = (const cx<double>*)c->fp_U;
  const cx<float>* L32 = (const cx<float>*)c->fp_L;
  const cx<float>* U32 = (const cx<float>*)c->fp_U;
  if (c->fp_f64 && wide)
    band_solve_kernel<double, R, BS_GROUP_BACK_WIDE, false><<<gb, 64, 0, s>>>(g, L64, U64, c->fp_piv, ishift,
                                                                              shift_step, spec, active, sA);
  else if (c->fp_f64)
    band_solve_kernel<double, R, BS_GROUP_BACK, false><<<gb, 64, 0, s>>>(g, L64, U64, c->fp_piv, ishift, shift_step,
                                                                         spec, active, sA);
  else if (wide)
    band_solve_kernel<float, R, BS_GROUP_BACK_WIDE, true><<<gb, 64, 0, s>>>(g, L32, U32, c->fp_piv, ishift,
                                                                            shift_step, spec, active, sA);
  else
    band_solve_kernel<float, R, BS_GROUP_BACK, true><<<gb, 64, 0, s>>>(g, L32, U32, c->fp_piv, ishift, shift_step,
                                                                       spec, active, sA);
  cx<R>* xin = spec;
  if (g.nd == 3) {
    fft_z<R><<<gz, FFT_THREADS, zlds, s>>>(g, pz, ub, ubm, B, tz, 1, A, active, sA);
    xin = A;
  }
  fft_x_inv<R><<<gx, FFT_THREADS, xlds, s>>>(g, px, P, Pm, xin, tx, z, sV, active, sA);
  const long long per = (long long)g.nv * g.nz * 2 * g.nx;
  zero_walls<R><<<dim3((unsigned)((per + 255) / 256), (unsigned)nrhs), 256, 0, s>>>(g, z, sV, active, sA);
  return hipGetLastError();
}
template hipError_t fourier_apply<double>(Ctx*, int, int, const double*, double*, const int*, int, long long,
                                          long long, hipStream_t);
template hipError_t fourier_apply<float>(Ctx*, int, int, const float*, float*, const int*, int, long long, long long,
                                         hipStream_t);

int fourier_setup(Ctx* c, const sa_precond_opts* o, int nshift, const double* shifts_host) {
  if (c->op.bcy != 1) return c->fail(SA_EINVAL, "sa_precond_setup: the mean-flow preconditioner needs walls in y");
  if (o->factor_prec != SA_F32 && o->factor_prec != SA_F64)
    return c->fail(SA_EINVAL, "sa_precond_setup: factor precision must be SA_F32 or SA_F64");
  const FGeom g = geom_of(c);
  // the probes' responses must not wrap onto each other along x and z, and
  // a mode's vector (complex FP64) and the x lines must fit in LDS
  if (g.nx < NOFF || (g.nd == 3 && g.nz < NOFF) || g.ny - 2 < 1)
    return c->fail(SA_EINVAL, "sa_precond_setup: the mean-flow preconditioner needs nx, nz >= %d", NOFF);
  if ((size_t)g.N * sizeof(cx<double>) > LDS_CAP || (size_t)g.nx * 3 * sizeof(cx<double>) > LDS_CAP ||
      (size_t)g.nz * 3 * sizeof(cx<double>) > LDS_CAP)
    return c->fail(SA_EINVAL, "sa_precond_setup: grid too large for the mean-flow preconditioner");
  // the banded solve keeps the window, a group's entering rows and the rows
  // it finishes in one wavefront: kl + 1 + 2 BS_GROUP <= 64 and
  // KW + 2 BS_GROUP_BACK <= 64 (kl = 4 nv - 1, KW = 8 nv - 1), i.e. nv <= 5
  if (c->nv > 5 || g.kl + 1 + 2 * BS_GROUP > 64 || g.KW + 2 * BS_GROUP_BACK > 64)
    return c->fail(SA_EINVAL, "sa_precond_setup: at most 5 variables");
  hipStream_t s = c->stream;
  const long long n = c->n, np = c->op.npts;
  const int nv = c->nv;
  // q_bar with its pointwise fields and base-derivative data
  double* qb = (double*)c->buffer("fp_qbar", sizeof(double) * (size_t)(nv + 3) * np, false);
  float* qb32 = (float*)c->buffer("fp_qbar32", sizeof(float) * (size_t)(nv + 3) * np, false);
  double* bd = (double*)c->buffer("fp_bdata", sizeof(double) * (size_t)base_data_fields(g.nd) * np, false);
  // zero_fill writes whole 16-byte words: the buffers it clears are padded
  int* flag = (int*)c->buffer("fp_flag", 16, false);
  double* P = (double*)c->buffer("fp_probe", sizeof(double) * (size_t)nv * n + 16, false);
  double* Y = (double*)c->buffer("fp_resp", sizeof(double) * (size_t)nv * n, false);
  const size_t nS = (size_t)g.N * g.KW * NOFF * NOFF;
  double* S = (double*)c->buffer("fp_stencil", sizeof(double) * nS + 16, false);
  double* sh = (double*)c->buffer("fp_shifts", sizeof(double) * nshift, false);
  const size_t fs = o->factor_prec == SA_F64 ? sizeof(double) : sizeof(float);
  const size_t nfac = (size_t)nshift * g.nmodes * g.N;
  // per (shift, mode): N KW (U) or N kl (L) entries and one zero slot
  const size_t nfm = (size_t)nshift * g.nmodes;
  void* Uf = c->buffer("fp_U", 2 * fs * nfm * ((size_t)g.N * g.KW + 1), false);
  void* Lf = c->buffer("fp_L", 2 * fs * nfm * ((size_t)g.N * g.kl + 1), false);
  int* pv = (int*)c->buffer("fp_piv", sizeof(int) * nfac, false);
  const int cap = nshift > 1 ? nshift : 1;
  void* A64 = c->buffer("fp_specA64", fourier_spec_bytes(c, cap, 8), false);
  void* B64 = c->buffer("fp_specB64", fourier_spec_bytes(c, cap, 8), false);
  void* A32 = c->buffer("fp_specA32", fourier_spec_bytes(c, cap, 4), false);
  void* B32 = c->buffer("fp_specB32", fourier_spec_bytes(c, cap, 4), false);
  void* tx64 = c->buffer("fp_twx64", 16 * (size_t)g.nx, false);
  void* tx32 = c->buffer("fp_twx32", 8 * (size_t)g.nx, false);
  void* tz64 = c->buffer("fp_twz64", 16 * (size_t)g.nz, false);
  void* tz32 = c->buffer("fp_twz32", 8 * (size_t)g.nz, false);
  if (!qb || !qb32 || !bd || !flag || !P || !Y || !S || !sh || !Uf || !Lf || !pv || !A64 || !B64 || !A32 || !B32 ||
      !tx64 || !tx32 || !tz64 || !tz32)
    return c->fail(SA_ENOMEM, "sa_precond_setup: out of device memory");
  // twiddle tables e^{-2 pi i m / n}
  {
    std::vector<double> h64(2 * (size_t)std::max(g.nx, g.nz));
    std::vector<float> h32(h64.size());
    for (int pass = 0; pass < 2; ++pass) {
      const int len = pass == 0 ? g.nx : g.nz;
      for (int m = 0; m < len; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)len;
        h64[2 * m] = std::cos(a);
        h64[2 * m + 1] = std::sin(a);
        h32[2 * m] = (float)h64[2 * m];
        h32[2 * m + 1] = (float)h64[2 * m + 1];
      }
      hipError_t e = hipMemcpy(pass == 0 ? tx64 : tz64, h64.data(), 16 * (size_t)len, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(pass == 0 ? tx32 : tz32, h32.data(), 8 * (size_t)len, hipMemcpyHostToDevice);
      if (e != hipSuccess) return c->hip_fail(e, "sa_precond_setup twiddles");
    }
  }
  hipError_t e = hipMemcpyAsync(sh, shifts_host, sizeof(double) * nshift, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return c->hip_fail(e, "sa_precond_setup shifts");
  mean_base_kernel<<<(unsigned)(nv * g.ny), 256, 0, s>>>(g, c->base64, qb);
  zero_fill(flag, 16, s);
  // the explicit-difference operator of q_bar (also for a compact-scheme
  // context: there the preconditioner is the cheaper explicit operator)
  OpParams op = c->op;
  op.iso[0] = op.iso[1] = nullptr;
  op.scheme = 0;
  e = launch_base_derive(op, qb, qb32, flag, s);
  if (e == hipSuccess) e = launch_base_data(op, qb, bd, s);
  if (e != hipSuccess) return c->hip_fail(e, "sa_precond_setup mean base");
  zero_fill(S, sizeof(double) * nS, s);
  for (int col = 0; col < NCOL; ++col) {
    zero_fill(P, sizeof(double) * (size_t)nv * n, s);
    const int nrow = g.ny - 2;
    probe_kernel<<<(unsigned)((nv * nrow + 255) / 256), 256, 0, s>>>(g, col, P);
    e = launch_jv<double>(op, qb, bd, P, Y, nv, 0.0, nullptr, s, -1);
    if (e != hipSuccess) return c->hip_fail(e, "sa_precond_setup probes");
    gather_kernel<<<(unsigned)((nS + 255) / 256), 256, 0, s>>>(g, col, Y, S);
  }
  zero_fill(flag, 16, s);
  const unsigned nblk = (unsigned)((long long)g.nmodes * nshift);
  if (o->factor_prec == SA_F64)
    band_lu_kernel<double><<<nblk, 64, 0, s>>>(g, S, sh, (cx<double>*)Uf, (cx<double>*)Lf, pv, flag);
  else
    band_lu_kernel<float><<<nblk, 64, 0, s>>>(g, S, sh, (cx<float>*)Uf, (cx<float>*)Lf, pv, flag);
  e = hipGetLastError();
  if (e != hipSuccess) return c->hip_fail(e, "sa_precond_setup factor");
  int hflag = 0;
  e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return c->hip_fail(e, "sa_precond_setup sync");
  if (hflag) return c->fail(SA_ESINGULAR, "sa_precond_setup: zero pivot in a mode of the mean-flow operator");
  // the common extent of U's columns, then the packed layout the solve reads
  c->fp_ku = 0;
  zero_fill(flag, 16, s);
  const long long nfb = (long long)nshift * g.nmodes;
  const unsigned ny_grid = (unsigned)std::min<long long>(nfb, 4096);
  const dim3 gext((unsigned)((g.N * g.KW + 255) / 256), (unsigned)std::min<long long>(nfb, 64));
  if (o->factor_prec == SA_F64)
    u_extent_kernel<double><<<gext, 256, 0, s>>>(g, nfb, (const cx<double>*)Uf, flag);
  else
    u_extent_kernel<float><<<gext, 256, 0, s>>>(g, nfb, (const cx<float>*)Uf, flag);
  int hext = 0;
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&hext, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return c->hip_fail(e, "sa_precond_setup extent");
  const int KU = std::min(hext + 1, g.KW);
  void* Uc = c->buffer("fp_Uc", 2 * fs * nfm * ((size_t)g.N * KU + 1), false);
  if (!Uc) return c->fail(SA_ENOMEM, "sa_precond_setup: out of device memory");
  const dim3 gpk((unsigned)((g.N * KU + 1 + 255) / 256), ny_grid);
  if (o->factor_prec == SA_F64)
    u_pack_kernel<double><<<gpk, 256, 0, s>>>(g, nfb, KU, (const cx<double>*)Uf, (cx<double>*)Uc);
  else
    u_pack_kernel<float><<<gpk, 256, 0, s>>>(g, nfb, KU, (const cx<float>*)Uf, (cx<float>*)Uc);
  e = hipGetLastError();
  if (e != hipSuccess) return c->hip_fail(e, "sa_precond_setup pack");
  void* Lsolve = Lf;
  void* Usolve = Uc;
  if (o->factor_prec != SA_F64) {
    // FP32 factors: the step-pair layout (16-byte loads, one per two steps)
    const size_t NP = (size_t)(g.N + 1) / 2;
    void* Lp = c->buffer("fp_Lp", 16 * nfm * (NP * g.kl + 1), false);
    void* Up = c->buffer("fp_Up", 16 * nfm * (NP * KU + 1), false);
    if (!Lp || !Up) return c->fail(SA_ENOMEM, "sa_precond_setup: out of device memory");
    const dim3 gpl((unsigned)((NP * g.kl + 1 + 255) / 256), ny_grid);
    const dim3 gpu((unsigned)((NP * KU + 1 + 255) / 256), ny_grid);
    pair_rows_kernel<<<gpl, 256, 0, s>>>(g.N, g.kl, 0, nfb, (const cx<float>*)Lf, (cx<float>*)Lp);
    pair_rows_kernel<<<gpu, 256, 0, s>>>(g.N, KU, 1, nfb, (const cx<float>*)Uc, (cx<float>*)Up);
    e = hipGetLastError();
    if (e != hipSuccess) return c->hip_fail(e, "sa_precond_setup pairs");
    Lsolve = Lp;
    Usolve = Up;
  }
  c->fp_ku = KU;
  c->fp_U = Usolve;
  c->fp_L = Lsolve;
  c->fp_piv = pv;
  c->fp_f64 = o->factor_prec == SA_F64;
  c->fp_specA64 = A64;
  c->fp_specB64 = B64;
  c->fp_specA32 = A32;
  c->fp_specB32 = B32;
  c->fp_twx64 = tx64;
  c->fp_twx32 = tx32;
  c->fp_twz64 = tz64;
  c->fp_twz32 = tz32;
  c->fp_nrhs_cap = cap;
  return SA_OK;
}

}  // namespace sa
