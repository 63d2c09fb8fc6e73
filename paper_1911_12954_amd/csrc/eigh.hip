// FP64 symmetric eigendecomposition of the HOSVD Gram matrices (Fig. 1B of
// the paper: the isometries are the leading eigenvectors of the two-site
// environment) and the selection of the truncated isometry.
//
// Eigensolver: cyclic two-sided Jacobi in parallel (round-robin) order, one
// workgroup per matrix.  Each round rotates n/2 disjoint index pairs: rows
// first (A <- J^T A), then columns (A <- A J, V <- V J).  A sweep is n-1
// rounds; sweeps repeat until the off-diagonal Frobenius norm falls below
// 1e-14 of the matrix norm, plus one final sweep.  The matrix and vectors live in global memory
// (they are small and stay in L2); the rotation parameters of a round are
// in LDS.  Everything is deterministic: fixed pairing order, fixed
// reduction trees.
#include <cmath>

#include "internal.h"

namespace trg {
namespace {

constexpr int EIGH_THREADS = 512;
constexpr int MAX_N = 1024;
constexpr int MAX_SWEEPS = 40;

__device__ inline double wg_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = EIGH_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(EIGH_THREADS)
jacobi_kernel(double *Aall, double *wall, double *Vall, int *sweeps_out, int n) {
  __shared__ double sh[EIGH_THREADS];
  __shared__ int pp[MAX_N / 2], pq[MAX_N / 2];
  __shared__ double pc[MAX_N / 2], ps[MAX_N / 2];
  __shared__ double wdiag[MAX_N];
  __shared__ int rank[MAX_N];

  const int b = blockIdx.x;
  double *A = Aall + size_t(b) * n * n;
  double *V = Vall + size_t(b) * n * n;
  double *w = wall + size_t(b) * n;
  const int t = threadIdx.x;
  const int n2 = n * n;

  for (int i = t; i < n2; i += EIGH_THREADS) V[i] = (i / n == i % n) ? 1.0 : 0.0;
  double fro = 0.0;
  for (int i = t; i < n2; i += EIGH_THREADS) fro += A[i] * A[i];
  __syncthreads();
  const double norm2 = wg_sum(fro, sh);

  const int np = (n + 1) & ~1;  // even number of players; index n is a dummy
  const int half = np / 2;
  // converged once the off-diagonal norm is below 1e-14 of the matrix norm;
  // one more sweep then brings it to the rounding level
  int used = -1;
  bool last = false;
  for (int sweep = 0; sweep <= MAX_SWEEPS; ++sweep) {
    if (last) {
      used = sweep;
      break;
    }
    double off = 0.0;
    for (int i = t; i < n2; i += EIGH_THREADS)
      if (i / n != i % n) off += A[i] * A[i];
    const double offs = wg_sum(off, sh);
    if (offs == 0.0 || norm2 == 0.0) {
      used = sweep;
      break;
    }
    if (offs <= 1e-28 * norm2) last = true;
    if (sweep == MAX_SWEEPS) break;
    for (int r = 0; r < np - 1; ++r) {
      // circle pairing: player np-1 fixed, the others rotate
      for (int j = t; j < half; j += EIGH_THREADS) {
        int p, q;
        if (j == 0) {
          p = r;
          q = np - 1;
        } else {
          p = (r + j) % (np - 1);
          q = (r - j + (np - 1)) % (np - 1);
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * n + q];
          if (apq != 0.0) {
            const double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
            const double tt = copysign(1.0, tau) / (fabs(tau) + hypot(1.0, tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        pp[j] = p;
        pq[j] = q < n ? q : p;
        pc[j] = c;
        ps[j] = s;
      }
      __syncthreads();
      // rows: A[p,:], A[q,:] <- c A[p,:] - s A[q,:], s A[p,:] + c A[q,:]
      for (int e = t; e < half * n; e += EIGH_THREADS) {
        const int j = e / n, col = e % n;
        const int p = pp[j], q = pq[j];
        if (p == q) continue;
        const double c = pc[j], s = ps[j];
        const double ap = A[p * n + col], aq = A[q * n + col];
        A[p * n + col] = c * ap - s * aq;
        A[q * n + col] = s * ap + c * aq;
      }
      __syncthreads();
      // columns of A and V
      for (int e = t; e < half * n; e += EIGH_THREADS) {
        const int j = e / n, row = e % n;
        const int p = pp[j], q = pq[j];
        if (p == q) continue;
        const double c = pc[j], s = ps[j];
        const double ap = A[row * n + p], aq = A[row * n + q];
        A[row * n + p] = c * ap - s * aq;
        A[row * n + q] = s * ap + c * aq;
        const double vp = V[row * n + p], vq = V[row * n + q];
        V[row * n + p] = c * vp - s * vq;
        V[row * n + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  if (t == 0) sweeps_out[b] = used;

  // sort descending (ties by index): rank of each eigenvalue
  for (int i = t; i < n; i += EIGH_THREADS) wdiag[i] = A[i * n + i];
  __syncthreads();
  for (int i = t; i < n; i += EIGH_THREADS) {
    const double v = wdiag[i];
    int rk = 0;
    for (int j = 0; j < n; ++j) rk += (wdiag[j] > v) || (wdiag[j] == v && j < i);
    rank[i] = rk;
  }
  __syncthreads();
  for (int i = t; i < n; i += EIGH_THREADS) w[rank[i]] = wdiag[i];
  // move V to A (scratch), then scatter columns into sorted order
  for (int i = t; i < n2; i += EIGH_THREADS) A[i] = V[i];
  __syncthreads();
  for (int i = t; i < n2; i += EIGH_THREADS) {
    const int row = i / n, col = i % n;
    V[row * n + rank[col]] = A[i];
  }
}

// ------------------------------------------ tridiagonalisation + QL (large n) ---
// For larger orders a sweep-based Jacobi streams the whole matrix through one
// CU thousands of times.  This solver reduces A to tridiagonal form with
// Householder reflections (A <- H A H, H = I - 2 v v^T / v^T v, one column at
// a time), accumulates Q = H_0 H_1 ..., then diagonalises the tridiagonal
// matrix by implicit QL iterations with Wilkinson-type shifts; the QL step
// follows the order of the published tql2 procedure (Bowdler, Martin, Reinsch
// and Wilkinson, Numer. Math. 11 (1968) 293-306).  Thread 0 runs
// the scalar QL recurrence and records the Givens rotations of one sweep in
// LDS; all threads then apply the sweep to their rows of the eigenvector
// matrix.  Deterministic (fixed order everywhere).
constexpr int TQ_THREADS = 1024;
constexpr int TQ_MAX = 1024;
constexpr int TQ_CHUNK = 16;

__device__ inline double tq_max(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = TQ_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ inline double tq_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = TQ_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// out[j] = sum_i v[i] B[i][j] for the m x m block B (row stride ld) of a
// matrix in global memory, j < m: column j is summed by one thread, or by
// two (the upper and the lower half of the rows, added through w2) when 2 m
// fits the workgroup; loads go out eight at a time so that several are in
// flight per thread.  Ends with a barrier.
__device__ inline void tq_colvec(const double *B, int ld, int m, const double *v, double *out, double *w2, int t) {
  const bool split = 2 * m <= TQ_THREADS;
  const int half = split ? t / (TQ_THREADS / 2) : 0;
  const int j0 = split ? t % (TQ_THREADS / 2) : t;
  const int stride = split ? TQ_THREADS / 2 : TQ_THREADS;
  const int i0 = split ? half * (m / 2) : 0, i1 = split ? (half ? m : m / 2) : m;
  for (int j = j0; j < m; j += stride) {
    double a0 = 0.0, a1 = 0.0;
    int i = i0;
    for (; i + 8 <= i1; i += 8) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = B[size_t(i + u) * ld + j];
#pragma unroll
      for (int u = 0; u < 8; u += 2) {
        a0 += x[u] * v[i + u];
        a1 += x[u + 1] * v[i + u + 1];
      }
    }
    for (; i < i1; ++i) a0 += B[size_t(i) * ld + j] * v[i];
    if (half) w2[j] = a0 + a1;
    else out[j] = a0 + a1;
  }
  __syncthreads();
  if (split)
    for (int j = t; j < m; j += TQ_THREADS) out[j] += w2[j];
  __syncthreads();
}

// Householder reduction of the symmetric n x n matrix A (global memory) to
// tridiagonal form, diagonal in dd and subdiagonal in ee (LDS); reflector k
// is left in column k of V (rows k+1..n-1), scaled so that H_k = I - u u^T.
// A is overwritten.  Every thread of the workgroup calls it.
__device__ void tq_tridiagonalise(double *A, double *V, int n, double *sh, double *vv, double *ww, double *w2,
                                  double *dd, double *ee) {
  const int t = threadIdx.x;
  for (int i = t; i < n * n; i += TQ_THREADS) V[i] = 0.0;
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;              // length of the column below the diagonal
    // The reflector is built from the column scaled by a power of two that
    // brings its largest entry into [1, 2): H = I - 2 v v^T / v^T v does not
    // depend on the scale of v, and sums of squares of columns far below
    // the matrix's scale (a parity block of a Gram whose weights are
    // 1e-150 of the other block's) neither underflow nor make tau overflow.
    double amax = 0.0;
    for (int i = t; i < m; i += TQ_THREADS) {
      const double x = A[(k + 1 + i) * n + k];
      vv[i] = x;
      amax = fmax(amax, fabs(x));
    }
    amax = tq_max(amax, sh);
    if (amax == 0.0) continue;           // column already reduced: H = I
    int ex;
    (void)frexp(amax, &ex);
    double s2 = 0.0;
    for (int i = t; i < m; i += TQ_THREADS) {
      const double x = ldexp(vv[i], -ex);
      vv[i] = x;
      s2 += x * x;
    }
    const double nrm2 = tq_sum(s2, sh);
    const double x0 = vv[0];
    const double alpha = x0 >= 0.0 ? -sqrt(nrm2) : sqrt(nrm2);
    const double vtv = nrm2 - 2.0 * alpha * x0 + alpha * alpha;  // |x - alpha e1|^2
    __syncthreads();
    if (t == 0) vv[0] = x0 - alpha;
    __syncthreads();
    if (!(vtv > 0.0)) continue;          // column already reduced: H = I
    const double tau = 2.0 / vtv;
    // p = tau A_sub v  (A symmetric: column access, coalesced across threads)
    tq_colvec(A + (k + 1) * n + (k + 1), n, m, vv, ww, w2, t);
    for (int j = t; j < m; j += TQ_THREADS) ww[j] *= tau;
    __syncthreads();
    double pv = 0.0;
    for (int i = t; i < m; i += TQ_THREADS) pv += ww[i] * vv[i];
    const double K = 0.5 * tau * tq_sum(pv, sh);
    for (int j = t; j < m; j += TQ_THREADS) ww[j] -= K * vv[j];   // w = p - K v
    __syncthreads();
    // A_sub <- A_sub - v w^T - w v^T (TQ_CHUNK independent elements per
    // thread loaded before any is stored, so their loads overlap)
    for (int base = t; base < m * m; base += TQ_THREADS * TQ_CHUNK) {
      double a[TQ_CHUNK];
#pragma unroll
      for (int u = 0; u < TQ_CHUNK; ++u) {
        const int idx = base + u * TQ_THREADS;
        if (idx < m * m) a[u] = A[(k + 1 + idx / m) * n + (k + 1 + idx % m)];
      }
#pragma unroll
      for (int u = 0; u < TQ_CHUNK; ++u) {
        const int idx = base + u * TQ_THREADS;
        if (idx < m * m) {
          const int i = idx / m, j = idx % m;
          A[(k + 1 + i) * n + (k + 1 + j)] = a[u] - (vv[i] * ww[j] + ww[i] * vv[j]);
        }
      }
    }
    for (int i = t; i < m; i += TQ_THREADS) {
      const double val = i == 0 ? ldexp(alpha, ex) : 0.0;
      A[(k + 1 + i) * n + k] = val;
      A[k * n + (k + 1 + i)] = val;
      V[(k + 1 + i) * n + k] = vv[i] * sqrt(tau);   // scaled: H = I - u u^T
    }
    __syncthreads();
  }
  for (int i = t; i < n; i += TQ_THREADS) {
    dd[i] = A[i * n + i];
    ee[i] = i + 1 < n ? A[(i + 1) * n + i] : 0.0;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(TQ_THREADS)
tridiag_ql_kernel(double *Aall, double *wall, double *Vall, int *status, int n) {
  __shared__ double sh[TQ_THREADS];
  __shared__ double vv[TQ_MAX], ww[TQ_MAX], w2[TQ_MAX];
  __shared__ double dd[TQ_MAX], ee[TQ_MAX];
  __shared__ double rc[TQ_MAX], rs[TQ_MAX];
  __shared__ int rank[TQ_MAX];
  __shared__ int sweep_lo, sweep_hi, done_flag, iters_total;
  const int b = blockIdx.x;
  double *A = Aall + size_t(b) * n * n;
  double *V = Vall + size_t(b) * n * n;   // Householder vectors, then Q, then eigenvectors
  double *w = wall + size_t(b) * n;
  const int t = threadIdx.x;

  // ---- Householder tridiagonalisation; v_k stored in column k of V (rows k+1..n-1)
  tq_tridiagonalise(A, V, n, sh, vv, ww, w2, dd, ee);
  // ---- Q = H_0 H_1 ... H_{n-3}, built backwards in A (Q_k = H_k Q_{k+1})
  for (int i = t; i < n * n; i += TQ_THREADS) A[i] = (i / n == i % n) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    const int m = n - k - 1;
    for (int i = t; i < m; i += TQ_THREADS) vv[i] = V[(k + 1 + i) * n + k];
    __syncthreads();
    // ww[j] = sum_i u_i Q[k+1+i][k+1+j]; then Q_sub -= u ww^T
    tq_colvec(A + (k + 1) * n + (k + 1), n, m, vv, ww, w2, t);
    __syncthreads();
    for (int base = t; base < m * m; base += TQ_THREADS * TQ_CHUNK) {
      double a[TQ_CHUNK];
#pragma unroll
      for (int u = 0; u < TQ_CHUNK; ++u) {
        const int idx = base + u * TQ_THREADS;
        if (idx < m * m) a[u] = A[(k + 1 + idx / m) * n + (k + 1 + idx % m)];
      }
#pragma unroll
      for (int u = 0; u < TQ_CHUNK; ++u) {
        const int idx = base + u * TQ_THREADS;
        if (idx < m * m) {
          const int i = idx / m, j = idx % m;
          A[(k + 1 + i) * n + (k + 1 + j)] = a[u] - vv[i] * ww[j];
        }
      }
    }
    __syncthreads();
  }
  // ---- Z = Q^T into V (the Householder vectors are no longer needed), so
  // that a rotation of columns (i, i+1) of Q reads and writes two contiguous
  // rows of Z across the threads
  for (int idx = t; idx < n * n; idx += TQ_THREADS) {
    const int r = idx / n, c = idx % n;
    V[c * n + r] = A[idx];
  }
  __syncthreads();
  // ---- implicit QL on (dd, ee) with rotations applied to the columns of Q.
  // An off-diagonal entry deflates when it is at the rounding level of its
  // neighbours or of the whole matrix (anorm): next to rounding-level zero
  // diagonals (rank-deficient Grams) a purely relative test never fires.
  __shared__ double anorm;
  if (t == 0) {
    iters_total = 0;
    done_flag = 0;
    double md = 0.0, me = 0.0;
    for (int i = 0; i < n; ++i) {
      md = fmax(md, fabs(dd[i]));
      me = fmax(me, fabs(ee[i]));
    }
    anorm = md + me;
  }
  __syncthreads();
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    while (true) {
      // Thread 0's sweep is one dependent chain of FP64 operations per
      // rotation, so each Givens rotation takes r, c, s from one reciprocal
      // square root refined by two Newton steps (y <- y (3 - x y^2) / 2
      // doubles the correct bits of the hardware estimate) instead of hypot
      // and two divisions; f and g are first scaled by the power of two that
      // brings the larger into [1, 2), so that f^2 + g^2 neither underflows
      // nor overflows (f = g = 0 is the zero rotation).
      if (t == 0) {
        int mm = l;
        for (; mm < n - 1; ++mm) {
          const double s = fabs(dd[mm]) + fabs(dd[mm + 1]);
          if (fabs(ee[mm]) <= 2.220446049250313e-16 * (s + anorm)) break;
        }
        done_flag = (mm == l) || iter >= 60;
        if (iter >= 60) iters_total = -1000000;
        sweep_lo = l;
        sweep_hi = l - 1;   // empty rotation list unless a sweep runs
        if (!done_flag) {
          double g = (dd[l + 1] - dd[l]) / (2.0 * ee[l]);
          double r = hypot(g, 1.0);
          g = dd[mm] - dd[l] + ee[l] / (g + (g >= 0.0 ? fabs(r) : -fabs(r)));
          double s = 1.0, c = 1.0, p = 0.0;
          int i = mm - 1;
          bool underflow = false;
          for (; i >= l; --i) {
            const double f = s * ee[i], bb = c * ee[i];
            const double a = fmax(fabs(f), fabs(g));
            if (a == 0.0) {
              ee[i + 1] = 0.0;
              dd[i + 1] -= p;
              ee[mm] = 0.0;
              underflow = true;
              break;
            }
            int ex;
            (void)frexp(a, &ex);
            const double fs = ldexp(f, -ex), gs = ldexp(g, -ex);
            const double x = fma(fs, fs, gs * gs);   // in [1/4, 2)
            double y = __builtin_amdgcn_rsq(x);
            y = y * fma(-0.5 * x * y, y, 1.5);
            y = y * fma(-0.5 * x * y, y, 1.5);
            r = ldexp(x * y, ex);
            ee[i + 1] = r;
            s = fs * y;
            c = gs * y;
            g = dd[i + 1] - p;
            r = (dd[i] - g) * s + 2.0 * c * bb;
            p = s * r;
            dd[i + 1] = g + p;
            g = c * r - bb;
            rc[i] = c;
            rs[i] = s;
          }
          sweep_hi = mm - 1;
          sweep_lo = underflow ? i + 1 : l;
          if (!underflow) {
            dd[l] -= p;
            ee[l] = g;
            ee[mm] = 0.0;
          }
          ++iters_total;
        }
      }
      __syncthreads();
      if (done_flag) break;
      // rotations i = hi down to lo act on columns (i, i+1) of every row of
      // Q, i.e. on rows (i, i+1) of Z; the new entry i is carried in a
      // register into the next rotation.  Entries are read TQ_CHUNK at a
      // time before any of them is written back (each rotation reads entry
      // i and writes entry i + 1, so a chunk's reads all precede its
      // writes), which keeps TQ_CHUNK loads in flight instead of one.
      const int lo = sweep_lo, hi = sweep_hi;
      if (hi >= lo) {
        for (int row = t; row < n; row += TQ_THREADS) {
          double *z = V + row;
          double carry = z[size_t(hi + 1) * n];
          for (int i0 = hi; i0 >= lo; i0 -= TQ_CHUNK) {
            const int cnt = i0 - lo + 1 < TQ_CHUNK ? i0 - lo + 1 : TQ_CHUNK;
            double v[TQ_CHUNK];
#pragma unroll
            for (int u = 0; u < TQ_CHUNK; ++u)
              if (u < cnt) v[u] = z[size_t(i0 - u) * n];
#pragma unroll
            for (int u = 0; u < TQ_CHUNK; ++u)
              if (u < cnt) {
                const int i = i0 - u;
                const double zi = v[u], f = carry;
                v[u] = rs[i] * zi + rc[i] * f;      // new entry i + 1
                carry = rc[i] * zi - rs[i] * f;
              }
#pragma unroll
            for (int u = 0; u < TQ_CHUNK; ++u)
              if (u < cnt) z[size_t(i0 - u + 1) * n] = v[u];
          }
          z[size_t(lo) * n] = carry;
        }
      }
      ++iter;
      __syncthreads();
    }
  }
  if (t == 0) status[b] = iters_total >= 0 ? iters_total : -1;
  // ---- sort descending (ties by index) and write w, V
  for (int i = t; i < n; i += TQ_THREADS) {
    const double v = dd[i];
    int rk = 0;
    for (int j = 0; j < n; ++j) rk += (dd[j] > v) || (dd[j] == v && j < i);
    rank[i] = rk;
  }
  __syncthreads();
  for (int i = t; i < n; i += TQ_THREADS) w[rank[i]] = dd[i];
  // eigenvector col = row col of Z, sorted into column rank[col] of V
  for (int i = t; i < n * n; i += TQ_THREADS) {
    const int col = i / n, row = i % n;
    A[row * n + rank[col]] = V[i];
  }
  __syncthreads();
  for (int i = t; i < n * n; i += TQ_THREADS) V[i] = A[i];
}

// ------------------------------------------ leading eigenpairs (large n) ---
// The isometry selection needs every eigenvalue (the discarded weight, the
// degenerate-cut flag, the spectrum record) but the eigenvectors only of the
// kept indices and of the rest of a cluster of near-degenerate eigenvalues
// that the cut splits.  tridiag_top_kernel computes exactly that, with no
// serial QL sweeps and no n x n rotation accumulation:
//   1. Householder reduction to tridiagonal T (as for the full solver);
//   2. T splits into blocks where an off-diagonal is negligible against its
//      neighbours or exactly zero (as between the parity sectors of a
//      sector-ordered matrix); every eigenvalue of every block by bisection
//      on Sturm counts, one thread per eigenvalue, then sorted descending;
//   3. the number kk of vectors needed: k, extended while the next
//      eigenvalue continues a cluster (gap <= cluster_rel * lambda_max);
//   4. each needed eigenvector of its block by inverse iteration: LU with
//      partial pivoting of T_b - lambda I (pivots below eps ||T_b|| raised to
//      that size), three solves from a fixed start vector, each followed by
//      Gram-Schmidt against the block's earlier vectors and normalisation;
//      one wave per block, vectors in descending order (Wilkinson, The
//      Algebraic Eigenvalue Problem, 1965, ch. 5 and 9);
//   5. back-transformation by the reflectors, one wave per vector;
//   6. V gets the kk vectors as its leading columns (zeros elsewhere), w
//      every eigenvalue, status the number of vectors computed.
// work: per matrix 2 n^2 + TOP_WAVES * 6 n doubles (reflectors row by row,
// the vectors, each wave's LU factors and iterate).
constexpr int TOP_THREADS = 1024;
constexpr int TOP_WAVES = TOP_THREADS / 64;
constexpr int TOP_ITERS = 3;

__device__ inline double top_wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// fixed start vector of inverse iteration: entries in [-1, 1) from a hash of
// the vector's rank and the entry's index
__device__ inline double top_start(int r, int i) {
  uint32_t x = uint32_t(r) * 0x9E3779B1u ^ (uint32_t(i) + 0x7F4A7C15u) * 0x85EBCA77u;
  x ^= x >> 15;
  x *= 0x2C1B3C6Du;
  x ^= x >> 12;
  x *= 0x297A2D39u;
  x ^= x >> 15;
  return double(x) * (2.0 / 4294967296.0) - 1.0;
}

__global__ void __launch_bounds__(TOP_THREADS)
tridiag_top_kernel(double *Aall, double *wall, double *Vall, int *status, int n, int k, double cluster_rel,
                   double *workall) {
  __shared__ double sh[TOP_THREADS];
  __shared__ double vv[TQ_MAX], ww[TQ_MAX], w2[TQ_MAX];
  __shared__ double dd[TQ_MAX], ee[TQ_MAX];
  __shared__ int blk_of[TQ_MAX], bstart[TQ_MAX + 1], slot_of[TQ_MAX];
  __shared__ int nblk_s, kk_s;
  double *lam = vv, *ee2 = w2;   // reused once the reduction is done
  const int b = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double *A = Aall + size_t(b) * n * n;
  double *V = Vall + size_t(b) * n * n;
  double *w = wall + size_t(b) * n;
  double *work = workall + size_t(b) * (size_t(2) * n * n + size_t(TOP_WAVES) * 6 * n);
  double *Ur = work;                          // reflector j in row j (entries of rows j+1..n-1)
  double *Zv = work + size_t(n) * n;          // vector of rank r in row r
  double *scr = work + size_t(2) * n * n + size_t(wave) * 6 * n;
  const double eps = 2.220446049250313e-16;

  // ---- 1. tridiagonal T; reflectors out of V's columns into rows of Ur
  tq_tridiagonalise(A, V, n, sh, vv, ww, w2, dd, ee);
  for (int idx = t; idx < n * n; idx += TOP_THREADS) {
    const int j = idx / n, i = idx % n;
    Ur[idx] = (i < n - j - 1) ? V[size_t(j + 1 + i) * n + j] : 0.0;
    Zv[idx] = 0.0;
  }
  __syncthreads();
  // ---- 2. blocks, bisection
  if (t == 0) {
    int nb = 0;
    bstart[0] = 0;
    for (int i = 0; i + 1 < n; ++i) {
      const double lim = eps * sqrt(fabs(dd[i])) * sqrt(fabs(dd[i + 1]));
      if (ee[i] == 0.0 || fabs(ee[i]) <= lim) {
        ee[i] = 0.0;
        bstart[++nb] = i + 1;
      }
    }
    bstart[++nb] = n;
    nblk_s = nb;
  }
  __syncthreads();
  const int nblk = nblk_s;
  for (int i = t; i < n; i += TOP_THREADS) {
    int lo = 0, hi = nblk;   // bstart[lo] <= i < bstart[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (bstart[mid] <= i) lo = mid;
      else hi = mid;
    }
    blk_of[i] = lo;
    ee2[i] = ee[i] * ee[i];
  }
  __syncthreads();
  for (int slot = t; slot < n; slot += TOP_THREADS) {
    const int bb = blk_of[slot], s0 = bstart[bb], e0 = bstart[bb + 1];
    const int target = e0 - slot;   // (slot - s0 + 1)-th largest = target-th smallest
    double lo = 0.0, hi = 0.0, emax2 = 0.0;
    for (int i = s0; i < e0; ++i) {
      const double r = (i > s0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < e0 ? fabs(ee[i]) : 0.0);
      lo = i == s0 ? dd[i] - r : fmin(lo, dd[i] - r);
      hi = i == s0 ? dd[i] + r : fmax(hi, dd[i] + r);
      if (i + 1 < e0) emax2 = fmax(emax2, ee2[i]);
    }
    const double bn = fmax(fabs(lo), fabs(hi));
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
    lo -= 2.0 * eps * bn + pivmin;
    hi += 2.0 * eps * bn + pivmin;
    for (int it = 0; it < 120; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (!(mid > lo && mid < hi) || hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin) break;
      // Sturm count: eigenvalues of the block below mid
      int cnt = 0;
      double q = dd[s0] - mid;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
      for (int i = s0 + 1; i < e0; ++i) {
        q = (dd[i] - mid) - ee2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
      }
      if (cnt >= target) hi = mid;
      else lo = mid;
    }
    lam[slot] = 0.5 * (lo + hi);
  }
  __syncthreads();
  // ---- sort descending (ties by slot)
  for (int slot = t; slot < n; slot += TOP_THREADS) {
    const double v = lam[slot];
    int rk = 0;
    for (int u = 0; u < n; ++u) rk += (lam[u] > v) || (lam[u] == v && u < slot);
    w[rk] = v;
    slot_of[rk] = slot;
  }
  __syncthreads();
  // ---- 3. vectors needed
  if (t == 0) {
    const double tol = cluster_rel * fmax(w[0], 0.0);
    int bnd = k < n ? k : n;
    while (bnd < n && w[bnd - 1] - w[bnd] <= tol) ++bnd;
    kk_s = bnd;
  }
  __syncthreads();
  const int kk = kk_s;
  // ---- 4. inverse iteration, one wave per block
  double *DL = scr, *D = scr + n, *DU = scr + 2 * n, *DU2 = scr + 3 * n, *PV = scr + 4 * n, *X = scr + 5 * n;
  for (int bb = wave; bb < nblk; bb += TOP_WAVES) {
    const int s0 = bstart[bb], e0 = bstart[bb + 1], nb = e0 - s0;
    double bnorm = 0.0;
    for (int i = s0 + lane; i < e0; i += 64)
      bnorm = fmax(bnorm, fabs(dd[i]) + (i > s0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < e0 ? fabs(ee[i]) : 0.0));
    for (int off = 32; off > 0; off >>= 1) bnorm = fmax(bnorm, __shfl_xor(bnorm, off, 64));
    const double ptol = fmax(eps * bnorm, 2.2250738585072014e-308);
    for (int r = 0; r < kk; ++r) {
      const int slot = slot_of[r];
      if (slot < s0 || slot >= e0) continue;   // uniform: every lane reads the same slot
      const double sigma = w[r];
      if (lane == 0) {
        // LU with partial pivoting of T_b - sigma I (rows i, i+1 swapped where PV[i] = 1)
        for (int i = 0; i < nb; ++i) {
          D[i] = dd[s0 + i] - sigma;
          DL[i] = i + 1 < nb ? ee[s0 + i] : 0.0;
          DU[i] = DL[i];
          DU2[i] = 0.0;
        }
        for (int i = 0; i + 1 < nb; ++i) {
          if (fabs(D[i]) >= fabs(DL[i])) {
            PV[i] = 0.0;
            const double f = D[i] != 0.0 ? DL[i] / D[i] : 0.0;
            DL[i] = f;
            D[i + 1] -= f * DU[i];
          } else {
            PV[i] = 1.0;
            const double f = D[i] / DL[i];
            D[i] = DL[i];
            DL[i] = f;
            const double tmp = DU[i];
            DU[i] = D[i + 1];
            D[i + 1] = tmp - f * D[i + 1];
            if (i + 2 < nb) {
              DU2[i] = DU[i + 1];
              DU[i + 1] = -f * DU[i + 1];
            }
          }
        }
      }
      for (int i = lane; i < nb; i += 64) X[i] = top_start(r, i);
      __builtin_amdgcn_wave_barrier();
      __threadfence_block();
      for (int it = 0; it < TOP_ITERS; ++it) {
        if (lane == 0) {
          for (int i = 0; i + 1 < nb; ++i) {
            if (PV[i] == 0.0) {
              X[i + 1] -= DL[i] * X[i];
            } else {
              const double tmp = X[i];
              X[i] = X[i + 1];
              X[i + 1] = tmp - DL[i] * X[i];
            }
          }
          for (int i = nb - 1; i >= 0; --i) {
            double piv = D[i];
            if (fabs(piv) < ptol) piv = piv >= 0.0 ? ptol : -ptol;
            double v = X[i];
            if (i + 1 < nb) v -= DU[i] * X[i + 1];
            if (i + 2 < nb) v -= DU2[i] * X[i + 2];
            X[i] = v / piv;
          }
        }
        __builtin_amdgcn_wave_barrier();
        __threadfence_block();
        // Gram-Schmidt against the block's earlier vectors, then normalise
        for (int r2 = 0; r2 < r; ++r2) {
          const int sl2 = slot_of[r2];
          if (sl2 < s0 || sl2 >= e0) continue;
          const double *z = Zv + size_t(r2) * n + s0;
          double dot = 0.0;
          for (int i = lane; i < nb; i += 64) dot += z[i] * X[i];
          dot = top_wave_sum(dot);
          for (int i = lane; i < nb; i += 64) X[i] -= dot * z[i];
        }
        double nrm = 0.0;
        for (int i = lane; i < nb; i += 64) nrm += X[i] * X[i];
        nrm = top_wave_sum(nrm);
        const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
        for (int i = lane; i < nb; i += 64) X[i] *= inv;
        __builtin_amdgcn_wave_barrier();
        __threadfence_block();
      }
      for (int i = lane; i < nb; i += 64) Zv[size_t(r) * n + s0 + i] = X[i];
      __builtin_amdgcn_wave_barrier();
      __threadfence_block();
    }
  }
  __syncthreads();
  // ---- 5. back-transformation z <- H_0 ... H_{n-3} z, one wave per vector
  for (int r = wave; r < kk; r += TOP_WAVES) {
    double *z = Zv + size_t(r) * n;
    for (int j = n - 3; j >= 0; --j) {
      const int m = n - j - 1;
      const double *u = Ur + size_t(j) * n;
      double dot = 0.0;
      for (int i = lane; i < m; i += 64) dot += u[i] * z[j + 1 + i];
      dot = top_wave_sum(dot);
      if (dot != 0.0)
        for (int i = lane; i < m; i += 64) z[j + 1 + i] -= u[i] * dot;
    }
  }
  __syncthreads();
  // ---- 6. output
  for (int idx = t; idx < n * n; idx += TOP_THREADS) {
    const int i = idx / n, c = idx % n;
    V[idx] = c < kk ? Zv[size_t(c) * n + i] : 0.0;
  }
  if (t == 0) status[b] = kk;
}

// ------------------------------------------------------------- selection ---
constexpr int SEL_THREADS = 256;
constexpr double TIE_REL = 1e-10;      // side rule: backward only if clearly better
constexpr double SIGN_REL = 1e-9;      // "largest" coordinate within this relative window
constexpr double DEGEN_REL = 1e-8;     // degenerate-cut flag

__device__ inline double sel_reduce(double v, double *sh, bool is_max) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = SEL_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = is_max ? fmax(sh[t], sh[t + s]) : (sh[t] + sh[t + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ inline int sel_min_index(int v, int *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = SEL_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = min(sh[t], sh[t + s]);
    __syncthreads();
  }
  const int r = sh[0];
  __syncthreads();
  return r;
}

// w2/V2: the two sides' sorted eigensystems (side 0 backward, 1 forward).
__global__ void __launch_bounds__(SEL_THREADS)
select_kernel(const double *w2, const double *V2, const int *sweeps2, int n, int k, int force_side,
              double cluster_rel, double *U, double *rec_eps, int *rec_int, double *spectrum) {
  __shared__ double sh[SEL_THREADS];
  __shared__ int shi[SEL_THREADS];
  __shared__ double diag[MAX_N];
  __shared__ double col[MAX_N];
  const int t = threadIdx.x;

  double eps[2];
  for (int side = 0; side < 2; ++side) {
    double s = 0.0;
    for (int j = k + t; j < n; j += SEL_THREADS) s += fmax(w2[side * n + j], 0.0);
    eps[side] = sel_reduce(s, sh, false);
  }
  int side = (eps[0] < (1.0 - TIE_REL) * eps[1]) ? 0 : 1;
  if (force_side == 0 || force_side == 1) side = force_side;
  const double *w = w2 + side * n;
  const double *V = V2 + size_t(side) * n * n;
  for (int j = t; j < n; j += SEL_THREADS) spectrum[j] = w[j];

  // neighbouring eigenvalues within cluster_rel lambda_max form one
  // eigenspace, kept in its canonical basis; every larger gap is resolved by
  // the leading eigenvectors (plain truncated HOSVD)
  const double tol = cluster_rel * fmax(w[0], 0.0);
  int a = 0;
  while (a < k) {
    int bnd = a + 1;
    while (bnd < n && w[bnd - 1] - w[bnd] <= tol) ++bnd;  // cluster [a, bnd)
    const int stop = bnd < k ? bnd : k;
    for (int j = a; j < stop; ++j) {
      // remaining weight of each coordinate in the cluster's projector
      double mx = 0.0;
      for (int i = t; i < n; i += SEL_THREADS) {
        double dg = 0.0;
        for (int c = a; c < bnd; ++c) dg += V[i * n + c] * V[i * n + c];
        for (int c = a; c < j; ++c) dg -= U[i * k + c] * U[i * k + c];
        diag[i] = dg;
        mx = fmax(mx, dg);
      }
      mx = sel_reduce(mx, sh, true);
      int first = n;
      for (int i = t; i < n; i += SEL_THREADS)
        if (diag[i] >= (1.0 - SIGN_REL) * mx && i < first) first = i;
      const int r = sel_min_index(first, shi);
      // column of the remaining projector at coordinate r
      for (int i = t; i < n; i += SEL_THREADS) {
        double v = 0.0;
        for (int c = a; c < bnd; ++c) v += V[i * n + c] * V[r * n + c];
        for (int c = a; c < j; ++c) v -= U[i * k + c] * U[r * k + c];
        col[i] = v;
      }
      __syncthreads();
      const double inv = 1.0 / sqrt(col[r]);
      for (int i = t; i < n; i += SEL_THREADS) U[i * k + j] = col[i] * inv;
      __syncthreads();
    }
    a = bnd;
  }
  if (t == 0) {
    rec_eps[0] = eps[0];
    rec_eps[1] = eps[1];
    const int degenerate = (k < n && w[k - 1] > 0.0 && (w[k - 1] - w[k]) <= DEGEN_REL * w[k - 1]) ? 1 : 0;
    rec_int[0] = side;
    rec_int[1] = k;
    rec_int[2] = degenerate;
    rec_int[3] = sweeps2[side];
  }
}

}  // namespace

// Jacobi up to order JACOBI_MAX_N (accurate, and cheap while the matrix is
// small), tridiagonalisation + QL above.

void eigh_batched(double *A, double *w, double *V, int *sweeps, int n, int batch, hipStream_t st) {
  TRG_REQUIRE(n >= 1 && n <= MAX_N && batch >= 1, "eigh: order must be in [1, 1024]");
  if (n <= JACOBI_MAX_N)
    hipLaunchKernelGGL(jacobi_kernel, dim3(batch), dim3(EIGH_THREADS), 0, st, A, w, V, sweeps, n);
  else
    hipLaunchKernelGGL(tridiag_ql_kernel, dim3(batch), dim3(TQ_THREADS), 0, st, A, w, V, sweeps, n);
  TRG_HIP_CHECK(hipGetLastError());
}

size_t eigh_top_work_doubles(int n, int batch) {
  return size_t(batch) * (size_t(2) * n * n + size_t(TOP_WAVES) * 6 * n);
}

void eigh_top_batched(double *A, double *w, double *V, int *sweeps, int n, int batch, int k, double cluster_rel,
                      double *work, hipStream_t st) {
  TRG_REQUIRE(n >= 1 && n <= MAX_N && batch >= 1 && k >= 1, "eigh_top: bad sizes");
  if (n <= JACOBI_MAX_N) {
    hipLaunchKernelGGL(jacobi_kernel, dim3(batch), dim3(EIGH_THREADS), 0, st, A, w, V, sweeps, n);
  } else {
    TRG_REQUIRE(work != nullptr, "eigh_top: workspace missing");
    hipLaunchKernelGGL(tridiag_top_kernel, dim3(batch), dim3(TOP_THREADS), 0, st, A, w, V, sweeps, n, k,
                       cluster_rel, work);
  }
  TRG_HIP_CHECK(hipGetLastError());
}

void select_isometry(const double *w2, const double *V2, const int *sweeps2, int n, int k,
                     int force_side, double cluster_rel, SelectOut out, hipStream_t st) {
  TRG_REQUIRE(n >= 1 && n <= MAX_N && k >= 1 && k <= n, "select: bad sizes");
  TRG_REQUIRE(cluster_rel >= 0.0 && cluster_rel < 1.0, "select: bad degeneracy window");
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(SEL_THREADS), 0, st, w2, V2, sweeps2, n, k, force_side,
                     cluster_rel, out.U, out.rec_eps, out.rec_int, out.spectrum);
  TRG_HIP_CHECK(hipGetLastError());
}

}  // namespace trg
