// ATRG coarse-graining step (Sec. 2 and Fig. 2 of the paper) on the GPU.
//
// A site tensor is kept as two pieces T[b, f] = sum_l G[b, l] H[l, f]
// (b: the d backward legs, f: the d forward legs; D^{d+1} elements each).
// One step along mu:
//   1. canonical form T = U diag(s) V: QR of G and of H^T (shifted
//      CholeskyQR3) and the SVD of the small core, obtained from the
//      eigendecomposition of [[0, C], [C^T, 0]] (no squared condition number);
//      each singular-vector pair signed so that the first largest entry of
//      the left vector is positive;
//   2. the swap (dark-blue tensors of Fig. 2B): the matrix
//      M[(kA, b_perp), (f_perp, kB)] = sum_j Vt[kA, f_perp, j] Ut[j, b_perp, kB]
//      (Ut = U sqrt(s), Vt = sqrt(s) V) is truncated to rank Dcut by a
//      randomized SVD whose products M Z and M^T Z are applied in factored
//      form (two GEMMs each, 2 D^{d+2} r flops), with a Philox4x32-10 +
//      Box-Muller Gaussian trial matrix and q re-orthonormalised iterations;
//   3. HOSVD of the two-site product sum_l G H: Gram matrices of each
//      transverse leg pair in factored form (D^{d+3}), eigendecomposition and
//      the isometry selection shared with HOTRG;
//   4. the contraction that completes the block-spin transformation (red
//      dotted circle of Fig. 2B): the isometries applied to both pieces, the
//      dominant GEMM has M = D^4, K = D^2, N = D^3 in 4D;
//   5. normalisation c = sqrt(Tr[(G'^T G')(H' H'^T)]), pieces scaled by
//      c^{-1/2}, acc += 2^{-n} ln c.
// Impure tensors: impurity j is its own pair of pieces G_S[b, m], H_S[m, f];
// each impure two-site middle matrix (impurity on the lower site: H_S with
// the pure Ut; on the upper site: the pure Vt with G_S) gets its own
// randomized partial SVD of rank <= Dcut, the pure step's isometries
// compress both terms, which sit side by side along m (bond 2 Dcut), and the
// pieces take c^{-1/2} (and 1/2 on the forward piece).
// Contractions of named legs go through einsum2: both operands are packed
// (K-contiguous, zero-padded) by the strided map kernel and multiplied by the
// MFMA GEMM of the HOTRG join.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>

#include "context.h"

namespace trg {
namespace {

// ------------------------------------------------------------------ kernels ---
// U0[b, sigma] = e^{beta h sigma/2} prod_nu W[sigma, b_nu]; H0[sigma, b] the same
__global__ void atrg_ising_kernel(double *G, double *H, int d, double beta, double h) {
  const int n = 1 << d;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * n) return;
  const int sig = idx & 1, b = idx >> 1;
  const double spin = sig == 0 ? 1.0 : -1.0;
  const double c = sqrt(cosh(beta)), s = sqrt(sinh(beta));
  double v = exp(0.5 * beta * h * spin);
  for (int a = 0; a < d; ++a) v *= ((b >> (d - 1 - a)) & 1) ? spin * s : c;
  G[b * 2 + sig] = v;
  H[sig * n + b] = v;
}

// Forward pieces of the impurities on the backward piece U0 (bond sigma):
// HM[sigma, f] = sigma H0[sigma, f]; HE[sigma, f] = e^{beta h sigma/2}
// (h sigma prod_nu W[sigma, f_nu] + sum_nu 2 W'[sigma, f_nu] prod_{nu' != nu}
// W[sigma, f_nu']): the derivative of each bond weight on its forward end.
// Either pointer may be null.
__global__ void atrg_impurity_kernel(double *HE, double *HM, int d, double beta, double h) {
  const int n = 1 << d;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * n) return;
  const int sig = idx & 1, b = idx >> 1;
  const double spin = sig == 0 ? 1.0 : -1.0;
  const double ch = cosh(beta), sh = sinh(beta);
  const double w[2] = {sqrt(ch), spin * sqrt(sh)};
  const double dw[2] = {sh / (2.0 * sqrt(ch)), spin * ch / (2.0 * sqrt(sh))};
  const double pref = exp(0.5 * beta * h * spin);
  double v = pref;
  for (int a = 0; a < d; ++a) v *= w[(b >> (d - 1 - a)) & 1];
  double e = h * spin * v;
  for (int nu = 0; nu < d; ++nu) {
    double t = pref;
    for (int a = 0; a < d; ++a) {
      const int bit = (b >> (d - 1 - a)) & 1;
      t *= a == nu ? 2.0 * dw[bit] : w[bit];
    }
    e += t;
  }
  if (HM) HM[sig * n + b] = spin * v;
  if (HE) HE[sig * n + b] = e;
}

// Philox4x32 with 10 rounds (Salmon et al., SC'11)
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = uint64_t(0xD2511F53u) * c[0];
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c[2];
    const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
    const uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Omega[e] for e < count: counter (e, step, stream, 0), key (k0, k1);
// Box-Muller sqrt(-2 ln u1) cos(2 pi u2) with u = (w + 0.5) / 2^32.  Stream 0
// is the pure swap, 1 + 2 kind + term the impurity SVDs.
__global__ void trial_kernel(double *out, uint32_t count, uint32_t step, uint32_t stream, uint32_t k0,
                             uint32_t k1) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  uint32_t c[4] = {e, step, stream, 0u};
  philox4x32_10(c, k0, k1);
  const double u1 = (double(c[0]) + 0.5) / 4294967296.0;
  const double u2 = (double(c[1]) + 0.5) / 4294967296.0;
  out[e] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

// Upper Cholesky factor R of C + shift I (shift = shift_coef * trace C) and
// the matrix Rinv that maps Y to Q = Y Rinv; one workgroup, n <= 1024.  A
// pivot at or below 1e-26 of the largest diagonal entry marks its column as
// numerically dependent on the previous ones (rank-deficient Y): that column
// of Q is set to zero (column of Rinv zero) and its row of R is zero, so
// Y = Q R still holds and no division by a vanishing pivot occurs.
__global__ void __launch_bounds__(256)
chol_inv_kernel(const double *C, int n, double shift_coef, double *R, double *Rinv, int *err) {
  __shared__ double sh[256];
  __shared__ double shm[256];
  __shared__ int dead[1024];
  const int t = threadIdx.x;
  double tr = 0.0, mx = 0.0;
  for (int i = t; i < n; i += 256) {
    tr += C[i * n + i];
    mx = fmax(mx, C[i * n + i]);
  }
  sh[t] = tr;
  shm[t] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      sh[t] += sh[t + s];
      shm[t] = fmax(shm[t], shm[t + s]);
    }
    __syncthreads();
  }
  const double shift = shift_coef * sh[0];
  const double tol = 1e-26 * (shm[0] + shift);
  __syncthreads();
  for (int i = t; i < n * n; i += 256) {
    const int r = i / n, c = i % n;
    R[i] = r <= c ? C[i] + (r == c ? shift : 0.0) : 0.0;
    Rinv[i] = 0.0;
  }
  for (int i = t; i < n; i += 256) dead[i] = 0;
  __syncthreads();
  // row j of R from the rows above it
  for (int j = 0; j < n; ++j) {
    if (t == 0) {
      double dj = R[j * n + j];
      for (int k = 0; k < j; ++k) dj -= R[k * n + j] * R[k * n + j];
      if (!(dj > tol)) {
        if (!isfinite(dj)) *err |= 4;
        dead[j] = 1;
        dj = 1.0;
      }
      R[j * n + j] = sqrt(dj);
    }
    __syncthreads();
    const double rjj = R[j * n + j];
    const bool dj_dead = dead[j] != 0;
    for (int i = j + 1 + t; i < n; i += 256) {
      double v = R[j * n + i];
      for (int k = 0; k < j; ++k) v -= R[k * n + j] * R[k * n + i];
      R[j * n + i] = dj_dead ? 0.0 : v / rjj;
    }
    __syncthreads();
  }
  // inverse of the upper triangular R (dead rows are unit rows of R), one
  // column per thread; then dead columns of Rinv and dead rows of R vanish
  for (int j = t; j < n; j += 256) {
    for (int i = j; i >= 0; --i) {
      double v = (i == j) ? 1.0 : 0.0;
      for (int k = i + 1; k <= j; ++k) v -= R[i * n + k] * Rinv[k * n + j];
      Rinv[i * n + j] = v / R[i * n + i];
    }
  }
  __syncthreads();
  for (int i = t; i < n * n; i += 256) {
    const int r = i / n, c = i % n;
    if (dead[c]) Rinv[i] = 0.0;
    if (dead[r]) R[i] = 0.0;
  }
}

// The same factorisation for n <= 128, with the matrix in registers: wave w
// (of four) owns the rows p = w (mod 4) and lane l the columns l and l + 64,
// so thread (w, l) holds the 32 x 2 elements (w + 4 pp, l + 64 qq).
// Column j of the elimination: the wave owning row j takes the pivot from
// the lane holding the diagonal, scales the row (a pivot at or below the
// dead tolerance makes the row zero and its pivot 1) and publishes it as a
// 128-entry LDS row that is zero outside j < q < n; after one barrier every
// thread subtracts R[j][p] R[j][q] from all its elements, which leaves the
// rows at or above j unchanged (their entry of the published row is zero).
// The published row alternates between two buffers, so one barrier per
// column suffices: a buffer is written again only after the next barrier.
// R is also kept transposed in LDS (zero below its diagonal) for the
// inverse, which runs the same way from the last row up: row k of
// X = R^-1 is final once every row below it has been eliminated, is scaled
// by 1 / R[k][k] and published, and every thread subtracts R[p][k] X[k][q].
// All LDS reads are unconditional, so they go out together.
constexpr int CHOL_REG_MAX = 128;
constexpr int CHOL_THREADS = 256;
constexpr int CHOL_RT_LD = CHOL_REG_MAX + 1;   // row stride of R^T in LDS (lanes write a column)

__global__ void __launch_bounds__(CHOL_THREADS)
chol_inv_reg_kernel(const double *C, int n, double shift_coef, double *Rg, double *Rinv, int *err) {
  extern __shared__ double RT[];   // CHOL_REG_MAX x CHOL_RT_LD: RT[q][p] = R[p][q] for p < q, else 0
  __shared__ double sh[CHOL_THREADS];
  __shared__ double shm[CHOL_THREADS];
  __shared__ double row[2][CHOL_REG_MAX];
  __shared__ double pivs[CHOL_REG_MAX];
  __shared__ int dead[CHOL_REG_MAX];
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  double tr = 0.0, mx = 0.0;
  for (int i = t; i < n; i += CHOL_THREADS) {
    tr += C[i * n + i];
    mx = fmax(mx, C[i * n + i]);
  }
  sh[t] = tr;
  shm[t] = mx;
  for (int i = t; i < CHOL_REG_MAX * CHOL_RT_LD; i += CHOL_THREADS) RT[i] = 0.0;
  __syncthreads();
  for (int s = CHOL_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) {
      sh[t] += sh[t + s];
      shm[t] = fmax(shm[t], shm[t + s]);
    }
    __syncthreads();
  }
  const double shift = shift_coef * sh[0];
  const double tol = 1e-26 * (shm[0] + shift);
  double E[32][2];
#pragma unroll
  for (int pp = 0; pp < 32; ++pp)
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) {
      const int p = w + 4 * pp, q = l + 64 * qq;
      E[pp][qq] = (p <= q && q < n) ? C[p * n + q] + (p == q ? shift : 0.0) : 0.0;
    }
  for (int j = 0; j < n; ++j) {
    double *rj = row[j & 1];
    if (w == (j & 3)) {
      const int pj = j >> 2;
      double r0 = 0.0, r1 = 0.0;
#pragma unroll
      for (int pp = 0; pp < 32; ++pp)
        if (pp == pj) {
          r0 = E[pp][0];
          r1 = E[pp][1];
        }
      const double mine = (j >> 6) ? r1 : r0;
      const int lo = __builtin_amdgcn_readlane(int(__double_as_longlong(mine)), j & 63);
      const int hi = __builtin_amdgcn_readlane(int(__double_as_longlong(mine) >> 32), j & 63);
      const double dj = __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
      const bool isdead = !(dj > tol);
      const double piv = isdead ? 1.0 : sqrt(dj);
      const double inv = isdead ? 0.0 : 1.0 / piv;
      const double v0 = (l > j && l < n) ? r0 * inv : 0.0;
      const double v1 = (l + 64 > j && l + 64 < n) ? r1 * inv : 0.0;
      rj[l] = v0;
      rj[l + 64] = v1;
      if (l > j && l < n) RT[l * CHOL_RT_LD + j] = v0;
      if (l + 64 > j && l + 64 < n) RT[(l + 64) * CHOL_RT_LD + j] = v1;
      if (l == (j & 63)) {
        pivs[j] = piv;
        dead[j] = isdead ? 1 : 0;
        if (isdead && !isfinite(dj)) *err |= 4;
      }
    }
    __syncthreads();
    double rq[2], rv[32];
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) rq[qq] = rj[l + 64 * qq];
#pragma unroll
    for (int pp = 0; pp < 32; ++pp) rv[pp] = rj[w + 4 * pp];
#pragma unroll
    for (int pp = 0; pp < 32; ++pp)
#pragma unroll
      for (int qq = 0; qq < 2; ++qq) E[pp][qq] -= rv[pp] * rq[qq];
  }
  __syncthreads();
  // X = R^-1 in the same registers
#pragma unroll
  for (int pp = 0; pp < 32; ++pp)
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) {
      const int p = w + 4 * pp, q = l + 64 * qq;
      E[pp][qq] = (p == q && q < n) ? 1.0 : 0.0;
    }
  for (int k = n - 1; k >= 0; --k) {
    double *xk = row[k & 1];
    if (w == (k & 3)) {
      const int pk = k >> 2;
      const double ik = 1.0 / pivs[k];
#pragma unroll
      for (int pp = 0; pp < 32; ++pp)
        if (pp == pk) {
          E[pp][0] *= ik;
          E[pp][1] *= ik;
          xk[l] = E[pp][0];
          xk[l + 64] = E[pp][1];
        }
    }
    __syncthreads();
    double xq[2], rv[32];
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) xq[qq] = xk[l + 64 * qq];
#pragma unroll
    for (int pp = 0; pp < 32; ++pp) rv[pp] = RT[k * CHOL_RT_LD + w + 4 * pp];
#pragma unroll
    for (int pp = 0; pp < 32; ++pp)
#pragma unroll
      for (int qq = 0; qq < 2; ++qq) E[pp][qq] -= rv[pp] * xq[qq];
  }
  __syncthreads();
  for (int i = t; i < n * n; i += CHOL_THREADS) {
    const int r = i / n, c = i % n;
    Rg[i] = (r <= c && !dead[r]) ? (r == c ? pivs[r] : RT[c * CHOL_RT_LD + r]) : 0.0;
  }
#pragma unroll
  for (int pp = 0; pp < 32; ++pp)
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) {
      const int p = w + 4 * pp, q = l + 64 * qq;
      if (p < n && q < n) Rinv[p * n + q] = (p <= q && !dead[q]) ? E[pp][qq] : 0.0;
    }
}

void launch_chol_inv(const double *C, int n, double shift, double *R, double *Rinv, int *err, hipStream_t st) {
  TRG_REQUIRE(n >= 1 && n <= 1024, "chol: bad order");
  if (n <= CHOL_REG_MAX) {
    const size_t lds = size_t(CHOL_REG_MAX) * CHOL_RT_LD * 8;   // R^T for the inverse
    static bool attr = false;
    if (!attr) {
      TRG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(&chol_inv_reg_kernel),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
      attr = true;
    }
    hipLaunchKernelGGL(chol_inv_reg_kernel, dim3(1), dim3(CHOL_THREADS), lds, st, C, n, shift, R, Rinv, err);
  } else {
    hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(256), 0, st, C, n, shift, R, Rinv, err);
  }
  TRG_HIP_CHECK(hipGetLastError());
}

// Gram matrix C = Y^T Y of a tall m x k row-major matrix (k <= 128) on FP64
// MFMA, read in place: workgroup b sums the rows [b rpw, (b+1) rpw) into its
// own 128 x 128 slab part[b]; the slabs are then summed in a fixed order, so
// the result is deterministic.  Only the nb (nb + 1) / 2 blocks of 16 x 16
// on and above the diagonal are computed (nb = ceil(k / 16)), dealt round
// robin to the four waves; each block is written to the slab together with
// its transpose.  Rows are staged through LDS 32 at a time, double-buffered:
// the next chunk is loaded into registers while the current one is
// multiplied, and stored to the other buffer after it (one barrier per
// chunk; a buffer is refilled only after every wave passed the barrier that
// ended its last use).  Row stride 144 doubles: the four rows a k-step reads
// fall on the two halves of the banks.  v_mfma_f64_16x16x4: lane (g, r16)
// supplies A[r16][g] = Y[row g][col r16] and B[g][r16] likewise; accumulator
// e of the lane is C[g + 4e][r16].
constexpr int TSG_K = 128, TSG_ROWS = 32, TSG_LD = 144;
constexpr int TSG_MAXB = 9;   // blocks per wave: ceil(36 / 4)

typedef double tsg_v4d __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256)
ts_gram_kernel(const double *__restrict__ Y, int64_t m, int k, int64_t rpw, double *__restrict__ part) {
  __shared__ double L[2][TSG_ROWS * TSG_LD];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  const int nb = (k + 15) / 16;
  int bi[TSG_MAXB], bj[TSG_MAXB], nmine = 0;
#pragma unroll
  for (int q = 0; q < TSG_MAXB; ++q) bi[q] = bj[q] = 0;
  for (int i = 0, e = 0; i < nb; ++i)
    for (int j = i; j < nb; ++j, ++e)
      if ((e & 3) == wave && nmine < TSG_MAXB) {
        bi[nmine] = i;
        bj[nmine] = j;
        ++nmine;
      }
  const int64_t r0 = int64_t(blockIdx.x) * rpw;
  const int64_t r1 = r0 + rpw < m ? r0 + rpw : m;
  const int nch = r1 > r0 ? int((r1 - r0 + TSG_ROWS - 1) / TSG_ROWS) : 0;
  constexpr int PER = TSG_ROWS * TSG_K / 256;   // values per thread per chunk
  double pre[PER];
  auto gload = [&](int ch) {
    const int64_t base = r0 + int64_t(ch) * TSG_ROWS;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = t + 256 * u, r = idx / TSG_K, col = idx % TSG_K;
      pre[u] = (base + r < r1 && col < k) ? Y[(base + r) * k + col] : 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = t + 256 * u, r = idx / TSG_K, col = idx % TSG_K;
      L[buf][r * TSG_LD + col] = pre[u];
    }
  };
  tsg_v4d acc[TSG_MAXB];
#pragma unroll
  for (int q = 0; q < TSG_MAXB; ++q) acc[q] = tsg_v4d{0.0, 0.0, 0.0, 0.0};
  if (nch > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    if (ch + 1 < nch) gload(ch + 1);
    const double *Lb = L[ch & 1];
#pragma unroll
    for (int s = 0; s < TSG_ROWS / 4; ++s) {
      const double *row = Lb + (4 * s + g) * TSG_LD + r16;
#pragma unroll
      for (int q = 0; q < TSG_MAXB; ++q)
        if (q < nmine) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[16 * bi[q]], row[16 * bj[q]], acc[q], 0, 0, 0);
    }
    if (ch + 1 < nch) sstore((ch + 1) & 1);
    __syncthreads();
  }
  double *out = part + size_t(blockIdx.x) * TSG_K * TSG_K;
#pragma unroll
  for (int q = 0; q < TSG_MAXB; ++q)
    if (q < nmine)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = 16 * bi[q] + g + 4 * e, col = 16 * bj[q] + r16;
        out[row * TSG_K + col] = acc[q][e];
        out[col * TSG_K + row] = acc[q][e];
      }
}

// Q = Y R for a tall m x k row-major Y and an upper triangular k x k R
// (k <= 128; the inverse Cholesky factor) on FP64 MFMA.  R is staged once
// per workgroup in LDS (row stride 144 doubles: the four k-rows that one
// MFMA's B fragment reads fall on the two halves of the banks); the
// workgroup then walks row tiles of 256 rows, each of its eight waves 32
// rows x all columns, with Y read straight from memory into the A fragments
// (lane (g, r16) takes columns 16u + 4g .. 16u + 4g + 3 of its two rows for
// K chunk u, the next chunk prefetched while the current one is multiplied)
// and Q written from the accumulators.  K index 16u + 4g + e feeds MFMA e of
// chunk u on both sides, so the order of K inside a chunk is permuted alike
// for A and B.  Blocks of R below the diagonal are zero and skipped: chunk u
// only meets column blocks j >= u.
constexpr int TSM_WAVES = 8, TSM_ROWS = 32 * TSM_WAVES, TSM_LD = 144;

__global__ void __launch_bounds__(64 * TSM_WAVES)
ts_mul_kernel(const double *__restrict__ Y, int64_t m, int k, const double *__restrict__ R, double *__restrict__ Q) {
  extern __shared__ double Rl[];   // TSG_K x TSM_LD
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  for (int idx = t; idx < TSG_K * TSG_K; idx += 64 * TSM_WAVES) {
    const int r = idx / TSG_K, c = idx % TSG_K;
    Rl[r * TSM_LD + c] = (r < k && c < k) ? R[r * k + c] : 0.0;
  }
  __syncthreads();
  const int nu = (k + 15) / 16;   // K chunks = column blocks
  const int64_t ntiles = (m + TSM_ROWS - 1) / TSM_ROWS;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t rbase = tile * TSM_ROWS + 32 * wave;
    int64_t rows[2];
    bool rok[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      rows[h] = rbase + 16 * h + r16;
      rok[h] = rows[h] < m;
    }
    auto load = [&](int u, double (&a)[2][4]) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int col = 16 * u + 4 * g + e;
          a[h][e] = (rok[h] && col < k) ? Y[rows[h] * k + col] : 0.0;
        }
    };
    tsg_v4d acc[2][8];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[h][j] = tsg_v4d{0.0, 0.0, 0.0, 0.0};
    double a[2][4], an[2][4];
    load(0, a);
    for (int u = 0; u < nu; ++u) {
      if (u + 1 < nu) load(u + 1, an);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double *brow = Rl + (16 * u + 4 * g + e) * TSM_LD + r16;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j >= u && j < nu) {
            const double b = brow[16 * j];
#pragma unroll
            for (int h = 0; h < 2; ++h) acc[h][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h][e], b, acc[h][j], 0, 0, 0);
          }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 4; ++e) a[h][e] = an[h][e];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = rbase + 16 * h + g + 4 * e;
          const int col = 16 * j + r16;
          if (row < m && col < k) Q[row * k + col] = acc[h][j][e];
        }
  }
}

void launch_ts_mul(const double *Y, int64_t m, int k, const double *R, double *Q, hipStream_t st) {
  TRG_REQUIRE(k >= 1 && k <= TSG_K, "ts_mul: k out of range");
  const size_t lds = size_t(TSG_K) * TSM_LD * 8;
  static bool attr = false;
  if (!attr) {
    TRG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(&ts_mul_kernel),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    attr = true;
  }
  // one workgroup per CU (the LDS copy of R), each walking its row tiles
  const int64_t ntiles = (m + TSM_ROWS - 1) / TSM_ROWS;
  const uint32_t grid = uint32_t(ntiles < 256 ? ntiles : 256);
  hipLaunchKernelGGL(ts_mul_kernel, dim3(grid), dim3(64 * TSM_WAVES), lds, st, Y, m, k, R, Q);
  TRG_HIP_CHECK(hipGetLastError());
}

// One isometry applied to a leg pair on FP64 MFMA:
//   out[kept..., B] = sum_{a, b} src[..., a, ..., b, ...] P[a, b, B]
// with P row-major [a][b][B] (dn x dn x nd).  Rows m of the product are the
// kept legs (mixed radix over size[], outermost first; src strides sstr,
// out strides ostr), K = (a, b) and N = B.  Each wave takes 32 rows and
// every column block of B, so each source element is read once; lane
// (g, r16) loads rows 16 h + r16 (consecutive source addresses when the
// innermost kept leg has source stride 1) at K index 4 s + g, and the P
// fragment comes through the cache (P is small).
struct PairSpec {
  int nk;
  int64_t size[7], sstr[7], ostr[7];
  int64_t M;
  int dn, nd;
  int64_t sa, sb, ostrB;
};
constexpr int PC_WAVES = 4;

__global__ void __launch_bounds__(64 * PC_WAVES)
pair_contract_kernel(const double *__restrict__ src, const double *__restrict__ P, double *__restrict__ out,
                     PairSpec ps) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  const int64_t m0 = (int64_t(blockIdx.x) * PC_WAVES + wave) * 32;
  if (m0 >= ps.M) return;
  const int K = ps.dn * ps.dn;
  const int nj = (ps.nd + 15) / 16;
  // source offsets of this lane's two A rows
  int64_t soff[2];
  bool rok[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int64_t m = m0 + 16 * h + r16;
    rok[h] = m < ps.M;
    int64_t off = 0;
    for (int f = ps.nk - 1; f >= 0; --f) {
      const int64_t q = m / ps.size[f];
      off += (m - q * ps.size[f]) * ps.sstr[f];
      m = q;
    }
    soff[h] = rok[h] ? off : 0;
  }
  tsg_v4d acc[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[h][j] = tsg_v4d{0.0, 0.0, 0.0, 0.0};
  int a = g / ps.dn, b = g - (g / ps.dn) * ps.dn;   // (a, b) of K index k = 4 s + g
  for (int k = g; k - g < K; k += 4) {
    const bool kok = k < K;
    const int64_t koff = int64_t(a) * ps.sa + int64_t(b) * ps.sb;
    double av[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) av[h] = (rok[h] && kok) ? src[soff[h] + koff] : 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < nj) {
        const int n = 16 * j + r16;
        const double bv = (kok && n < ps.nd) ? P[int64_t(k) * ps.nd + n] : 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[h][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h], bv, acc[h][j], 0, 0, 0);
      }
    b += 4;
    while (b >= ps.dn) {
      b -= ps.dn;
      ++a;
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int64_t m = m0 + 16 * h + g + 4 * e;
      if (m >= ps.M) continue;
      int64_t off = 0;
      for (int f = ps.nk - 1; f >= 0; --f) {
        const int64_t q = m / ps.size[f];
        off += (m - q * ps.size[f]) * ps.ostr[f];
        m = q;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 16 * j + r16;
        if (j < nj && n < ps.nd) out[off + int64_t(n) * ps.ostrB] = acc[h][j][e];
      }
    }
}

// C = A B for n x n matrices (one workgroup)
__global__ void small_matmul_kernel(const double *A, const double *B, double *C, int n) {
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
    const int r = i / n, c = i % n;
    double v = 0.0;
    for (int k = 0; k < n; ++k) v += A[r * n + k] * B[k * n + c];
    C[i] = v;
  }
}

// J = [[0, C], [C^T, 0]] (2n x 2n) for C (n x n)
__global__ void jw_build_kernel(const double *C, int n, double *J) {
  const int m = 2 * n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m * m; i += gridDim.x * blockDim.x) {
    const int r = i / m, c = i % m;
    double v = 0.0;
    if (r < n && c >= n) v = C[r * n + (c - n)];
    if (r >= n && c < n) v = C[c * n + (r - n)];
    J[i] = v;
  }
}

// From the sorted eigensystem of J: s[i] = max(w[i], 0), sqrt_s[i],
// W[:, i] = sqrt(2) V[0:n, i], Z[:, i] = sqrt(2) V[n:2n, i] for i < k
__global__ void jw_extract_kernel(const double *w, const double *V, int n, int k, double *s, double *sqs,
                                  double *W, double *Z) {
  const int m = 2 * n;
  const double r2 = 1.4142135623730951;
  for (int i = threadIdx.x; i < n * k; i += blockDim.x) {
    const int row = i / k, col = i % k;
    W[row * k + col] = r2 * V[row * m + col];
    Z[row * k + col] = r2 * V[(n + row) * m + col];
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const double v = w[i] > 0.0 ? w[i] : 0.0;
    s[i] = v;
    sqs[i] = sqrt(v);
  }
}

// Sign gauge of the canonical form: for column j of U (n x k), the first
// entry whose modulus is within a relative 1e-9 of the column maximum is made
// positive: out[j] = sign * sqs[j] (one block per column).
__global__ void __launch_bounds__(256)
sign_gauge_kernel(const double *U, int64_t n, int k, const double *sqs, double *out) {
  __shared__ double sh[256];
  __shared__ long long si[256];
  const int j = blockIdx.x, t = threadIdx.x;
  double mx = 0.0;
  for (int64_t i = t; i < n; i += 256) mx = fmax(mx, fabs(U[i * k + j]));
  sh[t] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  const double thr = (1.0 - 1e-9) * sh[0];
  __syncthreads();
  long long first = n;
  for (int64_t i = t; i < n; i += 256)
    if (fabs(U[i * k + j]) >= thr && i < first) first = i;
  si[t] = first;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) si[t] = si[t] < si[t + s] ? si[t] : si[t + s];
    __syncthreads();
  }
  if (t == 0) {
    const long long r = si[0] < n ? si[0] : 0;
    out[j] = (U[r * k + j] < 0.0 ? -1.0 : 1.0) * sqs[j];
  }
}

// c^2 = sum_ij GtG[i,j] HHt[i,j]; scal[0] = c, scal[1] = c^{-1/2}, scal[2] = ln c
__global__ void atrg_norm_kernel(const double *GtG, const double *HHt, int r, double *scal, double *acc,
                                 double weight, int *err) {
  __shared__ double sh[256];
  const int t = threadIdx.x;
  double v = 0.0;
  for (int i = t; i < r * r; i += 256) v += GtG[i] * HHt[i];
  sh[t] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  if (t == 0) {
    const double c = sqrt(sh[0]);
    const bool ok = c > 0.0 && isfinite(c);
    scal[0] = c;
    scal[1] = ok ? 1.0 / sqrt(c) : 0.0;
    scal[2] = ok ? log(c) : 0.0;
    if (ok) acc[0] += weight * log(c);
    else *err |= 1;
  }
}

// out = sum_{b, l} G[b * r + l] H[l * n + b] (deterministic: fixed block sums, then one block)
__global__ void __launch_bounds__(256) gh_trace_partial(const double *G, const double *H, int64_t n, int r,
                                                        double *partial) {
  __shared__ double sh[256];
  const int64_t total = n * r;
  const int64_t per = (total + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = int64_t(blockIdx.x) * per;
  const int64_t e = b0 + per < total ? b0 + per : total;
  double v = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < e; i += 256) {
    const int64_t b = i / r, l = i % r;
    v += G[i] * H[l * n + b];
  }
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) sum_partials(const double *partial, int nb, double *out) {
  __shared__ double sh[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) v += partial[i];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// --------------------------------------------------------------- Z2 sectors ---
// In the Z2 mode every leg index and bond index has a parity (0 even, 1
// odd) and the pieces vanish unless the legs' parities add up to the bond's.
// Every kernel of the step keeps such zeros exact (a product with an exact
// zero is zero, and the decompositions below only combine indices of one
// sector), so no projection is ever needed.

// Bond of the initial pieces rotated to definite parity: the column pair
// (l0, l1) of the n x 2 row-major G becomes ((l0 + l1), (l0 - l1)) / sqrt 2,
// likewise the two rows of the 2 x n H.  At h = 0 the spin-down entries are
// the spin-up ones times (-1)^(number of odd legs) exactly, so the rotated
// entries of the wrong parity are exact zeros.  Either pointer may be null.
__global__ void z2_rotate_kernel(double *G, double *H, int64_t n) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const double r = 0.70710678118654752440;
  if (G) {
    const double a = G[2 * i], b = G[2 * i + 1];
    G[2 * i] = (a + b) * r;
    G[2 * i + 1] = (a - b) * r;
  }
  if (H) {
    const double a = H[i], b = H[n + i];
    H[i] = (a + b) * r;
    H[n + i] = (a - b) * r;
  }
}

// Parity of a composite row index (row-major over nf legs, outermost
// first) from the legs' parity tables packed in `par` at off[f].
struct ParSpec {
  int nf;
  int size[5];
  int off[5];
};

__device__ inline int spec_parity(const int *par, const ParSpec &s, int64_t i) {
  int p = 0;
  for (int f = s.nf - 1; f >= 0; --f) {
    const int64_t sz = s.size[f];
    const int64_t q = i / sz;
    p ^= par[s.off[f] + int(i - q * sz)];
    i = q;
  }
  return p;
}

// Trial matrix Om[rows, cols] (rows (f_perp, kB)): an entry survives only
// when its row parity equals the sector of its column, c mod 2 for c < 2 h
// and `big` beyond.
__global__ void z2_mask_kernel(double *Om, int64_t rows, int cols, const int *par, ParSpec spec, int h, int big) {
  const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t row = e / cols;
  const int col = int(e - row * cols);
  const int sec = col < 2 * h ? (col & 1) : big;
  if (spec_parity(par, spec, row) != sec) Om[e] = 0.0;
}

// B[b][i][j] = A[b][perm_b[i]][perm_b[j]] for the batch of symmetric n x n
// matrices (grid.y = batch; perm holds n entries per matrix)
__global__ void gather_sym_kernel(const double *A, double *B, const int *perm, int n) {
  const int64_t nn = int64_t(n) * n;
  const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (e >= nn) return;
  const int i = int(e / n), j = int(e - int64_t(e / n) * n);
  const int *p = perm + size_t(blockIdx.y) * n;
  B[size_t(blockIdx.y) * nn + e] = A[size_t(blockIdx.y) * nn + size_t(p[i]) * n + p[j]];
}

// eigenvector rows back to the original order: V[b][perm_b[i]][c] = Vs[b][i][c]
__global__ void scatter_rows_kernel(const double *Vs, double *V, const int *perm, int n) {
  const int64_t nn = int64_t(n) * n;
  const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (e >= nn) return;
  const int i = int(e / n), col = int(e - int64_t(e / n) * n);
  const int *p = perm + size_t(blockIdx.y) * n;
  V[size_t(blockIdx.y) * nn + size_t(p[i]) * n + col] = Vs[size_t(blockIdx.y) * nn + e];
}

// ------------------------------------------------------------- host helpers ---
// Step trace for diagnosing an ATRG run: with TRG_DEBUG set in the
// environment, every named intermediate is copied back and summarised on
// stderr (size, non-finite count, max |x|, 2-norm, device error flags).  Off
// by default (one cached getenv, no synchronisation).
void dbg(trg_ctx &c, const char *name, const double *p, int64_t count) {
  static const bool on = std::getenv("TRG_DEBUG") != nullptr;
  if (!on) return;
  TRG_HIP_CHECK(hipStreamSynchronize(c.st));
  std::vector<double> h(static_cast<size_t>(count));
  TRG_HIP_CHECK(hipMemcpy(h.data(), p, size_t(count) * 8, hipMemcpyDeviceToHost));
  double mx = 0, s2 = 0;
  int64_t bad = 0;
  for (double v : h) {
    if (!std::isfinite(v)) ++bad;
    else {
      mx = std::max(mx, std::fabs(v));
      s2 += v * v;
    }
  }
  int e = 0;
  TRG_HIP_CHECK(hipMemcpy(&e, c.errp(), 4, hipMemcpyDeviceToHost));
  std::fprintf(stderr, "[trg debug] %-10s n=%lld nonfinite=%lld max=%.3e norm=%.6e err=%d first=%.6e\n", name,
               (long long)count, (long long)bad, mx, std::sqrt(s2), e, h.empty() ? 0.0 : h[0]);
}

std::vector<std::pair<std::string, int64_t>> legs_of(const View &v) {
  std::vector<std::pair<std::string, int64_t>> out;
  for (const auto &l : v) out.push_back({l.name, l.size});
  return out;
}

View pick(const View &v, const std::vector<std::string> &names) {
  View out;
  for (const auto &n : names) out.push_back(find_leg(v, n));
  return out;
}

// Orthonormalise the columns of the m x k row-major matrix Y (m >= k) by
// shifted CholeskyQR3 (Fukaya et al.): three passes of Y <- Y R^{-1} with
// R^T R = Y^T Y (+ a shift of 11 (mk + k(k+1)) u tr(Y^T Y) on the first pass
// so that the Cholesky factorisation exists for ill-conditioned Y).  Q must
// not alias Y; Rout (optional) receives R = R3 R2 R1 with Y = Q R.
void cholqr3(trg_ctx &c, const double *Y, int64_t m, int k, double *Q, double *Rout, const std::string &tag) {
  TRG_REQUIRE(m >= k && k >= 1 && k <= 1024, "cholqr: bad shape");
  TRG_REQUIRE(Q != Y, "cholqr: output aliases input");
  double *Cg = c.wsp<double>("qrC" + tag, size_t(k) * k * 8);
  double *R = c.wsp<double>("qrR" + tag, size_t(k) * k * 8);
  double *Ri = c.wsp<double>("qrRi" + tag, size_t(k) * k * 8);
  double *Racc = c.wsp<double>("qrRa" + tag, size_t(k) * k * 8);
  double *Rtmp = c.wsp<double>("qrRt" + tag, size_t(k) * k * 8);
  double *bufA = c.wsp<double>("qrA" + tag, size_t(m) * k * 8);
  double *bufB = c.wsp<double>("qrB" + tag, size_t(m) * k * 8);
  const View vy = contiguous({{"i", m}, {"c", k}});
  const View vk = contiguous({{"i", m}, {"k", k}});
  const double u = std::ldexp(1.0, -53);
  const double *src = Y;
  const bool tsg = k <= TSG_K;
  // about 512 workgroups (two per CU), each a whole number of 32-row chunks
  const int64_t tsg_rows = std::max<int64_t>(TSG_ROWS, ((m + 511) / 512 + TSG_ROWS - 1) / TSG_ROWS * TSG_ROWS);
  const int64_t tsg_wg = (m + tsg_rows - 1) / tsg_rows;
  double *part = tsg ? c.wsp<double>("qrP" + tag, size_t(tsg_wg) * TSG_K * TSG_K * 8) : nullptr;
  for (int pass = 0; pass < 3; ++pass) {
    if (tsg) {
      hipLaunchKernelGGL(ts_gram_kernel, dim3(uint32_t(tsg_wg)), dim3(256), 0, c.st, src, m, k, tsg_rows, part);
      TRG_HIP_CHECK(hipGetLastError());
      reduce_splits(part, int(tsg_wg), k, k, TSG_K, int64_t(TSG_K) * TSG_K, Cg, k, c.st);
    } else {
      einsum2(c, src, vy, src, rename(vy, {{"c", "c2"}}), Cg, {"c", "c2"}, TRG_FP64, "qr" + tag);
    }
    const double shift = pass == 0 ? 11.0 * (double(m) * k + double(k) * (k + 1)) * u : 0.0;
    launch_chol_inv(Cg, k, shift, R, Ri, c.errp(), c.st);
    double *dst = pass == 2 ? Q : (pass == 0 ? bufA : bufB);
    if (tsg) {
      launch_ts_mul(src, m, k, Ri, dst, c.st);
    } else {
      einsum2(c, src, vk, Ri, contiguous({{"k", k}, {"c", k}}), dst, {"i", "c"}, TRG_FP64, "qm" + tag);
    }
    if (Rout) {
      if (pass == 0) {
        TRG_HIP_CHECK(hipMemcpyAsync(Racc, R, size_t(k) * k * 8, hipMemcpyDeviceToDevice, c.st));
      } else {
        hipLaunchKernelGGL(small_matmul_kernel, dim3(1), dim3(256), 0, c.st, R, Racc, Rtmp, k);
        TRG_HIP_CHECK(hipGetLastError());
        TRG_HIP_CHECK(hipMemcpyAsync(Racc, Rtmp, size_t(k) * k * 8, hipMemcpyDeviceToDevice, c.st));
      }
    }
    src = dst;
  }
  if (Rout) TRG_HIP_CHECK(hipMemcpyAsync(Rout, Racc, size_t(k) * k * 8, hipMemcpyDeviceToDevice, c.st));
}

// ---- Z2 bookkeeping on the host
using Par = std::vector<int8_t>;

// numbers of even and odd composite indices of legs with these parities
std::array<int64_t, 2> parity_counts(const std::vector<const Par *> &legs) {
  int64_t e = 1, o = 0;
  for (const Par *p : legs) {
    int64_t pe = 0, po = 0;
    for (int8_t x : *p) (x ? po : pe) += 1;
    const int64_t ne = e * pe + o * po, no = e * po + o * pe;
    e = ne;
    o = no;
  }
  return {e, o};
}

// composite parity of the row-major index over two legs
Par pair_parity(const Par &a, const Par &b) {
  Par out;
  out.reserve(a.size() * b.size());
  for (int8_t x : a)
    for (int8_t y : b) out.push_back(int8_t(x ^ y));
  return out;
}

// the indices of parity 0 in order, then those of parity 1, appended to out
void append_sector_order(const Par &p, std::vector<int> &out) {
  for (int s = 0; s < 2; ++s)
    for (size_t i = 0; i < p.size(); ++i)
      if (p[i] == s) out.push_back(int(i));
}

// Parity of each column of the rows x cols row-major device matrix M whose
// rows have parities rowpar: the sector that holds the larger part of the
// column's squared norm (the other part is zero for a column inside one
// sector).  Synchronises.
Par column_parities(trg_ctx &c, const double *M, int64_t rows, int cols, const Par &rowpar) {
  TRG_REQUIRE(int64_t(rowpar.size()) == rows, "z2: row parity table has the wrong size");
  std::vector<double> h(size_t(rows) * cols);
  TRG_HIP_CHECK(hipMemcpyAsync(h.data(), M, h.size() * 8, hipMemcpyDeviceToHost, c.st));
  sync_check(c);
  Par out(size_t(cols), 0);
  for (int j = 0; j < cols; ++j) {
    double w[2] = {0.0, 0.0};
    for (int64_t i = 0; i < rows; ++i) w[rowpar[size_t(i)]] += h[size_t(i) * cols + j] * h[size_t(i) * cols + j];
    out[size_t(j)] = int8_t(w[1] > w[0]);
  }
  return out;
}

// host table -> device buffer `tag`, queued on the context's stream; the
// table is one of the context's staging vectors, so it outlives the copy
int *upload(trg_ctx &c, const std::vector<int> &v, const std::string &tag) {
  int *d = c.wsp<int>(tag, v.size() * 4);
  TRG_HIP_CHECK(hipMemcpyAsync(d, v.data(), v.size() * 4, hipMemcpyHostToDevice, c.st));
  return d;
}

// eigh_top_batched (every eigenvalue, the leading eigenvectors: k, extended
// over a cluster that the cut splits) of `batch` symmetric n x n matrices
// whose indices may fall into two parity sectors, with perm (device, n
// entries per matrix) the sector order of each: Jacobi keeps sectors apart
// by itself; above its range the matrices are diagonalised in sector order
// and the eigenvector rows put back.  perm == nullptr: no reordering.
void eigh_sectors(trg_ctx &c, double *A, double *w, double *V, int *sw, int n, int batch, const int *perm, int k,
                  double cluster_rel, const std::string &tag) {
  double *work = n > JACOBI_MAX_N ? c.wsp<double>("ztop" + tag, eigh_top_work_doubles(n, batch) * 8) : nullptr;
  if (!perm || n <= JACOBI_MAX_N) {
    eigh_top_batched(A, w, V, sw, n, batch, k, cluster_rel, work, c.st);
    return;
  }
  double *As = c.wsp<double>("zA" + tag, size_t(batch) * n * n * 8);
  double *Vs = c.wsp<double>("zV" + tag, size_t(batch) * n * n * 8);
  const dim3 grid(uint32_t((int64_t(n) * n + 255) / 256), uint32_t(batch));
  hipLaunchKernelGGL(gather_sym_kernel, grid, dim3(256), 0, c.st, A, As, perm, n);
  TRG_HIP_CHECK(hipGetLastError());
  eigh_top_batched(As, w, Vs, sw, n, batch, k, cluster_rel, work, c.st);
  hipLaunchKernelGGL(scatter_rows_kernel, grid, dim3(256), 0, c.st, Vs, V, perm, n);
  TRG_HIP_CHECK(hipGetLastError());
}

// SVD of the k x k matrix Cm = W diag(s) Z^T through the eigendecomposition
// of [[0, Cm], [Cm^T, 0]]; keeps the first kk columns.  par (optional): the
// parity of the k row indices and of the k column indices of a Cm that
// vanishes between different parities; stage: the context staging vector
// for the sector order of the eigenproblem.
void small_svd(trg_ctx &c, const double *Cm, int k, int kk, double *s, double *sqs, double *W, double *Z,
               const std::string &tag, const Par *par = nullptr, std::vector<int> *stage = nullptr) {
  const int m = 2 * k;
  double *J = c.wsp<double>("svdJ" + tag, size_t(m) * m * 8);
  double *w = c.wsp<double>("svdw" + tag, size_t(m) * 8);
  double *V = c.wsp<double>("svdV" + tag, size_t(m) * m * 8);
  int *sw = c.wsp<int>("svdsw" + tag, 16);
  hipLaunchKernelGGL(jw_build_kernel, dim3(64), dim3(256), 0, c.st, Cm, k, J);
  TRG_HIP_CHECK(hipGetLastError());
  const int *perm = nullptr;
  if (par && m > JACOBI_MAX_N) {
    TRG_REQUIRE(int(par->size()) == k && stage, "small_svd: bad sector table");
    Par jp(*par);
    jp.insert(jp.end(), par->begin(), par->end());
    stage->clear();
    append_sector_order(jp, *stage);
    perm = upload(c, *stage, "svdperm" + tag);
  }
  eigh_sectors(c, J, w, V, sw, m, 1, perm, kk, 0.0, "svd" + tag);
  hipLaunchKernelGGL(jw_extract_kernel, dim3(1), dim3(256), 0, c.st, w, V, k, kk, s, sqs, W, Z);
  TRG_HIP_CHECK(hipGetLastError());
}

}  // namespace

// ------------------------------------------------------------------ einsum2 ---
void einsum2(trg_ctx &c, const double *A, const View &va, const double *B, const View &vb, double *C,
             const std::vector<std::string> &out_names, int prec, const std::string &tag) {
  std::vector<std::string> con, fa, fb;
  for (const auto &l : va)
    if (has_leg(vb, l.name)) con.push_back(l.name);
  for (const auto &n : out_names) {
    if (has_leg(va, n) && !has_leg(vb, n)) fa.push_back(n);
    else if (has_leg(vb, n) && !has_leg(va, n)) fb.push_back(n);
    else throw Error(-1, "einsum2: output leg " + n + " must belong to exactly one operand");
  }
  TRG_REQUIRE(!con.empty(), "einsum2: no contracted leg");
  TRG_REQUIRE(fa.size() + fb.size() + con.size() * 2 == va.size() + vb.size(), "einsum2: stray leg");
  int64_t M = 1, N = 1, K = 1;
  std::vector<std::pair<std::string, int64_t>> ra, rb, kc;
  for (const auto &n : fa) {
    ra.push_back({n, find_leg(va, n).size});
    M *= ra.back().second;
  }
  for (const auto &n : fb) {
    rb.push_back({n, find_leg(vb, n).size});
    N *= rb.back().second;
  }
  for (const auto &n : con) {
    const int64_t s = find_leg(va, n).size;
    TRG_REQUIRE(s == find_leg(vb, n).size, "einsum2: contracted leg sizes differ");
    kc.push_back({n, s});
    K *= s;
  }
  // few output tiles and a long K (tall-skinny Gram products of the RSVD):
  // split K over many workgroups with the 64 x 64 FP64 kernel, then reduce
  const GemmTile t0 = gemm_tile(prec);
  const int64_t tiles128 = int64_t(round_up(M, t0.m) / t0.m) * int64_t(round_up(N, t0.n) / t0.n);
  const bool splitk = prec == TRG_FP64 && tiles128 < 128 && K >= 4096;
  int64_t splits = 1, kper = 0;
  GemmTile t = t0;
  if (splitk) {
    t = GemmTile{64, 64, 16};
    const int64_t tiles64 = int64_t(round_up(M, 64) / 64) * int64_t(round_up(N, 64) / 64);
    splits = (1024 + tiles64 - 1) / tiles64;
    const int64_t kt = (K + 15) / 16;
    if (splits > kt) splits = kt;
    kper = int64_t(round_up((K + splits - 1) / splits, 16));
  }
  const int64_t Mp = int64_t(round_up(M, t.m)), Np = int64_t(round_up(N, t.n));
  const int64_t Kp = splitk ? kper * splits : int64_t(round_up(K, t.k));
  const int esz = prec == TRG_FP64 ? 8 : 4;
  const int okind = prec == TRG_FP64 ? OUT_F64 : OUT_F32;
  void *Ap = c.wsp<char>("e2A" + tag, size_t(Mp) * Kp * esz);
  void *Bp = c.wsp<char>("e2B" + tag, size_t(Np) * Kp * esz);
  View pa = contiguous(ra, Kp), pb = contiguous(rb, Kp), pk = contiguous(kc);
  pa.insert(pa.end(), pk.begin(), pk.end());
  pb.insert(pb.end(), pk.begin(), pk.end());
  apply_map(A, IN_F64, va, nullptr, {}, {}, Ap, okind, 0, pa, c.st);
  zero_pad(Ap, M, Mp, K, Kp, esz, 1, 0, c.st);
  apply_map(B, IN_F64, vb, nullptr, {}, {}, Bp, okind, 0, pb, c.st);
  zero_pad(Bp, N, Np, K, Kp, esz, 1, 0, c.st);
  // the GEMM writes C directly when the output is [fa, fb] unpadded in FP64
  std::vector<std::string> natural = fa;
  natural.insert(natural.end(), fb.begin(), fb.end());
  const bool direct = !splitk && prec == TRG_FP64 && Mp == M && Np == N && natural == out_names;
  void *Cp = direct ? static_cast<void *>(C) : c.wsp<char>("e2C" + tag, size_t(Mp) * Np * esz);
  if (splitk) {
    double *part = c.wsp<double>("e2P" + tag, size_t(splits) * Mp * Np * 8);
    gemm_nt_splitk_f64(static_cast<const double *>(Ap), static_cast<const double *>(Bp), part, uint64_t(Mp),
                       uint64_t(Np), uint64_t(Kp), uint64_t(Kp), uint64_t(Kp), uint32_t(splits), uint64_t(kper), c.st);
    reduce_splits(part, int(splits), M, N, Np, Mp * Np, static_cast<double *>(Cp), Np, c.st);
  } else {
  // the ATRG contraction GEMMs ("k2") are the timed kernel of an ATRG step
  const bool timed = c.profiling && tag == "k2";
  hipEvent_t e0{}, e1{};
  if (timed) {
    TRG_HIP_CHECK(hipEventCreate(&e0));
    TRG_HIP_CHECK(hipEventCreate(&e1));
    TRG_HIP_CHECK(hipEventRecord(e0, c.st));
  }
  gemm_nt(prec, Ap, Bp, Cp, uint64_t(Mp), uint64_t(Np), uint64_t(Kp), uint64_t(Kp), uint64_t(Kp), uint64_t(Np),
          false, c.st);
  if (timed) {
    TRG_HIP_CHECK(hipEventRecord(e1, c.st));
    c.join_events.push_back({e0, e1});
    c.join_launches += 1;
    c.join_flops_pending += 2.0 * double(M) * double(N) * double(K);
  }
  }
  if (direct) return;
  View cv = contiguous(ra, Np), cb = contiguous(rb);
  cv.insert(cv.end(), cb.begin(), cb.end());
  std::vector<std::pair<std::string, int64_t>> ol;
  for (const auto &n : out_names) ol.push_back({n, has_leg(va, n) ? find_leg(va, n).size : find_leg(vb, n).size});
  apply_map(Cp, prec == TRG_FP64 ? IN_F64 : IN_F32, cv, nullptr, {}, {}, C, OUT_F64, 0, contiguous(ol), c.st);
}

// out (view outv) = src (view inv) with the leg pair (la, lb) contracted
// against P[la, lb, lB] (row-major, FP64): outv holds every other leg of inv
// and lB.  Rows are ordered as the kept legs appear in outv.
void pair_contract(trg_ctx &c, const double *src, const View &inv, const std::string &la, const std::string &lb,
                   const double *P, const std::string &lB, double *out, const View &outv) {
  PairSpec ps{};
  const Leg &A = find_leg(inv, la), &B = find_leg(inv, lb), &O = find_leg(outv, lB);
  TRG_REQUIRE(A.size == B.size && A.size <= 1024, "pair_contract: pair legs differ");
  TRG_REQUIRE(O.size >= 1 && O.size <= 64, "pair_contract: isometry width out of range");
  ps.dn = int(A.size);
  ps.nd = int(O.size);
  ps.sa = A.stride;
  ps.sb = B.stride;
  ps.ostrB = O.stride;
  ps.M = 1;
  for (const auto &l : outv) {
    if (l.name == lB) continue;
    TRG_REQUIRE(ps.nk < 7, "pair_contract: too many legs");
    const Leg &sl = find_leg(inv, l.name);
    TRG_REQUIRE(sl.size == l.size, "pair_contract: leg sizes differ");
    ps.size[ps.nk] = l.size;
    ps.sstr[ps.nk] = sl.stride;
    ps.ostr[ps.nk] = l.stride;
    ++ps.nk;
    ps.M *= l.size;
  }
  TRG_REQUIRE(int64_t(ps.nk) + 2 == int64_t(inv.size()) && ps.nk >= 1, "pair_contract: stray legs");
  const int64_t blocks = (ps.M + 32 * PC_WAVES - 1) / (32 * PC_WAVES);
  TRG_REQUIRE(blocks < (int64_t(1) << 31), "pair_contract: too many rows");
  hipLaunchKernelGGL(pair_contract_kernel, dim3(uint32_t(blocks)), dim3(64 * PC_WAVES), 0, c.st, src, P, out, ps);
  TRG_HIP_CHECK(hipGetLastError());
}

// --------------------------------------------------------------- init / step ---
void atrg_init_ising(trg_ctx &c, double beta, double h) {
  const int d = c.d;
  const int64_t n = int64_t(1) << d;
  c.r = 2;
  c.ensure(c.G, size_t(n) * 2 * 8);
  c.ensure(c.H, size_t(n) * 2 * 8);
  double *G = static_cast<double *>(c.G.ptr), *H = static_cast<double *>(c.H.ptr);
  hipLaunchKernelGGL(atrg_ising_kernel, dim3(1), dim3(64), 0, c.st, G, H, d, beta, h);
  TRG_HIP_CHECK(hipGetLastError());
  if (c.z2) {
    // bond of definite parity; every leg index b of the W basis has parity b
    TRG_REQUIRE(h == 0.0, "the Z2 mode needs h = 0");
    hipLaunchKernelGGL(z2_rotate_kernel, dim3(1), dim3(64), 0, c.st, G, H, n);
    TRG_HIP_CHECK(hipGetLastError());
    for (int a = 0; a < d; ++a) c.z2_legs[a] = {0, 1};
    c.z2_bond = {0, 1};
  }
  // c_0 = ||G H||_F, both pieces scaled by c_0^{-1/2}
  double *GtG = c.wsp<double>("nGtG", 4 * 8), *HHt = c.wsp<double>("nHHt", 4 * 8);
  View vg = contiguous({{"b", n}, {"l", 2}}), vh = contiguous({{"l", 2}, {"f", n}});
  einsum2(c, G, vg, G, rename(vg, {{"l", "l2"}}), GtG, {"l", "l2"}, TRG_FP64, "nrm");
  einsum2(c, H, vh, H, rename(vh, {{"l", "l2"}}), HHt, {"l", "l2"}, TRG_FP64, "nrm");
  hipLaunchKernelGGL(atrg_norm_kernel, dim3(1), dim3(256), 0, c.st, GtG, HHt, 2, c.scal(), c.scal() + 3, 1.0,
                     c.errp());
  TRG_HIP_CHECK(hipGetLastError());
  dbg(c, "init G", G, n * 2);
  dbg(c, "init GtG", GtG, 4);
  dbg(c, "init HHt", HHt, 4);
  scale_by_inverse(G, n * 2, c.scal(), 1.0, c.st);
  scale_by_inverse(H, n * 2, c.scal(), 1.0, c.st);
  dbg(c, "init scal", c.scal(), 4);
  // impurities: G_S = the scaled pure backward piece, H_S from the closed form
  for (int j = 0; j < c.nimp; ++j) {
    c.ensure(c.S[j], size_t(n) * 2 * 8);
    c.ensure(c.Sn[j], size_t(n) * 2 * 8);
    TRG_HIP_CHECK(hipMemcpyAsync(c.S[j].ptr, G, size_t(n) * 2 * 8, hipMemcpyDeviceToDevice, c.st));
    double *HS = static_cast<double *>(c.Sn[j].ptr);
    hipLaunchKernelGGL(atrg_impurity_kernel, dim3(1), dim3(64), 0, c.st, c.imp_kind[j] == 0 ? HS : nullptr,
                       c.imp_kind[j] == 1 ? HS : nullptr, d, beta, h);
    TRG_HIP_CHECK(hipGetLastError());
    if (c.z2) {   // the impurity's bond rotated like the pure one
      hipLaunchKernelGGL(z2_rotate_kernel, dim3(1), dim3(64), 0, c.st, nullptr, HS, n);
      TRG_HIP_CHECK(hipGetLastError());
    }
    scale_by_inverse(HS, n * 2, c.scal(), 1.0, c.st);
    c.imp_r[j] = 2;
  }
  TRG_HIP_CHECK(hipMemcpyAsync(rec_d(c, 0), c.scal() + 2, 8, hipMemcpyDeviceToDevice, c.st));
}

double atrg_trace(trg_ctx &c) {
  int64_t n = 1;
  for (int a = 0; a < c.d; ++a) n *= c.dims[a];
  const int nb = 256;
  double *partial = c.wsp<double>("trpart", nb * 8);
  hipLaunchKernelGGL(gh_trace_partial, dim3(nb), dim3(256), 0, c.st, static_cast<const double *>(c.G.ptr),
                     static_cast<const double *>(c.H.ptr), n, c.r, partial);
  TRG_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, c.st, partial, nb, c.scal() + 4);
  TRG_HIP_CHECK(hipGetLastError());
  sync_check(c);
  double v = 0.0;
  TRG_HIP_CHECK(hipMemcpy(&v, c.scal() + 4, 8, hipMemcpyDeviceToHost));
  return v;
}

double atrg_impurity_trace(trg_ctx &c, int j) {
  int64_t n = 1;
  for (int a = 0; a < c.d; ++a) n *= c.dims[a];
  const int nb = 256;
  double *partial = c.wsp<double>("trpart", nb * 8);
  hipLaunchKernelGGL(gh_trace_partial, dim3(nb), dim3(256), 0, c.st, static_cast<const double *>(c.S[j].ptr),
                     static_cast<const double *>(c.Sn[j].ptr), n, c.imp_r[j], partial);
  TRG_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, c.st, partial, nb, c.scal() + 5);
  TRG_HIP_CHECK(hipGetLastError());
  sync_check(c);
  double v = 0.0;
  TRG_HIP_CHECK(hipMemcpy(&v, c.scal() + 5, 8, hipMemcpyDeviceToHost));
  return v;
}

// Indicator matrix of the factored tensor: the legs of `axis` open, every
// other axis' backward leg (in G) joined to its forward leg (in H), the bond
// l summed: one GEMM with K = r prod_{nu != axis} d_nu
void atrg_indicator_traces(trg_ctx &c, int axis, double *M, double *out) {
  const int d = c.d;
  std::vector<std::pair<std::string, int64_t>> lg, lh{{"l", c.r}};
  for (int a = 0; a < d; ++a) {
    lg.push_back({a == axis ? std::string("x") : nm("t", a), c.dims[a]});
    lh.push_back({a == axis ? std::string("xp") : nm("t", a), c.dims[a]});
  }
  lg.push_back({"l", c.r});
  einsum2(c, static_cast<const double *>(c.G.ptr), contiguous(lg), static_cast<const double *>(c.H.ptr),
          contiguous(lh), M, {"x", "xp"}, TRG_FP64, "ind");
  indicator_reduce(M, c.dims[axis], out, c.st);
}

void atrg_step_impl(trg_ctx &c, int mu, int dcut) {
  const int d = c.d;
  const int r = c.r;
  const hipStream_t st = c.st;
  int dims[4] = {0, 0, 0, 0};
  int64_t n = 1;
  for (int a = 0; a < d; ++a) {
    dims[a] = c.dims[a];
    n *= dims[a];
  }
  std::vector<int> perp;
  for (int a = 0; a < d; ++a)
    if (a != mu) perp.push_back(a);
  int64_t nperp = 1;
  for (int a : perp) nperp *= dims[a];
  // 0 selects the paper's values (p = 4 Dcut, q = 2 Dcut); negative means none
  const int p = c.cfg.rsvd_p > 0 ? c.cfg.rsvd_p : (c.cfg.rsvd_p == 0 ? 4 * dcut : 0);
  const int q = c.cfg.rsvd_q > 0 ? c.cfg.rsvd_q : (c.cfg.rsvd_q == 0 ? 2 * dcut : 0);
  const int cprec = c.cfg.precision == TRG_FP32 ? TRG_FP32 : TRG_FP64;
  const int n_step = c.nsteps + 1;
  ensure_records(c, n_step + 1);
  double *rd = rec_d(c, n_step);
  int *ri = rec_i(c, n_step);
  const double *Gp = static_cast<const double *>(c.G.ptr);
  const double *Hp = static_cast<const double *>(c.H.ptr);

  // names of the canonical legs
  std::vector<std::string> bn, fn;
  for (int a = 0; a < d; ++a) {
    bn.push_back(nm("b", a));
    fn.push_back(nm("f", a));
  }

  // ---- 1. canonical form T = U diag(s) V
  TRG_REQUIRE(n >= r, "atrg: piece has fewer rows than its rank");
  const int k = r < dcut ? r : dcut;
  double *Qg = c.wsp<double>("cQg", size_t(n) * r * 8);
  double *Qh = c.wsp<double>("cQh", size_t(n) * r * 8);
  double *HT = c.wsp<double>("cHT", size_t(n) * r * 8);
  double *Rg = c.wsp<double>("cRg", size_t(r) * r * 8);
  double *Rh = c.wsp<double>("cRh", size_t(r) * r * 8);
  double *Cm = c.wsp<double>("cCm", size_t(r) * r * 8);
  dbg(c, "G", Gp, n * r);
  dbg(c, "H", Hp, n * r);
  cholqr3(c, Gp, n, r, Qg, Rg, "g");
  dbg(c, "Qg", Qg, n * r);
  dbg(c, "Rg", Rg, int64_t(r) * r);
  apply_map(Hp, IN_F64, contiguous({{"l", r}, {"f", n}}), nullptr, {}, {}, HT, OUT_F64, 0,
            contiguous({{"f", n}, {"l", r}}), st);
  cholqr3(c, HT, n, r, Qh, Rh, "h");
  // core = Rg Rh^T
  einsum2(c, Rg, contiguous({{"i", r}, {"j", r}}), Rh, contiguous({{"m", r}, {"j", r}}), Cm, {"i", "m"},
          TRG_FP64, "core");
  double *s = c.wsp<double>("cs", size_t(k) * 8), *sqs = c.wsp<double>("csq", size_t(k) * 8);
  double *W = c.wsp<double>("cW", size_t(r) * k * 8), *Z = c.wsp<double>("cZ", size_t(r) * k * 8);
  dbg(c, "Cm", Cm, int64_t(r) * r);
  if (c.z2) TRG_REQUIRE(int(c.z2_bond.size()) == r, "z2: bond parity table does not match the bond");
  small_svd(c, Cm, r, k, s, sqs, W, Z, "core", c.z2 ? &c.z2_bond : nullptr, &c.z2_stage[0]);
  // Z2: parity of each kept bond index (its left singular vector lies in one sector)
  const Par kpar = c.z2 ? column_parities(c, W, r, k, c.z2_bond) : Par{};
  dbg(c, "s", s, k);
  dbg(c, "W", W, int64_t(r) * k);
  // Ut[b..., k] = Qg W sqrt(s); Vt[k, f...] = sqrt(s) (Qh Z)^T
  double *Ut = c.wsp<double>("Ut", size_t(n) * k * 8);
  double *Vt = c.wsp<double>("Vt", size_t(n) * k * 8);
  {
    double *tmp = c.wsp<double>("cUtmp", size_t(n) * k * 8);
    double *ssq = c.wsp<double>("cssq", size_t(k) * 8);  // sign * sqrt(s)
    einsum2(c, Qg, contiguous({{"i", n}, {"j", r}}), W, contiguous({{"j", r}, {"k", k}}), tmp, {"i", "k"},
            TRG_FP64, "cu");
    hipLaunchKernelGGL(sign_gauge_kernel, dim3(k), dim3(256), 0, st, tmp, n, k, sqs, ssq);
    TRG_HIP_CHECK(hipGetLastError());
    apply_map(tmp, IN_F64, contiguous({{"i", n}, {"k", k}}), ssq, {{"k", 1}}, {}, Ut, OUT_F64, 0,
              contiguous({{"i", n}, {"k", k}}), st);
    einsum2(c, Qh, contiguous({{"i", n}, {"j", r}}), Z, contiguous({{"j", r}, {"k", k}}), tmp, {"i", "k"},
            TRG_FP64, "cu");
    apply_map(tmp, IN_F64, contiguous({{"i", n}, {"k", k}}), ssq, {{"k", 1}}, {}, Vt, OUT_F64, 0,
              contiguous({{"k", k}, {"i", n}}), st);
  }
  // views: Ut[b0..b_{d-1}, kk], Vt[kk, f0..f_{d-1}]
  std::vector<std::pair<std::string, int64_t>> lb, lf;
  for (int a = 0; a < d; ++a) lb.push_back({bn[a], dims[a]});
  lb.push_back({"kk", k});
  lf.push_back({"kk", k});
  for (int a = 0; a < d; ++a) lf.push_back({fn[a], dims[a]});
  const View vUt = contiguous(lb), vVt = contiguous(lf);

  // ---- 2. swap by randomized SVD of M[(kA, b_perp), (f_perp, kB)]
  const View vVA = rename(vVt, {{"kk", "kA"}, {fn[mu], "j"}});
  const View vUB = rename(vUt, {{"kk", "kB"}, {bn[mu], "j"}});
  const int64_t nsw = int64_t(k) * nperp;
  std::vector<std::string> fperp, bperp;
  for (int a : perp) {
    fperp.push_back(fn[a]);
    bperp.push_back(bn[a]);
  }
  // Partial SVD of rank <= dcut of M[(kA, b_perp), (f_perp, kB)] =
  // sum_j A[kA, f_perp, j] B[j, b_perp, kB] (kA of size ra, kB of size cb):
  // randomized, with the trial matrix of `stream`; M Z and M^T Z are applied
  // in factored form (two GEMMs each).  Returns Xs[kA, b_perp, l] =
  // Q W sqrt(sigma), Ys[l, f_perp, kB] = sqrt(sigma) (Qbt Z)^T and sigma in
  // workspace buffers named with `tag`, and the rank.
  // With `sectors` (Z2 mode, pure swap) the trial columns are split into the
  // two parity sectors (column c in sector c mod 2 while both have room,
  // i.e. fewer columns than rows and columns of that parity, the rest in
  // the larger sector) and the trial matrix keeps only the entries whose
  // row parity equals the column's sector; every later product and
  // factorisation keeps the sectors apart, and par receives the parity of
  // each kept singular vector.
  struct SwapOut {
    double *Xs, *Ys, *sig;
    int dc;
    Par par;
  };
  auto partial_svd = [&](const double *A, const View &vA, int64_t ra, const double *B, const View &vB,
                         int64_t cb, uint32_t stream, const std::string &tag, bool sectors) -> SwapOut {
    const int64_t nr = ra * nperp, nc = nperp * cb;
    int r2 = dcut + p;
    if (r2 > nr) r2 = int(nr);
    if (r2 > nc) r2 = int(nc);
    int zh = 0, zbig = 0;
    Par sec;
    if (sectors) {
      TRG_REQUIRE(ra == k && cb == k && int64_t(kpar.size()) == k, "z2: sectors apply to the pure swap only");
      // rows (kA, b_perp) and columns (f_perp, kB) carry the same parities
      std::vector<const Par *> f{&kpar};
      for (int a : perp) f.push_back(&c.z2_legs[a]);
      const auto room = parity_counts(f);
      if (r2 > room[0] + room[1]) r2 = int(room[0] + room[1]);
      zh = int(std::min(room[0], room[1]));
      zbig = room[0] >= room[1] ? 0 : 1;
      sec.resize(size_t(r2));
      for (int col = 0; col < r2; ++col) sec[size_t(col)] = int8_t(col < 2 * zh ? (col & 1) : zbig);
    }
    auto zview = [&](int64_t cols) {  // rows (f_perp, kB)
      std::vector<std::pair<std::string, int64_t>> l;
      for (int a : perp) l.push_back({fn[a], dims[a]});
      l.push_back({"kB", cb});
      l.push_back({"c", cols});
      return contiguous(l);
    };
    auto qview = [&](int64_t cols) {  // rows (kA, b_perp)
      std::vector<std::pair<std::string, int64_t>> l;
      l.push_back({"kA", ra});
      for (int a : perp) l.push_back({bn[a], dims[a]});
      l.push_back({"c", cols});
      return contiguous(l);
    };
    double *tbuf = c.wsp<double>("swT" + tag, size_t(ra) * dims[mu] * cb * r2 * 8);
    auto apply_M = [&](const double *Zin, double *out) {
      // t[kA, j, kB, c] = sum_f A[kA, f_perp, j] Z[f_perp, kB, c];
      // out[kA, b_perp, c] = sum_{j, kB} t B[j, b_perp, kB]
      einsum2(c, A, vA, Zin, zview(r2), tbuf, {"kA", "j", "kB", "c"}, TRG_FP64, "sw1");
      const View vt = contiguous({{"kA", ra}, {"j", dims[mu]}, {"kB", cb}, {"c", r2}});
      std::vector<std::string> o{"kA"};
      o.insert(o.end(), bperp.begin(), bperp.end());
      o.push_back("c");
      einsum2(c, tbuf, vt, B, vB, out, o, TRG_FP64, "sw2");
    };
    auto apply_MT = [&](const double *Qin, double *out) {
      einsum2(c, B, vB, Qin, qview(r2), tbuf, {"j", "kB", "kA", "c"}, TRG_FP64, "sw3");
      const View vt = contiguous({{"j", dims[mu]}, {"kB", cb}, {"kA", ra}, {"c", r2}});
      std::vector<std::string> o = fperp;
      o.push_back("kB");
      o.push_back("c");
      einsum2(c, A, vA, tbuf, vt, out, o, TRG_FP64, "sw4");
    };
    const int64_t nmax = nr > nc ? nr : nc;
    double *Om = c.wsp<double>("swOm" + tag, size_t(nc) * r2 * 8);
    double *Yb = c.wsp<double>("swY" + tag, size_t(nmax) * r2 * 8);
    double *Qb = c.wsp<double>("swQ" + tag, size_t(nr) * r2 * 8);
    double *Zb = c.wsp<double>("swZ" + tag, size_t(nc) * r2 * 8);
    {
      const uint64_t cnt = uint64_t(nc) * r2;
      TRG_REQUIRE(cnt < (1ull << 32), "atrg: trial matrix too large");
      const uint64_t seed = c.cfg.seed;
      hipLaunchKernelGGL(trial_kernel, dim3(uint32_t((cnt + 255) / 256)), dim3(256), 0, st, Om, uint32_t(cnt),
                         uint32_t(n_step), stream, uint32_t(seed & 0xffffffffu), uint32_t(seed >> 32));
      TRG_HIP_CHECK(hipGetLastError());
      if (sectors) {
        // parity tables of the row legs (f_perp..., kB), packed
        std::vector<int> &tab = c.z2_stage[1];
        tab.clear();
        ParSpec ps{};
        auto add = [&](const Par &pv) {
          ps.size[ps.nf] = int(pv.size());
          ps.off[ps.nf] = int(tab.size());
          for (int8_t x : pv) tab.push_back(x);
          ++ps.nf;
        };
        for (int a : perp) add(c.z2_legs[a]);
        add(kpar);
        const int *pd = upload(c, tab, "zmask");
        hipLaunchKernelGGL(z2_mask_kernel, dim3(uint32_t((cnt + 255) / 256)), dim3(256), 0, st, Om, nc, r2, pd, ps,
                           zh, zbig);
        TRG_HIP_CHECK(hipGetLastError());
      }
    }
    dbg(c, "Om", Om, nc * r2);
    apply_M(Om, Yb);
    dbg(c, "MOm", Yb, nr * r2);
    cholqr3(c, Yb, nr, r2, Qb, nullptr, "sw");
    dbg(c, "Q0", Qb, nr * r2);
    for (int it = 0; it < q; ++it) {
      apply_MT(Qb, Yb);
      cholqr3(c, Yb, nc, r2, Zb, nullptr, "sw");
      apply_M(Zb, Yb);
      cholqr3(c, Yb, nr, r2, Qb, nullptr, "sw");
    }
    // Bt = M^T Q = Qbt Rb; Q^T M = Rb^T Qbt^T; SVD of Rb^T
    double *Rb = c.wsp<double>("swRb", size_t(r2) * r2 * 8);
    double *RbT = c.wsp<double>("swRbT", size_t(r2) * r2 * 8);
    apply_MT(Qb, Yb);
    cholqr3(c, Yb, nc, r2, Zb, Rb, "sw");
    apply_map(Rb, IN_F64, contiguous({{"i", r2}, {"j", r2}}), nullptr, {}, {}, RbT, OUT_F64, 0,
              contiguous({{"j", r2}, {"i", r2}}), st);
    const int dcx = r2 < dcut ? r2 : dcut;
    double *sg = c.wsp<double>("swsig" + tag, size_t(dcx) * 8), *sqsig = c.wsp<double>("swsq", size_t(dcx) * 8);
    double *Wb = c.wsp<double>("swW", size_t(r2) * dcx * 8), *Zs = c.wsp<double>("swZs", size_t(r2) * dcx * 8);
    dbg(c, "Rb", Rb, int64_t(r2) * r2);
    small_svd(c, RbT, r2, dcx, sg, sqsig, Wb, Zs, "sw", sectors ? &sec : nullptr, &c.z2_stage[2]);
    dbg(c, "sigma", sg, dcx);
    SwapOut o{c.wsp<double>("Xs" + tag, size_t(nr) * dcx * 8), c.wsp<double>("Ys" + tag, size_t(nc) * dcx * 8), sg,
              dcx, sectors ? column_parities(c, Wb, r2, dcx, sec) : Par{}};
    double *tmp = c.wsp<double>("swtmp", size_t(nmax) * dcx * 8);
    einsum2(c, Qb, contiguous({{"i", nr}, {"j", r2}}), Wb, contiguous({{"j", r2}, {"l", dcx}}), tmp, {"i", "l"},
            TRG_FP64, "sx");
    apply_map(tmp, IN_F64, contiguous({{"i", nr}, {"l", dcx}}), sqsig, {{"l", 1}}, {}, o.Xs, OUT_F64, 0,
              contiguous({{"i", nr}, {"l", dcx}}), st);
    einsum2(c, Zb, contiguous({{"i", nc}, {"j", r2}}), Zs, contiguous({{"j", r2}, {"l", dcx}}), tmp, {"i", "l"},
            TRG_FP64, "sx");
    apply_map(tmp, IN_F64, contiguous({{"i", nc}, {"l", dcx}}), sqsig, {{"l", 1}}, {}, o.Ys, OUT_F64, 0,
              contiguous({{"l", dcx}, {"i", nc}}), st);
    return o;
  };
  dbg(c, "Ut", Ut, n * k);
  dbg(c, "Vt", Vt, n * k);
  const SwapOut pure = partial_svd(Vt, vVA, k, Ut, vUB, k, 0u, "", c.z2);
  double *Xs = pure.Xs, *Ys = pure.Ys, *sig = pure.sig;
  const int dc = pure.dc;
  c.ensure(c.atrg_sigma, size_t(dc) * 8);
  TRG_HIP_CHECK(hipMemcpyAsync(c.atrg_sigma.ptr, sig, size_t(dc) * 8, hipMemcpyDeviceToDevice, st));
  c.atrg_nsig = dc;
  // views of the pieces' factors
  View vXs, vYs;
  {
    std::vector<std::pair<std::string, int64_t>> l{{"kA", k}};
    for (int a : perp) l.push_back({nm("bB", a), dims[a]});
    l.push_back({"l", dc});
    vXs = contiguous(l);
    std::vector<std::pair<std::string, int64_t>> m{{"l", dc}};
    for (int a : perp) m.push_back({nm("fA", a), dims[a]});
    m.push_back({"kB", k});
    vYs = contiguous(m);
  }
  View vUA = vUt, vVB = vVt;  // site A backward legs (Ut), site B forward legs (Vt)
  for (int a = 0; a < d; ++a) {
    vUA = rename(vUA, {{bn[a], nm("bA", a)}});
    vVB = rename(vVB, {{fn[a], nm("fB", a)}});
  }
  vUA = rename(vUA, {{"kk", "kA"}});
  vVB = rename(vVB, {{"kk", "kB"}});

  // ---- 3. HOSVD isometries from factored Gram matrices
  double *UtU = c.wsp<double>("gUtU", size_t(k) * k * 8), *VVt = c.wsp<double>("gVVt", size_t(k) * k * 8);
  {
    std::map<std::string, std::string> ren{{"kA", "kA2"}};
    einsum2(c, Ut, vUA, Ut, rename(vUA, ren), UtU, {"kA", "kA2"}, TRG_FP64, "g0");
    einsum2(c, Vt, vVB, Vt, rename(vVB, {{"kB", "kB2"}}), VVt, {"kB", "kB2"}, TRG_FP64, "g0");
  }
  double *Wf = c.wsp<double>("gWf", size_t(dc) * dc * 8), *Wbk = c.wsp<double>("gWb", size_t(dc) * dc * 8);
  {
    // Wf[l, l2] = sum Ys[l, fA_perp, kB] VVt[kB, kB2] Ys[l2, fA_perp, kB2]
    double *YV = c.wsp<double>("gYV", size_t(nsw) * dc * 8);
    std::vector<std::string> o{"l"};
    for (int a : perp) o.push_back(nm("fA", a));
    o.push_back("kB2");
    einsum2(c, Ys, vYs, VVt, contiguous({{"kB", k}, {"kB2", k}}), YV, o, TRG_FP64, "g1");
    std::vector<std::pair<std::string, int64_t>> yl{{"l", dc}};
    for (int a : perp) yl.push_back({nm("fA", a), dims[a]});
    yl.push_back({"kB2", k});
    einsum2(c, YV, contiguous(yl), Ys, rename(vYs, {{"l", "l2"}, {"kB", "kB2"}}), Wf, {"l", "l2"}, TRG_FP64,
            "g2");
    // Wb[l, l2] = sum Xs[kA, bB_perp, l] UtU[kA, kA2] Xs[kA2, bB_perp, l2]
    std::vector<std::string> o2{"kA2"};
    for (int a : perp) o2.push_back(nm("bB", a));
    o2.push_back("l");
    einsum2(c, UtU, contiguous({{"kA", k}, {"kA2", k}}), Xs, vXs, YV, o2, TRG_FP64, "g1");
    std::vector<std::pair<std::string, int64_t>> xl{{"kA2", k}};
    for (int a : perp) xl.push_back({nm("bB", a), dims[a]});
    xl.push_back({"l", dc});
    einsum2(c, YV, contiguous(xl), Xs, rename(vXs, {{"l", "l2"}, {"kA", "kA2"}}), Wbk, {"l", "l2"}, TRG_FP64,
            "g2");
  }
  int nd[4] = {0, 0, 0, 0};
  for (int a = 0; a < d; ++a) {
    const int64_t sq = int64_t(dims[a]) * dims[a];
    nd[a] = a == mu ? dims[a] : int(sq < dcut ? sq : dcut);
  }
  // Grams of every transverse axis first, so that axes of one order share
  // one eigensolver launch (one workgroup per matrix)
  int nnmax = 0;
  bool same_n = true;
  for (int nu : perp) {
    nnmax = std::max(nnmax, dims[nu] * dims[nu]);
    same_n = same_n && dims[nu] == dims[perp[0]];
  }
  const int npp = int(perp.size());
  double *Gall = c.wsp<double>("gG", size_t(2) * npp * nnmax * nnmax * 8);
  double *Wall = c.wsp<double>("gW", size_t(2) * npp * nnmax * 8);
  double *Vall = c.wsp<double>("gV", size_t(2) * npp * nnmax * nnmax * 8);
  int *swall = c.wsp<int>("gsw", size_t(2) * npp * 4);
  for (int idx = 0; idx < npp; ++idx) {
    const int nu = perp[idx];
    const int dn = dims[nu], nn = dn * dn;
    double *G2 = Gall + size_t(2) * idx * nn * nn;   // contiguous batch when every nn agrees
    if (!same_n) G2 = Gall + size_t(2) * idx * nnmax * nnmax;
    double *PA = c.wsp<double>("gPA", size_t(nn) * k * k * 8);
    double *Xw = c.wsp<double>("gXw", size_t(nsw) * dc * 8);
    double *QX = c.wsp<double>("gQX", size_t(nn) * k * k * 8);
    // backward pair: PA[a, kA, a2, kA2] = sum_{bA other} Ut Ut
    {
      View v1 = rename(vUA, {{nm("bA", nu), "a"}});
      View v2 = rename(vUA, {{nm("bA", nu), "a2"}, {"kA", "kA2"}});
      einsum2(c, Ut, v1, Ut, v2, PA, {"a", "kA", "a2", "kA2"}, TRG_FP64, "h1");
      // Xw[kA2, bb2, others, l] = sum_l2 Xs[kA2, bb2, others, l2] Wf[l, l2]
      View vx = rename(vXs, {{"kA", "kA2"}, {nm("bB", nu), "bb2"}, {"l", "l2"}});
      std::vector<std::string> o{"kA2", "bb2"};
      std::vector<std::pair<std::string, int64_t>> xl{{"kA2", k}, {"bb2", dn}};
      for (int a : perp)
        if (a != nu) {
          o.push_back(nm("bB", a));
          xl.push_back({nm("bB", a), dims[a]});
        }
      o.push_back("l");
      xl.push_back({"l", dc});
      einsum2(c, Xs, vx, Wf, contiguous({{"l", dc}, {"l2", dc}}), Xw, o, TRG_FP64, "h2");
      // QX[kA, bb, kA2, bb2] = sum_{others, l} Xs Xw
      einsum2(c, Xs, rename(vXs, {{nm("bB", nu), "bb"}}), Xw, contiguous(xl), QX, {"kA", "bb", "kA2", "bb2"},
              TRG_FP64, "h3");
      // Gram[a, bb, a2, bb2] = sum_{kA, kA2} PA QX
      einsum2(c, PA, contiguous({{"a", dn}, {"kA", k}, {"a2", dn}, {"kA2", k}}), QX,
              contiguous({{"kA", k}, {"bb", dn}, {"kA2", k}, {"bb2", dn}}), G2, {"a", "bb", "a2", "bb2"}, TRG_FP64,
              "h4");
    }
    // forward pair: QY[fa, kB, fa2, kB2] from Ys and Wb, PV[kB, fb, kB2, fb2] from Vt
    {
      View v1 = rename(vVB, {{nm("fB", nu), "fb"}});
      View v2 = rename(vVB, {{nm("fB", nu), "fb2"}, {"kB", "kB2"}});
      einsum2(c, Vt, v1, Vt, v2, PA, {"kB", "fb", "kB2", "fb2"}, TRG_FP64, "h1");
      View vy = rename(vYs, {{"l", "l2"}, {nm("fA", nu), "fa2"}, {"kB", "kB2"}});
      std::vector<std::string> o{"l", "fa2"};
      std::vector<std::pair<std::string, int64_t>> yl{{"l", dc}, {"fa2", dn}};
      for (int a : perp)
        if (a != nu) {
          o.push_back(nm("fA", a));
          yl.push_back({nm("fA", a), dims[a]});
        }
      o.push_back("kB2");
      yl.push_back({"kB2", k});
      einsum2(c, Wbk, contiguous({{"l", dc}, {"l2", dc}}), Ys, vy, Xw, o, TRG_FP64, "h2");
      einsum2(c, Ys, rename(vYs, {{nm("fA", nu), "fa"}}), Xw, contiguous(yl), QX, {"fa", "kB", "fa2", "kB2"},
              TRG_FP64, "h3");
      einsum2(c, QX, contiguous({{"fa", dn}, {"kB", k}, {"fa2", dn}, {"kB2", k}}), PA,
              contiguous({{"kB", k}, {"fb", dn}, {"kB2", k}, {"fb2", dn}}), G2 + size_t(nn) * nn,
              {"fa", "fb", "fa2", "fb2"}, TRG_FP64, "h4");
    }
  }
  // Z2: the sector order of each Gram's pair index (both sides of an axis
  // share it), for the orders beyond the Jacobi range
  const int *gperm = nullptr;
  std::vector<size_t> gperm_off(size_t(npp), 0);
  if (c.z2 && nnmax > JACOBI_MAX_N) {
    std::vector<int> &tab = c.z2_stage[3];
    tab.clear();
    for (int idx = 0; idx < npp; ++idx) {
      const Par pp = pair_parity(c.z2_legs[perp[idx]], c.z2_legs[perp[idx]]);
      gperm_off[size_t(idx)] = tab.size();
      for (int side = 0; side < 2; ++side) append_sector_order(pp, tab);
    }
    gperm = upload(c, tab, "zgperm");
  }
  if (same_n) {
    const int nn = dims[perp[0]] * dims[perp[0]];
    eigh_sectors(c, Gall, Wall, Vall, swall, nn, 2 * npp, gperm, nd[perp[0]], degeneracy_window(producer_precision(c)),
                 "gram");
  } else {
    for (int idx = 0; idx < npp; ++idx) {
      const int nn = dims[perp[idx]] * dims[perp[idx]];
      eigh_sectors(c, Gall + size_t(2) * idx * nnmax * nnmax, Wall + size_t(2) * idx * nnmax,
                   Vall + size_t(2) * idx * nnmax * nnmax, swall + 2 * idx, nn, 2,
                   gperm ? gperm + gperm_off[size_t(idx)] : nullptr, nd[perp[idx]],
                   degeneracy_window(producer_precision(c)), "gram" + std::to_string(idx));
    }
  }
  for (int idx = 0; idx < 2 * npp; ++idx) {
    const int nn = dims[perp[idx / 2]] * dims[perp[idx / 2]];
    const size_t stride = same_n ? size_t(nn) : size_t(nnmax);
    dbg(c, "gram w", Wall + idx * stride, nn);
    dbg(c, "gram V", Vall + idx * stride * stride, int64_t(nn) * nn);
  }
  for (int idx = 0; idx < npp; ++idx) {
    const int nu = perp[idx];
    const int dn = dims[nu], nn = dn * dn, kn = nd[nu];
    const size_t stride = same_n ? size_t(nn) : size_t(nnmax);
    const double *Wv = Wall + 2 * idx * stride;
    const double *Vv = Vall + 2 * idx * stride * stride;
    const int *sw = swall + 2 * idx;
    c.ensure(c.U[nu], size_t(nn) * kn * 8);
    c.ensure(c.spec[nu], size_t(nn) * 8);
    c.Un[nu] = nn;
    c.Uk[nu] = kn;
    SelectOut so{static_cast<double *>(c.U[nu].ptr), rd + 1 + 2 * nu, ri + 4 * nu,
                 static_cast<double *>(c.spec[nu].ptr)};
    select_isometry(Wv, Vv, sw, nn, kn, c.force_side, degeneracy_window(producer_precision(c)), so, st);
  }
  // Z2: parity of each new leg index (its isometry column lies in one sector)
  Par new_legs[4];
  if (c.z2)
    for (int nu : perp)
      new_legs[nu] = column_parities(c, static_cast<const double *>(c.U[nu].ptr), int64_t(dims[nu]) * dims[nu], nd[nu],
                                     pair_parity(c.z2_legs[nu], c.z2_legs[nu]));

  dbg(c, "Wf", Wf, int64_t(dc) * dc);
  dbg(c, "Wb", Wbk, int64_t(dc) * dc);
  for (int nu : perp) dbg(c, "P", static_cast<const double *>(c.U[nu].ptr), int64_t(dims[nu]) * dims[nu] * nd[nu]);
  // ---- 4. contraction with the isometries
  int64_t nnew = 1;
  for (int a = 0; a < d; ++a) nnew *= nd[a];
  double *Gn = c.wsp<double>("newG", size_t(nnew) * dc * 8);
  double *Hn = c.wsp<double>("newH", size_t(nnew) * dc * 8);
  const int nu1 = perp[0];
  auto P = [&](int nu) { return static_cast<const double *>(c.U[nu].ptr); };
  // backward piece: Ut[bA..., kA] (kA of size k) and Xs[kA, bB_perp..., l]
  // (l of size dc) through the isometries into Gn[canonical legs..., l]
  auto gblock = [&](const double *Ut, const View &vUA, int64_t k, const double *Xs, const View &vXs,
                    int64_t dc, double *Gn) {
    // G: UP = Ut[bA..., kA] P1[bA_nu1, bB_nu1, B_nu1]
    const View vP1 = contiguous({{nm("bA", nu1), dims[nu1]}, {nm("bB", nu1), dims[nu1]}, {nm("B", nu1), nd[nu1]}});
    std::vector<std::string> o;
    std::vector<std::pair<std::string, int64_t>> ol;
    for (int a = 0; a < d; ++a)
      if (a != nu1) {
        o.push_back(nm("bA", a));
        ol.push_back({nm("bA", a), dims[a]});
      }
    o.insert(o.end(), {"kA", nm("bB", nu1), nm("B", nu1)});
    ol.insert(ol.end(), {{"kA", k}, {nm("bB", nu1), dims[nu1]}, {nm("B", nu1), nd[nu1]}});
    double *UP = c.wsp<double>("kUP", size_t(view_count(contiguous(ol))) * 8);
    einsum2(c, Ut, vUA, P(nu1), vP1, UP, o, TRG_FP64, "k1");
    // G1 = sum_{kA, bB_nu1} UP Xs  -> [bA (not nu1)..., B_nu1, bB (perp not nu1)..., l]
    std::vector<std::string> o2;
    std::vector<std::pair<std::string, int64_t>> ol2;
    for (int a = 0; a < d; ++a)
      if (a != nu1) {
        o2.push_back(nm("bA", a));
        ol2.push_back({nm("bA", a), dims[a]});
      }
    o2.push_back(nm("B", nu1));
    ol2.push_back({nm("B", nu1), nd[nu1]});
    for (int a : perp)
      if (a != nu1) {
        o2.push_back(nm("bB", a));
        ol2.push_back({nm("bB", a), dims[a]});
      }
    o2.push_back("l");
    ol2.push_back({"l", dc});
    double *G1 = c.wsp<double>("kG1", size_t(view_count(contiguous(ol2))) * 8);
    einsum2(c, UP, contiguous(ol), Xs, vXs, G1, o2, cprec, "k2");
    // remaining pairs: (bA_nu, bB_nu) -> B_nu, the last one writes the canonical order
    View cur = contiguous(ol2);
    const double *src = G1;
    for (size_t j = 1; j < perp.size(); ++j) {
      const int nu = perp[j];
      std::vector<std::pair<std::string, int64_t>> tl;
      const bool last = j + 1 == perp.size();
      if (last) {
        for (int a = 0; a < d; ++a) tl.push_back(a == mu ? std::make_pair(nm("bA", a), int64_t(dims[a]))
                                                         : std::make_pair(nm("B", a), int64_t(nd[a])));
        tl.push_back({"l", dc});
      } else {
        for (const auto &l : cur)
          if (l.name != nm("bA", nu) && l.name != nm("bB", nu)) tl.push_back({l.name, l.size});
        tl.push_back({nm("B", nu), nd[nu]});
      }
      const View tv = contiguous(tl);
      double *dst = last ? Gn : c.wsp<double>("kG2" + std::to_string(j), size_t(view_count(tv)) * 8);
      pair_contract(c, src, cur, nm("bA", nu), nm("bB", nu), P(nu), nm("B", nu), dst, tv);
      src = dst;
      cur = tv;
    }
    if (perp.size() == 1) {
      std::vector<std::pair<std::string, int64_t>> tl;
      for (int a = 0; a < d; ++a) tl.push_back(a == mu ? std::make_pair(nm("bA", a), int64_t(dims[a]))
                                                       : std::make_pair(nm("B", a), int64_t(nd[a])));
      tl.push_back({"l", dc});
      apply_map(G1, IN_F64, cur, nullptr, {}, {}, Gn, OUT_F64, 0, contiguous(tl), st);
    }
    };
  // forward piece: Ys[l, fA_perp..., kB] and Vt[kB, fB...] (kB of size k)
  // through the isometries into Hn[l, canonical legs...]
  auto hblock = [&](const double *Ys, const View &vYs, int64_t k, const double *Vt, const View &vVB,
                    int64_t dc, double *Hn) {
    // H: VP = Vt[kB, fB...] P1[fA_nu1, fB_nu1, F_nu1]
    const View vP1 = contiguous({{nm("fA", nu1), dims[nu1]}, {nm("fB", nu1), dims[nu1]}, {nm("F", nu1), nd[nu1]}});
    std::vector<std::string> o{"kB"};
    std::vector<std::pair<std::string, int64_t>> ol{{"kB", k}};
    for (int a = 0; a < d; ++a)
      if (a != nu1) {
        o.push_back(nm("fB", a));
        ol.push_back({nm("fB", a), dims[a]});
      }
    o.insert(o.end(), {nm("fA", nu1), nm("F", nu1)});
    ol.insert(ol.end(), {{nm("fA", nu1), dims[nu1]}, {nm("F", nu1), nd[nu1]}});
    double *VP = c.wsp<double>("kUP", size_t(view_count(contiguous(ol))) * 8);
    einsum2(c, Vt, vVB, P(nu1), vP1, VP, o, TRG_FP64, "k1");
    // H1 = sum_{kB, fA_nu1} Ys VP -> [l, fA (perp not nu1)..., fB (not nu1)..., F_nu1]
    std::vector<std::string> o2{"l"};
    std::vector<std::pair<std::string, int64_t>> ol2{{"l", dc}};
    for (int a : perp)
      if (a != nu1) {
        o2.push_back(nm("fA", a));
        ol2.push_back({nm("fA", a), dims[a]});
      }
    for (int a = 0; a < d; ++a)
      if (a != nu1) {
        o2.push_back(nm("fB", a));
        ol2.push_back({nm("fB", a), dims[a]});
      }
    o2.push_back(nm("F", nu1));
    ol2.push_back({nm("F", nu1), nd[nu1]});
    double *H1 = c.wsp<double>("kG1", size_t(view_count(contiguous(ol2))) * 8);
    einsum2(c, Ys, vYs, VP, contiguous(ol), H1, o2, cprec, "k2");
    View cur = contiguous(ol2);
    const double *src = H1;
    for (size_t j = 1; j < perp.size(); ++j) {
      const int nu = perp[j];
      std::vector<std::pair<std::string, int64_t>> tl;
      const bool last = j + 1 == perp.size();
      if (last) {
        tl.push_back({"l", dc});
        for (int a = 0; a < d; ++a) tl.push_back(a == mu ? std::make_pair(nm("fB", a), int64_t(dims[a]))
                                                         : std::make_pair(nm("F", a), int64_t(nd[a])));
      } else {
        for (const auto &l : cur)
          if (l.name != nm("fA", nu) && l.name != nm("fB", nu)) tl.push_back({l.name, l.size});
        tl.push_back({nm("F", nu), nd[nu]});
      }
      const View tv = contiguous(tl);
      double *dst = last ? Hn : c.wsp<double>("kG2" + std::to_string(j), size_t(view_count(tv)) * 8);
      pair_contract(c, src, cur, nm("fA", nu), nm("fB", nu), P(nu), nm("F", nu), dst, tv);
      src = dst;
      cur = tv;
    }
    if (perp.size() == 1) {
      std::vector<std::pair<std::string, int64_t>> tl{{"l", dc}};
      for (int a = 0; a < d; ++a) tl.push_back(a == mu ? std::make_pair(nm("fB", a), int64_t(dims[a]))
                                                       : std::make_pair(nm("F", a), int64_t(nd[a])));
      apply_map(H1, IN_F64, cur, nullptr, {}, {}, Hn, OUT_F64, 0, contiguous(tl), st);
    }
    };
  gblock(Ut, vUA, k, Xs, vXs, dc, Gn);
  hblock(Ys, vYs, k, Vt, vVB, dc, Hn);

  dbg(c, "Gn", Gn, nnew * dc);
  dbg(c, "Hn", Hn, nnew * dc);
  // ---- 5. normalisation
  double *GtG = c.wsp<double>("nGtG", size_t(dc) * dc * 8), *HHt = c.wsp<double>("nHHt", size_t(dc) * dc * 8);
  {
    const View vg = contiguous({{"b", nnew}, {"l", dc}}), vh = contiguous({{"l", dc}, {"f", nnew}});
    einsum2(c, Gn, vg, Gn, rename(vg, {{"l", "l2"}}), GtG, {"l", "l2"}, TRG_FP64, "nrm");
    einsum2(c, Hn, vh, Hn, rename(vh, {{"l", "l2"}}), HHt, {"l", "l2"}, TRG_FP64, "nrm");
  }
  hipLaunchKernelGGL(atrg_norm_kernel, dim3(1), dim3(256), 0, st, GtG, HHt, dc, c.scal(), c.scal() + 3,
                     std::ldexp(1.0, -n_step), c.errp());
  TRG_HIP_CHECK(hipGetLastError());
  scale_by_inverse(Gn, nnew * dc, c.scal(), 1.0, st);
  scale_by_inverse(Hn, nnew * dc, c.scal(), 1.0, st);
  TRG_HIP_CHECK(hipMemcpyAsync(rd, c.scal() + 2, 8, hipMemcpyDeviceToDevice, st));
  c.ensure(c.G, size_t(nnew) * dc * 8);
  c.ensure(c.H, size_t(nnew) * dc * 8);
  TRG_HIP_CHECK(hipMemcpyAsync(c.G.ptr, Gn, size_t(nnew) * dc * 8, hipMemcpyDeviceToDevice, st));
  TRG_HIP_CHECK(hipMemcpyAsync(c.H.ptr, Hn, size_t(nnew) * dc * 8, hipMemcpyDeviceToDevice, st));

  // ---- impurities: [C(S, T) + C(T, S)] / 2c.  Impurity j is the pair
  // G_S[b..., m] (S[j]) and H_S[m, f...] (Sn[j]); each impure two-site middle
  // matrix gets its own partial SVD of rank <= dcut, the isometries are the
  // pure step's, and the new impurity has the two terms side by side along m.
  for (int j = 0; j < c.nimp; ++j) {
    const uint32_t kind = uint32_t(c.imp_kind[j]);
    const int64_t m = c.imp_r[j];
    const double *GS = static_cast<const double *>(c.S[j].ptr);
    const double *HS = static_cast<const double *>(c.Sn[j].ptr);
    std::vector<std::pair<std::string, int64_t>> lbm, lfm{{"kk", m}};
    for (int a = 0; a < d; ++a) lbm.push_back({bn[a], dims[a]});
    lbm.push_back({"kk", m});
    for (int a = 0; a < d; ++a) lfm.push_back({fn[a], dims[a]});
    const View vGS = contiguous(lbm), vHS = contiguous(lfm);
    View vGSA = vGS, vHSB = vHS;
    for (int a = 0; a < d; ++a) {
      vGSA = rename(vGSA, {{bn[a], nm("bA", a)}});
      vHSB = rename(vHSB, {{fn[a], nm("fB", a)}});
    }
    vGSA = rename(vGSA, {{"kk", "kA"}});
    vHSB = rename(vHSB, {{"kk", "kB"}});
    auto xview = [&](int64_t rows, int64_t l) {  // [kA, bB_perp..., l]
      std::vector<std::pair<std::string, int64_t>> v{{"kA", rows}};
      for (int a : perp) v.push_back({nm("bB", a), dims[a]});
      v.push_back({"l", l});
      return contiguous(v);
    };
    auto yview = [&](int64_t l, int64_t cols) {  // [l, fA_perp..., kB]
      std::vector<std::pair<std::string, int64_t>> v{{"l", l}};
      for (int a : perp) v.push_back({nm("fA", a), dims[a]});
      v.push_back({"kB", cols});
      return contiguous(v);
    };
    const int64_t mcap = 2 * int64_t(dcut);
    double *GSn = c.wsp<double>("iG", size_t(nnew) * mcap * 8);
    double *HSn = c.wsp<double>("iH", size_t(nnew) * mcap * 8);
    double *gt = c.wsp<double>("iGt", size_t(nnew) * dcut * 8);
    // impurity on the lower site: M_1 = sum_j H_S[m, f_perp, j] Ut[j, b_perp, kB]
    const SwapOut s1 =
        partial_svd(HS, rename(vHS, {{"kk", "kA"}, {fn[mu], "j"}}), m, Ut, vUB, k, 1u + 2u * kind, "i", false);
    const int64_t d1 = s1.dc;
    gblock(GS, vGSA, m, s1.Xs, xview(m, d1), d1, gt);
    hblock(s1.Ys, yview(d1, k), k, Vt, vVB, d1, HSn);
    // impurity on the upper site: M_2 = sum_j Vt[kA, f_perp, j] G_S[j, b_perp, m]
    const SwapOut s2 =
        partial_svd(Vt, vVA, k, GS, rename(vGS, {{"kk", "kB"}, {bn[mu], "j"}}), m, 2u + 2u * kind, "i", false);
    const int64_t d2 = s2.dc, mn = d1 + d2;
    apply_map(gt, IN_F64, contiguous({{"b", nnew}, {"l", d1}}), nullptr, {}, {}, GSn, OUT_F64, 0,
              View{Leg{"b", nnew, mn}, Leg{"l", d1, 1}}, st);
    gblock(Ut, vUA, k, s2.Xs, xview(k, d2), d2, gt);
    apply_map(gt, IN_F64, contiguous({{"b", nnew}, {"l", d2}}), nullptr, {}, {}, GSn + d1, OUT_F64, 0,
              View{Leg{"b", nnew, mn}, Leg{"l", d2, 1}}, st);
    hblock(s2.Ys, yview(d2, m), m, HS, vHSB, d2, HSn + size_t(d1) * nnew);
    scale_by_inverse(GSn, nnew * mn, c.scal(), 1.0, st);
    scale_by_inverse(HSn, nnew * mn, c.scal(), 0.5, st);
    c.ensure(c.S[j], size_t(nnew) * mn * 8);
    c.ensure(c.Sn[j], size_t(nnew) * mn * 8);
    TRG_HIP_CHECK(hipMemcpyAsync(c.S[j].ptr, GSn, size_t(nnew) * mn * 8, hipMemcpyDeviceToDevice, st));
    TRG_HIP_CHECK(hipMemcpyAsync(c.Sn[j].ptr, HSn, size_t(nnew) * mn * 8, hipMemcpyDeviceToDevice, st));
    c.imp_r[j] = int(mn);
  }

  trg_step_rec hr{};
  hr.n = n_step;
  hr.axis = mu;
  hr.join_precision = c.cfg.precision;
  for (int a = 0; a < 4; ++a) {
    hr.dims[a] = a < d ? nd[a] : 0;
    hr.side[a] = -1;
  }
  c.host_rec.push_back(hr);
  for (int a = 0; a < d; ++a) c.dims[a] = nd[a];
  c.r = dc;
  c.nsteps = n_step;
  if (c.z2) {
    for (int nu : perp) c.z2_legs[nu] = new_legs[nu];
    c.z2_bond = pure.par;
  }
}

}  // namespace trg
