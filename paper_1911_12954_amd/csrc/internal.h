// Internal interfaces between the kernel files and the step engine of libtrg.
#pragma once

#include "common.h"

namespace trg {

// ------------------------------------------------------------------ GEMM ---
struct GemmTile {
  int m, n, k;
};
// join operand planes and bytes per element over all planes, per precision
// (FP64, FP32, BF16X3 = hi + lo, BF16X6 = hi + mid + lo)
inline int operand_planes(int prec) { return prec == 2 ? 2 : (prec == 3 ? 3 : 1); }
inline int operand_bytes(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2 * operand_planes(prec)); }
GemmTile gemm_tile(int prec);
// nb > 1: a strided batch of nb products in one launch (grid.z), product b
// reading A + b * batch_a, Bt + b * batch_b and writing C + b * batch_c
// (element strides)
void gemm_nt(int prec, const void *A, const void *Bt, void *C, uint64_t M, uint64_t N, uint64_t K,
             uint64_t lda, uint64_t ldb, uint64_t ldc, bool accum, hipStream_t st, uint32_t nb = 1,
             uint64_t batch_a = 0, uint64_t batch_b = 0, uint64_t batch_c = 0);
// split-K FP64 Gram product: C[s] = A[:, ks] * Bt[:, ks]^T for split s, tile 64
void gemm_nt_splitk_f64(const double *A, const double *Bt, double *Cpart, uint64_t M, uint64_t N,
                        uint64_t K, uint64_t lda, uint64_t ldb, uint32_t splits, uint64_t kper,
                        hipStream_t st);

// Contexts one batched launch serves (pointer tables are passed by value)
constexpr int TRG_MAXB = 64;

// ------------------------------------------------------------ tensor map ---
// out[sum_i o_i so_i] = sum_{s} in[sum_i o_i si_i + sum_j s_j ssi_j] *
//                                U[sum_i o_i su_i + sum_j s_j ssu_j]
// over the iteration space o (dims listed outermost first).  With nsum = 0
// and U == nullptr it is a strided copy.  Output kinds: FP64, FP32 or a BF16
// split of fl32(v) into planes lo_plane elements apart: two planes (hi, lo)
// or three (hi, mid, lo, which sum to fl32(v) exactly).
constexpr int MAP_MAXD = 12;
struct MapDim {
  int64_t size, so, si, su;
};
struct MapSum {
  int64_t size, si, su;
};
enum OutKind { OUT_F64 = 0, OUT_F32 = 1, OUT_BF16X2 = 2, OUT_BF16X3 = 3 };
enum InKind { IN_F64 = 0, IN_F32 = 1 };

void tensor_map(const void *in, int in_kind, const double *U, void *out, int out_kind,
                int64_t lo_plane, const MapDim *dims, int ndims, const MapSum *sums, int nsum,
                hipStream_t st);
// the same map for nb contexts in one launch (grid.y = context): context i
// reads ins[i] and Us[i] and writes outs[i]; every context has the same shape
void tensor_map_batch(const void *const *ins, int in_kind, const double *const *Us, void *const *outs, int nb,
                      int out_kind, int64_t lo_plane, const MapDim *dims, int ndims, const MapSum *sums,
                      int nsum, hipStream_t st);

// zero the padding of a row-major rows_pad x ld matrix whose valid part is
// rows x cols (elements of elem_bytes; `planes` planes plane_stride apart)
void zero_pad(void *buf, int64_t rows, int64_t rows_pad, int64_t cols, int64_t ld, int elem_bytes,
              int planes, int64_t plane_stride, hipStream_t st, int nb = 1, int64_t batch_stride = 0);
void fill_zero(void *buf, size_t bytes, hipStream_t st);

// sum of split-K partials: out[r*ldo + c] = sum_s part[s][r*ldp + c]
void reduce_splits(const double *part, int splits, int64_t rows, int64_t cols, int64_t ldp,
                   int64_t split_stride, double *out, int64_t ldo, hipStream_t st);

// Gram of the two-site tensor from the one-site environments P and Q
// (both (dmu*dn) x (dmu*dn), row index (i, a)): G[(a,b),(a',b')] =
// sum_{i,i'} P[(i,a),(i',a')] Q[(i,b),(i',b')]
void gram_combine(const double *P, const double *Q, int dmu, int dn, double *G, hipStream_t st);

// Frobenius norm of n doubles: partials then one block; writes
// scal[0] = c, scal[1] = 1/c, scal[2] = ln c, acc[0] += weight * ln c; sets
// *err |= 1 when c is zero or not finite.
void norm_and_accumulate(const double *x, int64_t n, double *partial, int nblocks, double *scal,
                         double *acc, double weight, int *err, hipStream_t st);
int norm_blocks();
// x[i] *= factor * scal[1]
void scale_by_inverse(double *x, int64_t n, const double *scal, double factor, hipStream_t st);
// both for nb contexts in one launch each: context i normalises xs[i] with
// its own scalars scals[i] (c, 1/c, ln c, acc at [3]), error flag errs[i],
// accumulator weight weight[i] (2^-n of its own step n), and writes ln c to
// recs[i] (may be null); partial holds nb * nblocks
struct NormBatch {
  const double *x[TRG_MAXB];
  double *scal[TRG_MAXB];
  int *err[TRG_MAXB];
  double *rec[TRG_MAXB];
  double weight[TRG_MAXB];
};
void norm_and_accumulate_batch(const NormBatch &b, int nb, int64_t n, double *partial, int nblocks,
                               hipStream_t st);
void scale_by_inverse_batch(double *const *xs, const double *const *scals, int nb, int64_t n, double factor,
                            hipStream_t st);

// traces: out[j] = sum_{x_nu} X_j[x, x, y, y, ...] for up to 3 tensors
// {Tr M, Tr(M M)} into out[0..1] for M[a][a'] = T with the legs of `axis`
// open and every other axis' leg pair traced (M: dims[axis]^2 workspace)
void indicator_traces(const double *T, const int *dims, int d, int axis, double *M, double *out, hipStream_t st);
// {Tr M, Tr(M M)} of an n x n matrix already formed
void indicator_reduce(const double *M, int n, double *out, hipStream_t st);
void periodic_traces(const double *const *X, int count, const int *dims, int d, double *out,
                     hipStream_t st);

// initial Ising tensors (closed form) into T, SE, SM (each may be null)
void ising_init(double *T, double *SE, double *SM, int d, double beta, double h, hipStream_t st);

// ------------------------------------------------------------- eigen ---
// batched Jacobi: A (batch x n x n) overwritten; w, V sorted descending
// Orders up to JACOBI_MAX_N use cyclic Jacobi (rotations only between
// coupled indices, so exact zeros of A stay exact zeros); larger orders use
// Householder tridiagonalisation + QL, which keeps a block-diagonal A block
// diagonal only when each block's indices are contiguous.
constexpr int JACOBI_MAX_N = 160;
void eigh_batched(double *A, double *w, double *V, int *sweeps, int n, int batch, hipStream_t st);
// Every eigenvalue (descending) but eigenvectors only for the leading kk
// indices: k, extended while the next eigenvalue continues a cluster (gap
// <= cluster_rel * lambda_max); the other columns of V are zero.  Above the
// Jacobi range: Householder, bisection and inverse iteration (sweeps receives
// kk); up to it, the full Jacobi solver.  work: eigh_top_work_doubles(n,
// batch) doubles of device memory.
size_t eigh_top_work_doubles(int n, int batch);
void eigh_top_batched(double *A, double *w, double *V, int *sweeps, int n, int batch, int k, double cluster_rel,
                      double *work, hipStream_t st);

// isometry selection of one transverse axis from both sides' eigensystems
struct SelectOut {
  double *U;        // n x k row-major
  double *rec_eps;  // [2]
  int *rec_int;     // [side, k, degenerate, sweeps]
  double *spectrum; // n (chosen side)
};
// Degenerate eigenspaces: neighbouring eigenvalues within cluster_rel
// lambda_max (see degeneracy_window) are expressed in a canonical basis.
void select_isometry(const double *w2, const double *V2, const int *sweeps2, int n, int k,
                     int force_side, double cluster_rel, SelectOut out, hipStream_t st);

// Window of select_isometry for a Gram built from a tensor that an FP64
// contraction produced: FP64 rounding leaves the degeneracies that a symmetry
// makes exact as gaps of ~1e-17 lambda_max, and every gap above the window is
// resolved by the leading eigenvectors.  A tensor from an FP32 or split-BF16
// contraction carries ~1e-7 lambda_max of rounding on its Gram spectrum, so its
// window is 1e-6: rounding then does not pick the member of a degenerate pair
// that survives a cut.
constexpr double CLUSTER_REL_FP64 = 1e-10;
constexpr double CLUSTER_REL_MIXED = 1e-6;
inline double degeneracy_window(int producer_precision) {
  return producer_precision == 0 ? CLUSTER_REL_FP64 : CLUSTER_REL_MIXED;
}

}  // namespace trg
