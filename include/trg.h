/*
 * libtrg -- HOTRG / ATRG coarse-graining of the Ising tensor network on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: S. Akiyama, Y. Kuramashi, T. Yamashita, Y. Yoshimura, "Phase
 * transition of four-dimensional Ising model with tensor network scheme",
 * Lattice 2019 (arXiv:1911.12954).  HOTRG: Sec. 2 and Fig. 1; ATRG: Sec. 2
 * and Fig. 2; impure-tensor observables: Sec. 3.1.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - A site tensor of a d-dimensional lattice (d in {2,3,4}) has 2d legs in the
 *   order (x, x', y, y', z, z', t, t'): for axis nu the backward leg is 2*nu,
 *   the forward leg 2*nu+1, and both legs of an axis have the same dim.
 *   Tensors are dense, row-major (last leg fastest), FP64, in device memory
 *   owned by the context.
 * - All work of a context is enqueued on the HIP stream given in its config
 *   (NULL = the legacy default stream).  Step calls are asynchronous; calls
 *   that return numbers to the host synchronise that stream.
 * - Return codes: TRG_OK (0) or a negative TRG_E* code.  No C++ exception
 *   crosses this interface.  An error found before any work is enqueued
 *   leaves the context unchanged.  An error found on the device (non-finite
 *   or zero norm, eigensolver not converged) is reported by the next call
 *   that synchronises; the context is then poisoned and every later call on
 *   it returns TRG_ESTATE.  trg_last_error() describes the latest error.
 * - Diagnostics from the environment, both off by default: TRG_PROGRESS
 *   makes every join launch synchronise its stream and print one line on
 *   stderr when it is done (for steps that run for minutes); TRG_DEBUG
 *   copies back and summarises each intermediate of an ATRG step on stderr.
 */
#ifndef TRG_H
#define TRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TRG_OK = 0,
  TRG_EINVAL = -1,   /* bad argument or shape */
  TRG_ENOMEM = -2,   /* device allocation failed */
  TRG_EHIP = -3,     /* HIP runtime error */
  TRG_ESTATE = -4,   /* wrong state: poisoned context, impurity not enabled, ... */
  TRG_ENUMERIC = -5  /* NaN/Inf or zero norm, eigensolver did not converge */
};

/* Arithmetic of the block-spin contraction (the D^{4d-1} join of Sec. 2).
 * Gram matrices, their eigendecomposition, normalisation and the
 * accumulated free energy are FP64 in every mode. */
enum {
  TRG_FP64 = 0,     /* FP64 operands, FP64 MFMA, FP64 result */
  TRG_FP32 = 1,     /* operands rounded to FP32, FP32 MFMA, FP32 result */
  TRG_BF16X3 = 2,   /* operands split a = hi + lo (two BF16), hi*hi + hi*lo +
                       lo*hi on BF16 MFMA with FP32 accumulation */
  TRG_BF16X6 = 3    /* operands rounded to FP32 and split exactly into three
                       BF16 planes, fl32(a) = hi + mid + lo; the six products
                       hi*hi + hi*mid + mid*hi + mid*mid + hi*lo + lo*hi on
                       BF16 MFMA, summed in FP32 over groups of 128 K elements
                       and the groups in FP64; FP32 result */
};

enum { TRG_HOTRG = 0, TRG_ATRG = 1 };

/* impurity bits: energy (S_E = dT0/dbeta) and magnetization (S_M) */
enum { TRG_IMPURE_E = 1u, TRG_IMPURE_M = 2u };

typedef struct trg_config {
  int precision;          /* TRG_FP64 (default), TRG_FP32, TRG_BF16X3, TRG_BF16X6
                             (HOTRG; ATRG takes TRG_FP64 or TRG_FP32) */
  int method;             /* TRG_HOTRG (default) or TRG_ATRG */
  int dcut;               /* bond dimension used by trg_run; > 0 */
  unsigned impure;        /* TRG_IMPURE_E | TRG_IMPURE_M, or 0 */
  int rsvd_p;             /* ATRG randomized SVD oversampling; 0 = 4*dcut, < 0 = none */
  int rsvd_q;             /* ATRG power iterations; 0 = 2*dcut, < 0 = none */
  uint64_t seed;          /* ATRG trial-matrix seed */
  void *stream;           /* hipStream_t; NULL = default stream */
  /* Device allocator.  NULL alloc = hipMalloc/hipFree.  alloc returns NULL on
   * failure; free must accept any pointer alloc returned.  A custom allocator
   * must be stream-ordered on `stream`: a block given to free may be handed
   * out again only to work enqueued on that stream after the free (torch's
   * caching allocator behaves so), because the library frees buffers that
   * queued kernels still use without waiting for them.  With hipFree the
   * library waits for the stream before a buffer is freed. */
  void *(*alloc)(size_t bytes, void *user);
  void (*free)(void *ptr, void *user);
  void *alloc_user;
  size_t workspace_bytes; /* cap on the join workspace; 0 = automatic */
  int fp64_steps;         /* HOTRG: the first fp64_steps steps join in FP64
                             whatever `precision` is (0 = none).  Step n
                             enters ln Z/V with weight 2^-n, so the leading
                             steps dominate the rounding error of f. */
  int z2;                 /* ATRG from trg_init_ising at h = 0 only: 1 keeps
                             the pure tensor exactly Z2 symmetric (the
                             symmetry of the h = 0 Ising tensor) by doing the
                             swap's randomized SVD, the canonical form and the
                             HOSVD parity sector by parity sector; 0 (default)
                             = plain decompositions. */
} trg_config;

typedef struct trg_ctx trg_ctx;

/* Per-step record of a HOTRG step (what the host can read back). */
typedef struct trg_step_rec {
  int n;                  /* step number, 1-based */
  int axis;               /* coarse-grained axis */
  int dims[4];            /* per-axis leg dims after the step */
  int side[4];            /* per transverse axis: 0 backward, 1 forward pair; -1 on axis */
  int kept[4];            /* kept columns k_nu; 0 on the coarse-grained axis */
  int degenerate_cut[4];  /* 1 if the cut splits a degenerate eigenspace */
  int sweeps[4];          /* chosen side: Jacobi sweeps (order <= 160), else the
                             number of eigenvectors computed */
  int join_precision;     /* TRG_FP64 / TRG_FP32 / TRG_BF16X3 / TRG_BF16X6 of this step's join */
  double ln_c;            /* ln of the Frobenius norm c_n of the new tensor */
  double eps[4][2];       /* discarded eigenvalue sum, [axis][backward, forward] */
  double seconds;         /* host wall time between launch of the step and the
                             next synchronisation, 0 if not measured */
} trg_step_rec;

/* Create a context holding the initial Ising site tensor T0 of the
 * d-dimensional Ising model that the paper studies (Sec. 1; the 4D model of
 * Sec. 3.1) at inverse temperature beta >= 0 and field h (weight
 * e^{-beta H}, H = -sum s_i s_j - h sum s_i), built from the bond split
 * W = [[sqrt(cosh b), sqrt(sinh b)], [sqrt(cosh b), -sqrt(sinh b)]] in closed
 * form, and the impure tensors requested by cfg->impure (S_E needs beta > 0).
 * The tensor is normalised by its Frobenius norm c_0 and ln c_0 starts the
 * free-energy accumulator.  cfg may be NULL (all defaults, dcut = 8).
 * Errors: TRG_EINVAL (d, beta, h, cfg fields), TRG_ENOMEM, TRG_EHIP. */
int trg_init_ising(trg_ctx **out, double beta, double h, int d, const trg_config *cfg);

/* Create a context from an arbitrary FP64 site tensor copied from host memory
 * (dims[nu] per axis, 2d legs in the conventional order, row-major).  The
 * tensor is normalised like T0.  Used for tests on random tensors and for
 * checkpoint restore.  Impurities are not available on such a context. */
int trg_init_tensor(trg_ctx **out, int d, const int *dims, const double *host_tensor,
                    const trg_config *cfg);

/* One HOTRG coarse-graining step along `axis` (0 <= axis < d) with bond
 * dimension `dcut` (Sec. 2, Fig. 1): HOSVD isometries from the two-site Gram
 * matrices (FP64 on the device: cyclic Jacobi up to order 160; above it
 * Householder tridiagonalisation, bisection for every eigenvalue and inverse
 * iteration for the kept eigenvectors), the block-spin
 * contraction in the configured precision, Frobenius normalisation and
 * acc += 2^{-n} ln c_n.  Impure tensors follow with the same isometries and
 * c_n.  Asynchronous.  Errors: TRG_EINVAL, TRG_ESTATE, TRG_ENOMEM, TRG_EHIP. */
int trg_hotrg_step(trg_ctx *ctx, int axis, int dcut);

/* The same step for n distinct contexts that share d, join precision,
 * current dims and the stream.  The Gram eigendecompositions of all n
 * contexts (every transverse axis, both sides) run in one launch; the Gram
 * products are formed context by context; then every kernel of the
 * contraction and the normalisation -- operand builds, zero padding, the
 * joins, the post-join maps, the norm and the scaling -- is launched once for
 * all contexts with the same impurities (up to 64 per launch, each context
 * in its own slot of the workspace of the first context of the batch).  The
 * batch's workspace budget is the sum of its contexts' cfg.workspace_bytes
 * (85 % of the free device memory if one of them is 0); contexts that do
 * not fit in it together are stepped in consecutive groups.  Results are
 * bit-identical to n separate trg_hotrg_step calls.
 * Errors: TRG_EINVAL (NULL or duplicate context, mismatched contexts, bad
 * axis or dcut) and TRG_ESTATE (a poisoned context) leave every context
 * unchanged.  TRG_EHIP or TRG_ENUMERIC poisons every context of the batch.
 * TRG_ENOMEM during the contraction can leave the first contexts stepped and
 * the rest not; trg_get_dims' step count tells which. */
int trg_hotrg_step_batch(trg_ctx *const *ctxs, int n, int axis, int dcut);

/* ATRG step along `axis` (Sec. 2, Fig. 2) with bond dimension `dcut`
 * (1..256): canonical form of the factored tensor, the index-swapping partial
 * SVD by randomized SVD (trial matrix N(0,1) from Philox4x32-10 keyed by
 * (cfg->seed, step); cfg->rsvd_p oversampling, cfg->rsvd_q iterations;
 * defaults p = 4 dcut, q = 2 dcut as in Sec. 3.2), the HOSVD isometries of
 * the two adjacent decomposed tensors and the contraction completing the
 * block-spin transformation; FP64 throughout, or the contraction GEMMs in
 * FP32 when cfg->precision == TRG_FP32.  The context must have been created
 * with method TRG_ATRG (trg_init_ising or trg_init_factors).  Impure
 * tensors requested by cfg->impure (trg_init_ising) are kept as their own
 * pair of pieces S = sum_m G_S[b, m] H_S[m, f] (bond 2 dcut after a step):
 * the energy impurity carries each bond's beta-derivative on its forward
 * end (same -Tr S_E / Tr T), each impure two-site product gets its own
 * randomized partial SVD of rank <= dcut (trial stream 1 + 2 kind + term,
 * kind 0 = E, 1 = M; term 0 = impurity on the lower site, 1 = upper), and
 * the pure step's HOSVD isometries and c_n are applied; the paper uses the
 * impure-tensor method within ATRG (Sec. 3.2) without giving it.
 * With cfg->z2 (see trg_atrg_parities) the trial matrix of the pure swap
 * keeps only the entries whose row parity equals the sector of its column
 * (column c in sector c mod 2 while both sectors have room for it, the rest
 * in the larger sector), and every factorisation of the step stays inside
 * one sector, so the zeros of the symmetric tensor stay exact zeros; the
 * impurity SVDs stay plain.
 * Asynchronous, except that a Z2 step waits for the device three times to
 * read back the parities of its new bonds and legs.  Errors: TRG_EINVAL, TRG_ESTATE, TRG_ENOMEM, TRG_EHIP. */
int trg_atrg_step(trg_ctx *ctx, int axis, int dcut);

/* Create an ATRG context from host pieces T[b, f] = sum_l G[b, l] H[l, f]:
 * G row-major (prod dims) x r with the d backward legs in axis order, H
 * row-major r x (prod dims) with the forward legs.  No normalisation is
 * applied.  For tests and checkpoint restore.  cfg->method must be ATRG. */
int trg_init_factors(trg_ctx **out, int d, const int *dims, int r, const double *host_G,
                     const double *host_H, const trg_config *cfg);

/* Singular values (descending, *n of them) of the latest ATRG swap. */
int trg_atrg_spectrum(trg_ctx *ctx, double *out, int cap, int *n);

/* Z2 sectors of an ATRG context created with cfg->z2 = 1.  The h = 0 Ising
 * tensor is invariant under the flip of every spin, the symmetry whose
 * spontaneous breaking X indicates (Sec. 3.1): in the
 * basis where each leg index and each bond index has a definite parity
 * (0 even, 1 odd), G[b, l] and H[l, f] vanish unless the parities of the
 * legs b (f) add up to that of l.  legs_out receives the parity of every leg
 * index, axis after axis (dims[0] + ... + dims[d-1] entries, the forward and
 * backward leg of an axis share them); bond_out the parity of each of the r
 * bond indices; *r_out (if not NULL) the bond r.  Either array pointer may
 * be NULL.  Host memory, caller owns it.
 * Synchronises.  Errors: TRG_EINVAL (capacity too small), TRG_ESTATE (not a
 * Z2 context). */
int trg_atrg_parities(trg_ctx *ctx, int *legs_out, size_t cap_legs, int *bond_out, size_t cap_bond, int *r_out);

/* The current pieces of an ATRG context, T[b, f] = sum_l G[b, l] H[l, f]
 * (Sec. 2, Fig. 2): host_G receives G row-major (prod dims) x r with the d
 * backward legs in axis order, host_H receives H row-major r x (prod dims)
 * with the forward legs (the layout trg_init_factors takes); *r_out the
 * bond r.  Either array pointer may be NULL (then only *r_out is written).
 * Host memory, caller owns it.  Synchronises.  Errors: TRG_EINVAL (capacity
 * too small), TRG_ESTATE (a HOTRG context). */
int trg_get_factors(trg_ctx *ctx, double *host_G, size_t cap_G, double *host_H, size_t cap_H, int *r_out);

/* Coarse-grain the periodic lattice L^d (L = 2^m, m >= 1; each step halves
 * the lattice, so the block volume reaches 2^n after n steps as in the
 * caption of Fig. 5, Sec. 3.1, and 1024^4 takes 40 steps): steps n along
 * axis (n-1) mod d with cfg->dcut, using the context's method, from the
 * context's next step up to n = d*m (all d*m steps for a fresh context; a
 * context imported from a checkpoint finishes the lattice).  TRG_EINVAL if
 * the context is already past d*m steps.  Synchronises once at the end and
 * returns TRG_ENUMERIC if a step failed. */
int trg_run(trg_ctx *ctx, long long L);

/* ln Z / V of the periodic lattice whose single block is the current tensor:
 * acc + 2^{-n} ln Tr T_n (Tr joins each backward leg to the forward leg of
 * the same axis).  This is the free energy per site up to the factor -1/beta
 * that the paper compares between ATRG and HOTRG and over the bond
 * dimension (Sec. 3.2, Figs. 7 and 8).  Synchronises.  Caller owns *out. */
int trg_free_energy(trg_ctx *ctx, double *lnz_per_site);

/* Degeneracy indicator of the current tensor T (the quantity the
 * paper follows against the iteration to locate the transition, Sec. 3.1,
 * Fig. 3; defined in its reference by Gu and Wen):
 *   X = (Tr M)^2 / Tr(M M),  M[a][a'] = sum over the other axes' diagonals
 *   of T[.., a, a', ..] (the legs of `axis` open, every other pair traced).
 * X -> 1 in the disordered phase, 2 with the Z2 symmetry broken.  Scale
 * invariant.  HOTRG and ATRG contexts (on the factored pieces:
 * M[a][a'] = sum_l sum G[.., a, .., l] H[l, .., a', ..] with the other legs
 * joined; the paper follows X with ATRG too, Sec. 3.2).  Synchronises the
 * stream.  Errors: TRG_EINVAL (bad axis), TRG_ENUMERIC (vanishing two-site
 * trace). */
int trg_indicator_x(trg_ctx *ctx, int axis, double *X);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): X of
 * trg_indicator_x for a HOTRG context, computed by the same kernels with the
 * partial-trace matrix and the two traces in a static device array of
 * 512 KiB + 256 bytes that the library holds on each GPU until the process
 * ends, instead of the context's workspace.  It allocates nothing: no
 * hipMalloc, hipFree or allocator callback.  Limit: dims[axis] <= 256.
 * Every call on one GPU uses that GPU's array and leaves its contents
 * behind (the kernels overwrite every entry they read); calls that overlap
 * on one GPU (from several threads or streams) race and give undefined
 * results.  Synchronises the context's stream.  Errors: TRG_EINVAL (NULL,
 * bad axis, dims[axis] > 256, ATRG context), TRG_ENUMERIC (vanishing
 * two-site trace). */
int trg_indicator_x_noalloc(trg_ctx *ctx, int axis, double *X);

/* E = <H>/V = -Tr S_E / Tr T and M = <s> = Tr S_M / Tr T (impure-tensor
 * method, Sec. 3.1; HOTRG and ATRG contexts).  Synchronises.  TRG_ESTATE if
 * that impurity was not enabled. */
int trg_impure_energy(trg_ctx *ctx, double *E);
int trg_impure_magnetization(trg_ctx *ctx, double *M);

/* Current leg dims per axis (d entries) and the number of steps taken. */
int trg_get_dims(const trg_ctx *ctx, int *dims, int *steps);

/* Copy the current normalised tensor (which = 0 pure, 1 S_E, 2 S_M) to host
 * memory (cap = capacity in doubles).  Synchronises. */
int trg_get_tensor(trg_ctx *ctx, int which, double *host_out, size_t cap);

/* Copy the isometry U_nu[(a,b),k] of the latest step for transverse axis nu
 * (row-major d_nu^2 x k_nu) and the descending spectrum of the chosen Gram
 * (d_nu^2 values).  Either pointer may be NULL.  Synchronises. */
int trg_get_isometry(trg_ctx *ctx, int nu, double *host_U, size_t capU,
                     double *host_spectrum, size_t capS);

/* Checkpoint of a context (the state after step n: the tensors -- T and the
 * impure S for HOTRG, the pieces G, H and each impurity's pair for ATRG --,
 * the free-energy accumulator, n, dims, the step records and the settings
 * that fix the numerics).  trg_export_state with host_buf NULL stores the
 * blob size in *size; otherwise it writes the blob (cap >= *size, else
 * TRG_EINVAL) to caller-owned host memory.  Synchronises.
 * trg_import_state creates a context from such a blob; the blob fixes method,
 * precision, dcut, impurities, RSVD settings and seed, cfg (may be NULL)
 * contributes the stream, allocator and workspace budget.  Stepping the
 * imported context gives the bits of the uninterrupted run.  The last ATRG
 * swap spectrum and the latest isometries are not part of the state.
 * Errors: TRG_EINVAL (NULL, bad magic, version or size, inconsistent
 * header), TRG_ENOMEM, TRG_EHIP. */
int trg_export_state(trg_ctx *ctx, void *host_buf, size_t cap, size_t *size);
int trg_import_state(trg_ctx **out, const void *host_buf, size_t size, const trg_config *cfg);

/* Copy up to cap step records (oldest first); *n receives the count. */
int trg_step_log(trg_ctx *ctx, trg_step_rec *out, int cap, int *n);

/* Free-energy accumulator sum_{k<=n} 2^{-k} ln c_k (synchronises). */
int trg_accumulator(trg_ctx *ctx, double *acc);

/* Device bytes of a context at steady state for (d, dcut, precision, method,
 * impure): trg_resident_bytes = its tensors (kept for the whole run),
 * trg_workspace_bytes = the join workspace of the default plan (whole Bt,
 * slices of about 32768 GEMM rows of A), trg_footprint_bytes = the sum.
 * Pure functions of their arguments (no device access). */
size_t trg_footprint_bytes(int d, int dcut, int precision, int method, unsigned impure);
size_t trg_resident_bytes(int d, int dcut, int precision, int method, unsigned impure);
size_t trg_workspace_bytes(int d, int dcut, int precision, int method, unsigned impure);

/* Let ctx use donor's workspace (its own is released).  Both contexts must
 * use the same stream, and both hipMalloc or both a custom allocator; their
 * calls must not overlap: steps of contexts that share a workspace are
 * serialised on that stream (one serving lane).  The workspace lives until
 * its last user is freed and is released through the free callback of the
 * context that created it, which must stay callable until then.
 * Errors: TRG_EINVAL for NULL or mismatched contexts. */
int trg_share_workspace(trg_ctx *ctx, trg_ctx *donor);

/* Wait for all work of the context's stream. */
int trg_sync(trg_ctx *ctx);

/* Destroy a context (NULL allowed); frees through the config's allocator. */
void trg_free(trg_ctx *ctx);

/* Text of the latest error on ctx (or of this thread's latest call that had
 * no context).  Valid until the next call on the same context/thread. */
const char *trg_last_error(const trg_ctx *ctx);

/* ---- kernel-level entry points (used by the kernel tests and the bench) ----
 * All pointers are device pointers; all calls are asynchronous on `stream`.
 */

/* C[m][n] (+)= sum_k A[m][k] * Bt[n][k] for the join GEMM (Sec. 2: the
 * D^{4d-1} contraction).  A is M x K with row stride lda, Bt is N x K with row
 * stride ldb, C is M x N with row stride ldc.  M, N must be multiples of the
 * tile (trg_gemm_tile), K a multiple of trg_gemm_tile's K granule; the
 * caller zero-pads.  precision selects the element types: FP64 (double in,
 * double out), FP32 (float in, float out), BF16X3 (A = A_hi, A + M*lda
 * elements = A_lo, likewise for Bt; bf16 in, float out), BF16X6 (three
 * planes M*lda elements apart: A_hi, A_mid, A_lo; likewise for Bt; bf16 in,
 * float out).  accumulate != 0 adds to C.  Returns TRG_EINVAL on shape
 * violations. */
int trg_gemm(int precision, const void *A, const void *Bt, void *C, long long M, long long N,
             long long K, long long lda, long long ldb, long long ldc, int accumulate,
             void *stream);

/* Tile sizes (rows of A, rows of Bt) and K granule of trg_gemm. */
int trg_gemm_tile(int precision, int *tile_m, int *tile_n, int *tile_k);

/* Batched symmetric eigendecomposition by cyclic Jacobi (FP64): for each of
 * `batch` matrices of order n (row-major, stride n*n apart) writes the
 * eigenvalues in descending order to w[b*n ...] and the eigenvectors as
 * columns of V[b*n*n ...] (row-major, column j belongs to w[j]).  A is
 * overwritten.  sweeps[b] receives the sweeps used (-1: not converged). */
int trg_eigh(double *A, double *w, double *V, int *sweeps, int n, int batch, void *stream);

/* The eigensolver of the isometry selection (Sec. 2: HOSVD of HOTRG and
 * ATRG keeps the eigenvectors of the largest eigenvalues of each Gram
 * matrix): for each of `batch` symmetric matrices of order n (layout as
 * trg_eigh) every eigenvalue in descending order, and eigenvectors only for
 * the leading kk indices, kk = k extended while the next eigenvalue is within
 * cluster_rel * w[0] of the previous one (a near-degenerate cluster that the
 * cut at k splits); columns kk.. of V are zero and sweeps[b] receives kk.
 * Orders up to 160 use the Jacobi solver of trg_eigh instead (every vector,
 * sweeps[b] the sweeps used); larger ones Householder reduction, bisection
 * for the eigenvalues and inverse iteration for the vectors.  A is overwritten.  work: device
 * memory of trg_eigh_top_work_bytes(n, batch) bytes (may be NULL when n <=
 * 160), owned by the caller, not kept.  Asynchronous on `stream`.  Errors:
 * TRG_EINVAL (n outside 1..1024, k < 1, batch < 1, cluster_rel outside
 * [0, 1), a NULL pointer). */
int trg_eigh_top(double *A, double *w, double *V, int *sweeps, int n, int batch, int k, double cluster_rel,
                 void *work, void *stream);
size_t trg_eigh_top_work_bytes(int n, int batch);

/* ---- diagnostics ----
 * Time the join GEMM launches of a context with HIP events on its stream
 * (on = 1 enables; trg_join_profile synchronises, returns the summed kernel
 * milliseconds, launch count and issued 2*M*N*K flops of the padded
 * problems since the last query, and resets them). */
int trg_set_profiling(trg_ctx *ctx, int on);
int trg_join_profile(trg_ctx *ctx, double *ms, long long *launches, double *flops);

/* Force the HOSVD side (0 backward pairs, 1 forward pairs, -1 automatic:
 * forward unless the backward truncation error is smaller by a relative
 * 1e-10).  A gauge choice used by the tests of gauge invariance. */
int trg_set_force_side(trg_ctx *ctx, int side);

#ifdef __cplusplus
}
#endif

#endif /* TRG_H */
