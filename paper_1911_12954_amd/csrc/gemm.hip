// Join GEMM of the HOTRG block-spin contraction on gfx950 MFMA.
//
// C[m][n] (+)= sum_k A[m][k] * Bt[n][k]: both operands K-contiguous, so a
// workgroup streams BM rows of A and BN rows of Bt through LDS in tiles of
// RB bytes of K per row.  Inside a tile, lane group g = lane/16 of a wave
// owns bytes [g RB/4, (g+1) RB/4) of every row it reads; the k values a lane
// feeds to successive MFMAs are therefore contiguous in LDS, and A and B use
// the same assignment, so the contraction over k is unchanged.
//
//   FP64   v_mfma_f64_16x16x4_f64   128 x 128 tile, four 64 x 64 waves,
//          RB 128 (16 doubles, 4 MFMA k-steps), two padded LDS stages
//   FP32   v_mfma_f32_16x16x4_f32   128 x 128 tile, eight 64 x 32 waves,
//          RB 128 (32 floats, 8 k-steps), two padded stages; the MFMA sums
//          4 K tiles (128 products) in FP32, the groups are summed in FP64
//   BF16X3 v_mfma_f32_16x16x32_bf16 256 x 256 tile, eight 128 x 64 waves,
//          RB 64 (32 bf16 per plane, 1 k-step, three products hi*hi +
//          hi*lo + lo*hi into one FP32 accumulator), two swizzled stages
//   BF16X6 v_mfma_f32_16x16x32_bf16 128 x 128 tile, eight 64 x 32 waves,
//          RB 64, three planes (fl32(a) = hi + mid + lo exactly), six
//          products hi*hi + hi*mid + mid*hi + mid*mid + hi*lo + lo*hi; the
//          MFMA sums BF6_FLUSH K tiles in FP32, the groups are summed in
//          FP64 (FP32-accurate operands and FP64-grade accumulation), two
//          swizzled stages
//
// With two stages the next tile's global loads are in flight while the
// current tile feeds the MFMAs (one barrier per tile); with one stage two
// workgroups per CU overlap each other's waits.
//
// Workgroup ids are remapped so that each XCD (ids are dealt round-robin to
// the 8 XCDs) works on one contiguous range of tiles, walked in groups of
// GROUP_M tile-rows: neighbouring tiles on one XCD share A and Bt rows in
// that XCD's L2.
#include <type_traits>

#include "common.h"
#include "internal.h"

namespace trg {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int NUM_XCD = 8;
// FP32 join: K tiles (32 floats each) summed by the MFMA in FP32 before the
// partial sum is added to the FP64 accumulator
constexpr uint32_t F32_FLUSH = 4;
#ifndef TRG_GROUP_M
#define TRG_GROUP_M 8
#endif
constexpr int GROUP_M = TRG_GROUP_M;

// LDS stages of the FP64 / FP32 join kernels (compile-time tuning knobs)
#ifndef TRG_F64_STAGES
#define TRG_F64_STAGES 2
#endif
#ifndef TRG_F32_STAGES
#define TRG_F32_STAGES 2
#endif
#ifndef TRG_F32_WN
#define TRG_F32_WN 4
#endif
// BF16X6 join: K tiles (32 elements each) per FP32 group, and LDS stages
#ifndef TRG_BF6_FLUSH
#define TRG_BF6_FLUSH 4
#endif
#ifndef TRG_BF6_STAGES
#define TRG_BF6_STAGES 2
#endif
// BF16X6 join: global -> LDS prefetch distance in K tiles (1 or 2)
#ifndef TRG_BF6_PF
#define TRG_BF6_PF 2
#endif
constexpr uint32_t BF6_FLUSH = TRG_BF6_FLUSH;

template <int PREC> struct Prec;
template <> struct Prec<0> {  // FP64
  using in_t = double;
  using out_t = double;
  using acc_t = v4d;
  using frag_t = d2;
  static constexpr int planes = 1;
  static constexpr int elem = 8;
};
template <> struct Prec<1> {  // FP32
  using in_t = float;
  using out_t = float;
  using acc_t = v4f;
  using frag_t = f4;
  static constexpr int planes = 1;
  static constexpr int elem = 4;
};
template <> struct Prec<2> {  // BF16 x3
  using in_t = uint16_t;
  using out_t = float;
  using acc_t = v4f;
  using frag_t = bf16x8;
  static constexpr int planes = 2;
  static constexpr int elem = 2;
};
template <> struct Prec<3> {  // BF16 x6
  using in_t = uint16_t;
  using out_t = float;
  using acc_t = v4f;
  using frag_t = bf16x8;
  static constexpr int planes = 3;
  static constexpr int elem = 2;
};

__device__ inline void tile_coords(uint32_t wg, uint32_t tiles_m, uint32_t tiles_n, uint32_t &tm,
                                   uint32_t &tn) {
  const uint32_t total = tiles_m * tiles_n;
  // XCD-contiguous renumbering (bijective for any total)
  const uint32_t xcd = wg % NUM_XCD, idx = wg / NUM_XCD;
  const uint32_t per = total / NUM_XCD, rem = total % NUM_XCD;
  const uint32_t w = xcd * per + (xcd < rem ? xcd : rem) + idx;
  // grouped raster: GROUP_M tile-rows walked column by column
  const uint32_t group_size = GROUP_M * tiles_n;
  const uint32_t group = w / group_size;
  const uint32_t first_m = group * GROUP_M;
  const uint32_t gm = (tiles_m - first_m) < GROUP_M ? (tiles_m - first_m) : GROUP_M;
  const uint32_t in_group = w % group_size;
  tm = first_m + in_group % gm;
  tn = in_group / gm;
}

// LDS layout of one operand tile: rows of RB bytes of K.  Padded (SWZ 0):
// row stride RB + 16.  Swizzled (SWZ 1): row stride RB, and the 16-byte
// chunk c of row r is stored at chunk c ^ ((r / (256 / RB)) % (RB / 16)).
// Either way the 16 rows that one lane group reads fall on 16 disjoint
// 4-bank groups of the 64-bank LDS; with the swizzle, 16 consecutive lanes
// also store 256 contiguous bytes (no padding, no store conflicts).
template <int RB, int SWZ>
__device__ inline int lds_off(int row, int chunk) {
  if constexpr (SWZ == 0) {
    return row * (RB + 16) + (chunk << 4);
  } else {
    constexpr int CPR = RB / 16, RPL = 256 / RB;
    return row * RB + ((chunk ^ ((row / RPL) % CPR)) << 4);
  }
}
template <int RB, int SWZ>
constexpr int lds_stride() { return SWZ ? RB : RB + 16; }

// BM x BN tile per workgroup, WM x WN waves of 64 lanes, K in tiles of RB
// bytes per row.
template <int PREC, int BM, int BN, int WM, int WN, int STAGES, int RB, int SWZ, int PF, bool ACCUM>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_nt_kernel(const typename Prec<PREC>::in_t *__restrict__ A,
               const typename Prec<PREC>::in_t *__restrict__ Bt,
               typename Prec<PREC>::out_t *__restrict__ C, uint32_t tiles_m, uint32_t tiles_n,
               uint32_t ktiles, uint64_t lda, uint64_t ldb, uint64_t ldc, uint64_t planeA,
               uint64_t planeB, uint64_t c_split_stride, uint64_t batch_a, uint64_t batch_b,
               uint64_t batch_c) {
  using P = Prec<PREC>;
  using in_t = typename P::in_t;
  using acc_t = typename P::acc_t;
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = BM / WM, TN = BN / WN;      // wave tile
  constexpr int FM = TM / 16, FN = TN / 16;      // 16x16 MFMA blocks per wave
  constexpr int PL = P::planes;
  constexpr int BK = RB / P::elem;               // K elements per tile
  constexpr int CPR = RB / 16;                   // 16-byte chunks per row
  constexpr int CH_A = BM * CPR;                 // chunks per A tile plane
  constexpr int CH_B = BN * CPR;
  static_assert(CH_A % NT == 0 && CH_B % NT == 0, "tile/threads mismatch");
  static_assert(RB == 64 || RB == 128, "RB must be 64 or 128");
  constexpr int LA = CH_A / NT, LB = CH_B / NT;  // chunks per thread
  constexpr int STR = lds_stride<RB, SWZ>();
  constexpr int STAGE = (BM + BN) * STR * PL;
  constexpr int NF = RB / 64;                    // 16-byte fragments per lane per block row

  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int g = lane >> 4, r16 = lane & 15;

  uint32_t tm, tn;
  tile_coords(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const uint64_t m0 = uint64_t(tm) * BM, n0 = uint64_t(tn) * BN;

  // batch: blockIdx.z selects a product of the strided batch (elements)
  A += uint64_t(blockIdx.z) * batch_a;
  Bt += uint64_t(blockIdx.z) * batch_b;
  C += uint64_t(blockIdx.z) * batch_c;
  // split-K: blockIdx.y selects a K range of ktiles tiles and its own C slab
  const uint64_t koff = uint64_t(blockIdx.y) * ktiles * BK;
  C += uint64_t(blockIdx.y) * c_split_stride;
  const unsigned char *gA = reinterpret_cast<const unsigned char *>(A + m0 * lda + koff);
  const unsigned char *gB = reinterpret_cast<const unsigned char *>(Bt + n0 * ldb + koff);
  const uint64_t ldaB = lda * P::elem, ldbB = ldb * P::elem;
  const uint64_t plA = planeA * P::elem, plB = planeB * P::elem;

  // PF register sets for the global -> LDS staging: with PF = 2 the loads
  // of tile t are issued two compute phases before tile t is stored to LDS
  static_assert(PF == 1 || (PF == 2 && STAGES == 2), "prefetch distance 2 needs two LDS stages");
  u32x4 ra[PF][PL][LA], rb[PF][PL][LB];

  auto gload = [&](uint32_t kt, int set) {
    const uint64_t kb = uint64_t(kt) * RB;
#pragma unroll
    for (int p = 0; p < PL; ++p) {
#pragma unroll
      for (int i = 0; i < LA; ++i) {
        const int c = tid + i * NT, row = c / CPR, col = c % CPR;
        ra[set][p][i] = *reinterpret_cast<const u32x4 *>(gA + p * plA + row * ldaB + kb + col * 16);
      }
#pragma unroll
      for (int i = 0; i < LB; ++i) {
        const int c = tid + i * NT, row = c / CPR, col = c % CPR;
        rb[set][p][i] = *reinterpret_cast<const u32x4 *>(gB + p * plB + row * ldbB + kb + col * 16);
      }
    }
  };
  auto sstore = [&](int stage, int set) {
    unsigned char *base = smem + stage * STAGE;
#pragma unroll
    for (int p = 0; p < PL; ++p) {
      unsigned char *sA = base + p * (BM + BN) * STR;
      unsigned char *sB = sA + BM * STR;
#pragma unroll
      for (int i = 0; i < LA; ++i) {
        const int c = tid + i * NT, row = c / CPR, col = c % CPR;
        *reinterpret_cast<u32x4 *>(sA + lds_off<RB, SWZ>(row, col)) = ra[set][p][i];
      }
#pragma unroll
      for (int i = 0; i < LB; ++i) {
        const int c = tid + i * NT, row = c / CPR, col = c % CPR;
        *reinterpret_cast<u32x4 *>(sB + lds_off<RB, SWZ>(row, col)) = rb[set][p][i];
      }
    }
  };

  acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{};
  // FP32 and BF16X6 products: the MFMA accumulates one group of K tiles in
  // FP32, the groups are summed in FP64, so the rounding of the sum no longer
  // grows with the full length of K
  constexpr bool F64SUM = PREC == 1 || PREC == 3;
  constexpr uint32_t FLUSH = PREC == 3 ? BF6_FLUSH : F32_FLUSH;
  v4d acc64[F64SUM ? FM : 1][F64SUM ? FN : 1];
  if constexpr (F64SUM) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc64[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  }

  // MFMAs of the tile in LDS stage `cur`, then the FP64 fold of a finished
  // group (K tile kt is the last of its group, or the last one)
  auto compute = [&](int cur, uint32_t kt) {
    const unsigned char *base = smem + cur * STAGE;
    // fragments: lane group g owns chunks [g NF, g NF + NF) of every row
    using frag_t = typename P::frag_t;
    frag_t fa[PL][FM][NF], fb[PL][FN][NF];
#pragma unroll
    for (int p = 0; p < PL; ++p) {
      const unsigned char *sA = base + p * (BM + BN) * STR;
      const unsigned char *sB = sA + BM * STR;
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int f = 0; f < NF; ++f)
          fa[p][i][f] = *reinterpret_cast<const frag_t *>(sA + lds_off<RB, SWZ>(wm * TM + i * 16 + r16, g * NF + f));
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int f = 0; f < NF; ++f)
          fb[p][j][f] = *reinterpret_cast<const frag_t *>(sB + lds_off<RB, SWZ>(wn * TN + j * 16 + r16, g * NF + f));
    }

    if constexpr (PREC == 0) {
#pragma unroll
      for (int s = 0; s < 2 * NF; ++s)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[0][i][s >> 1][s & 1],
                                                              fb[0][j][s >> 1][s & 1], acc[i][j], 0, 0, 0);
    } else if constexpr (PREC == 1) {
#pragma unroll
      for (int s = 0; s < 4 * NF; ++s)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[0][i][s >> 2][s & 3],
                                                              fb[0][j][s >> 2][s & 3], acc[i][j], 0, 0, 0);
    } else if constexpr (PREC == 3) {
      static_assert(NF == 1, "BF16X6 uses one 32-element k-step per K tile");
      // the six products of each block, the small ones first; each term
      // sweeps all accumulators so consecutive MFMAs are independent
      constexpr int TA[6] = {2, 0, 1, 1, 0, 0}, TB[6] = {0, 2, 1, 0, 1, 0};  // lo*hi, hi*lo, mid*mid, mid*hi, hi*mid, hi*hi
#pragma unroll
      for (int term = 0; term < 6; ++term)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[TA[term]][i][0], fb[TB[term]][j][0], acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
      // the three products of a block are spread over all accumulators so
      // that consecutive MFMAs never depend on each other
      for (int s = 0; s < NF; ++s)
#pragma unroll
        for (int term = 0; term < 3; ++term)
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
              const int pa = term == 0 ? 1 : 0, pb = term == 1 ? 1 : 0;  // lo*hi, hi*lo, hi*hi
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[pa][i][s], fb[pb][j][s], acc[i][j], 0, 0, 0);
            }
    }

    if constexpr (F64SUM) {
      if ((kt + 1) % FLUSH == 0 || kt + 1 == ktiles) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) acc64[i][j][e] += double(acc[i][j][e]);
            acc[i][j] = acc_t{};
          }
      }
    }
  };

  if constexpr (PF == 2) {
    // tile t: registers set t % 2, LDS stage t % 2.  Iteration t issues the
    // loads of tile t + 2 into the set that tile t has left, computes stage
    // t % 2, then stores tile t + 1 (loaded during iteration t - 1) into the
    // stage that iteration t - 1 computed; one barrier per tile.  The main
    // loop has no conditional loads or stores, so the wait before a store
    // leaves the six loads issued after it in flight; the last one to three
    // tiles run in a tail with the bounds checks.
    gload(0, 0);
    sstore(0, 0);
    if (ktiles > 1) gload(1, 1);
    __syncthreads();
    auto body = [&](uint32_t kt, auto half) {
      constexpr int h = decltype(half)::value;
      gload(kt + 2, h);
      // keep the loads ahead of the MFMAs: the compiler would otherwise sink
      // them towards their use and shorten the prefetch distance to one tile
      // (the empty asm with a memory clobber stops sinking in the IR, the
      // scheduling barrier reordering in the machine scheduler)
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      compute(h, kt);
      sstore(h ^ 1, h ^ 1);
      __syncthreads();
    };
    auto tail = [&](uint32_t kt, auto half) {
      constexpr int h = decltype(half)::value;
      if (kt + 2 < ktiles) gload(kt + 2, h);
      compute(h, kt);
      if (kt + 1 < ktiles) sstore(h ^ 1, h ^ 1);
      __syncthreads();
    };
    uint32_t kt = 0;
    for (; kt + 3 < ktiles; kt += 2) {
      body(kt, std::integral_constant<int, 0>{});
      body(kt + 1, std::integral_constant<int, 1>{});
    }
    // kt is even here and 1 to 3 tiles remain
    tail(kt, std::integral_constant<int, 0>{});
    if (kt + 1 < ktiles) tail(kt + 1, std::integral_constant<int, 1>{});
    if (kt + 2 < ktiles) tail(kt + 2, std::integral_constant<int, 0>{});
  } else {
    gload(0, 0);
    if constexpr (STAGES == 2) {
      sstore(0, 0);
      __syncthreads();
    }

    for (uint32_t kt = 0; kt < ktiles; ++kt) {
      // two stages: compute stage kt&1 while tile kt+1 is loaded, one barrier;
      // one stage: store, barrier, load the next tile into registers, compute,
      // barrier (two workgroups per CU then overlap each other's waits)
      const int cur = STAGES == 2 ? (kt & 1) : 0;
      if constexpr (STAGES == 1) {
        sstore(0, 0);
        __syncthreads();
      }
      if (kt + 1 < ktiles) gload(kt + 1, 0);
      compute(cur, kt);
      if constexpr (STAGES == 2) {
        if (kt + 1 < ktiles) sstore(cur ^ 1, 0);
      }
      __syncthreads();
    }
  }

  // epilogue: register e of lane (g, r16) holds column r16 of each 16x16
  // block, row 4g + e for the FP32-accumulating instructions and row g + 4e
  // for the FP64 one
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = PREC == 0 ? g + 4 * e : 4 * g + e;
        const uint64_t m = m0 + wm * TM + i * 16 + row;
        const uint64_t n = n0 + wn * TN + j * 16 + r16;
        auto *dst = C + m * ldc + n;
        if constexpr (F64SUM) {
          if constexpr (ACCUM)
            *dst = float(double(*dst) + acc64[i][j][e]);
          else
            *dst = float(acc64[i][j][e]);
        } else {
          if constexpr (ACCUM)
            *dst += acc[i][j][e];
          else
            *dst = acc[i][j][e];
        }
      }
}

template <int PREC, int BM, int BN, int WM, int WN, int STAGES = 2, int RB = 128, int SWZ = 0, int PF = 1>
void launch_gemm(const void *A, const void *Bt, void *C, uint64_t M, uint64_t N, uint64_t K,
                 uint64_t lda, uint64_t ldb, uint64_t ldc, bool accum, hipStream_t st,
                 uint32_t splits = 1, uint64_t c_split_stride = 0, uint32_t nb = 1, uint64_t batch_a = 0,
                 uint64_t batch_b = 0, uint64_t batch_c = 0) {
  using P = Prec<PREC>;
  constexpr int BK = RB / P::elem;
  TRG_REQUIRE(M % BM == 0 && N % BN == 0 && K % BK == 0, "gemm: M, N, K must be tile multiples");
  TRG_REQUIRE(lda >= K && ldb >= K && ldc >= N, "gemm: leading dimension too small");
  TRG_REQUIRE((lda * P::elem) % 16 == 0 && (ldb * P::elem) % 16 == 0, "gemm: rows must be 16-byte aligned");
  if (M == 0 || N == 0) return;
  const uint64_t tiles_m = M / BM, tiles_n = N / BN, tiles = tiles_m * tiles_n;
  TRG_REQUIRE(tiles < (1ull << 31) && K / BK < (1ull << 31), "gemm: problem too large for one launch");
  constexpr size_t lds = STAGES * size_t(BM + BN) * lds_stride<RB, SWZ>() * P::planes;
  static_assert(lds <= 160 * 1024, "LDS tile exceeds 160 KB");
  using in_t = typename P::in_t;
  using out_t = typename P::out_t;
  auto *a = static_cast<const in_t *>(A);
  auto *b = static_cast<const in_t *>(Bt);
  auto *c = static_cast<out_t *>(C);
  const uint64_t plA = M * lda, plB = N * ldb;
  TRG_REQUIRE(nb >= 1 && nb <= 65535, "gemm: batch size out of range");
  TRG_REQUIRE(nb == 1 || (batch_a >= M * lda * P::planes && batch_b >= N * ldb * P::planes && batch_c >= M * ldc),
              "gemm: batch strides overlap the products");
  if (K == 0) {
    if (!accum)
      for (uint32_t b = 0; b < nb; ++b) fill_zero(c + b * batch_c, sizeof(out_t) * M * ldc, st);
    return;
  }
  // K is split into `splits` equal ranges (the caller pads K to a multiple)
  TRG_REQUIRE(splits >= 1 && K % (uint64_t(splits) * BK) == 0, "gemm: K not divisible by splits");
  const uint32_t kt = uint32_t(K / BK / splits);
  dim3 grid(uint32_t(tiles), splits, nb), block(64 * WM * WN);
  // dynamic LDS above 64 KB must be allowed per kernel (once per instantiation)
  static bool attr_set = false;
  if (!attr_set) {
    TRG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(&gemm_nt_kernel<PREC, BM, BN, WM, WN, STAGES, RB, SWZ, PF, true>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    TRG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(&gemm_nt_kernel<PREC, BM, BN, WM, WN, STAGES, RB, SWZ, PF, false>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    attr_set = true;
  }
  if (accum)
    hipLaunchKernelGGL((gemm_nt_kernel<PREC, BM, BN, WM, WN, STAGES, RB, SWZ, PF, true>), grid, block, lds, st, a, b, c,
                       uint32_t(tiles_m), uint32_t(tiles_n), kt, lda, ldb, ldc, plA, plB, c_split_stride, batch_a,
                       batch_b, batch_c);
  else
    hipLaunchKernelGGL((gemm_nt_kernel<PREC, BM, BN, WM, WN, STAGES, RB, SWZ, PF, false>), grid, block, lds, st, a, b, c,
                       uint32_t(tiles_m), uint32_t(tiles_n), kt, lda, ldb, ldc, plA, plB, c_split_stride, batch_a,
                       batch_b, batch_c);
  TRG_HIP_CHECK(hipGetLastError());
}

}  // namespace

// BF16x3 join: 256 x 256 workgroup tile, eight waves of 128 x 64 (two per
// SIMD), 64-byte K rows (32 bf16 per plane), two swizzled LDS stages of
// 64 KB.  Measured against 128 x 128 tiles of four 64 x 64 waves with
// 128-byte rows: 1.6x the MFMA issue rate, 2.5x less L2 -> fabric traffic.
struct BF {
  static constexpr int BM = 256, BN = 256, WM = 2, WN = 4, S = 2, RB = 64, SWZ = 1;
};
// BF16x6 join: 128 x 128 workgroup tile, eight waves of 64 x 32 (two per
// SIMD: 32 FP32 accumulators, 64 FP64 group sums, 18 operand fragments of
// 16 bytes per lane), 64-byte K rows of three planes, swizzled LDS stages of
// 48 KB.  Six products per three planes read from LDS: per MFMA it reads a
// third less LDS than the BF16x3 join's two-plane, three-product blocks.
struct BF6 {
  static constexpr int BM = 128, BN = 128, WM = 2, WN = 4, S = TRG_BF6_STAGES, RB = 64, SWZ = 1, PF = TRG_BF6_PF;
};

GemmTile gemm_tile(int prec) {
  switch (prec) {
    case 0: return {128, 128, 16};
    case 1: return {128, 128, 32};
    case 2: return {BF::BM, BF::BN, BF::RB / 2};
    case 3: return {BF6::BM, BF6::BN, BF6::RB / 2};
  }
  throw Error(-1, "gemm: unknown precision");
}

void gemm_nt(int prec, const void *A, const void *Bt, void *C, uint64_t M, uint64_t N, uint64_t K,
             uint64_t lda, uint64_t ldb, uint64_t ldc, bool accum, hipStream_t st, uint32_t nb, uint64_t batch_a,
             uint64_t batch_b, uint64_t batch_c) {
  switch (prec) {
    case 0:
      launch_gemm<0, 128, 128, 2, 2, TRG_F64_STAGES>(A, Bt, C, M, N, K, lda, ldb, ldc, accum, st, 1, 0, nb, batch_a,
                                                     batch_b, batch_c);
      return;
    case 1:
      launch_gemm<1, 128, 128, 2, TRG_F32_WN, TRG_F32_STAGES>(A, Bt, C, M, N, K, lda, ldb, ldc, accum, st, 1, 0, nb,
                                                              batch_a, batch_b, batch_c);
      return;
    case 2:
      launch_gemm<2, BF::BM, BF::BN, BF::WM, BF::WN, BF::S, BF::RB, BF::SWZ>(A, Bt, C, M, N, K, lda, ldb, ldc, accum, st,
                                                                            1, 0, nb, batch_a, batch_b, batch_c);
      return;
    case 3:
      launch_gemm<3, BF6::BM, BF6::BN, BF6::WM, BF6::WN, BF6::S, BF6::RB, BF6::SWZ, BF6::PF>(
          A, Bt, C, M, N, K, lda, ldb, ldc, accum, st, 1, 0, nb, batch_a, batch_b, batch_c);
      return;
  }
  throw Error(-1, "gemm: unknown precision");
}

// Split-K FP64 products of the Gram reductions: 64 x 64 tiles (four 32 x 32
// waves); split s covers K range [s*kper, (s+1)*kper) and writes its own
// M x N slab of Cpart.  K must equal splits * kper (zero-padded).
void gemm_nt_splitk_f64(const double *A, const double *Bt, double *Cpart, uint64_t M, uint64_t N,
                        uint64_t K, uint64_t lda, uint64_t ldb, uint32_t splits, uint64_t kper,
                        hipStream_t st) {
  TRG_REQUIRE(K == uint64_t(splits) * kper, "splitk: K != splits * kper");
  launch_gemm<0, 64, 64, 2, 2>(A, Bt, Cpart, M, N, K, lda, ldb, N, false, st, splits, M * N);
}

}  // namespace trg
