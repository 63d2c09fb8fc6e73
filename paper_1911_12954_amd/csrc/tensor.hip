// Memory-bound tensor kernels of the HOTRG step: leg contractions with an
// isometry (operand construction and post-join compression), strided copies,
// padding, Frobenius normalisation, periodic traces and the initial Ising
// tensors.
#include <cmath>
#include <cstdlib>
#include <vector>

#include "internal.h"

namespace trg {
namespace {

// ------------------------------------------------------------- tensor map ---
// One thread per index of the thread dims; it keeps the NI outputs that
// differ only in the inner dim (a dim the input does not have, only the
// matrix: a leg that the contraction produces) in registers, so every input
// element it sums is loaded once for all of them.
constexpr int MAP_MAXI = 16;
struct MapParams {
  int ndims, nsum;
  FastDiv div[MAP_MAXD];
  int64_t so[MAP_MAXD], si[MAP_MAXD], su[MAP_MAXD];
  int32_t ssize[2];
  int64_t ssi[2], ssu[2];
  int32_t ni;           // inner dim size (1 = none)
  int64_t iso, isu;     // its output and matrix strides
  uint32_t count;
  int64_t lo_plane;
  int32_t u_lds;        // > 0: the matrix entries [0, u_lds) are staged in LDS
};
// largest matrix (doubles) a map workgroup stages in LDS
constexpr int MAP_ULDS_MAX = 6144;

template <int OUT>
__device__ inline void map_store(void *out, int64_t o, int64_t lo_plane, double v) {
  if constexpr (OUT == OUT_F64) {
    static_cast<double *>(out)[o] = v;
  } else if constexpr (OUT == OUT_F32) {
    static_cast<float *>(out)[o] = float(v);
  } else if constexpr (OUT == OUT_BF16X2) {
    // v = hi + lo with hi = bf16(fl32(v)), lo = bf16(fl32(v) - hi)
    const float a = float(v);
    const uint16_t hi = f32_to_bf16_rne(a);
    const uint16_t lo = f32_to_bf16_rne(a - bf16_to_f32(hi));
    static_cast<uint16_t *>(out)[o] = hi;
    static_cast<uint16_t *>(out)[o + lo_plane] = lo;
  } else {
    // fl32(v) = hi + mid + lo exactly: each residual is exact in FP32
    // (Sterbenz) and the last one has at most 8 significant bits
    const float a = float(v);
    const uint16_t hi = f32_to_bf16_rne(a);
    const float r1 = a - bf16_to_f32(hi);
    const uint16_t mid = f32_to_bf16_rne(r1);
    const uint16_t lo = f32_to_bf16_rne(r1 - bf16_to_f32(mid));
    static_cast<uint16_t *>(out)[o] = hi;
    static_cast<uint16_t *>(out)[o + lo_plane] = mid;
    static_cast<uint16_t *>(out)[o + 2 * lo_plane] = lo;
  }
}

// per-context pointers of a batched map (grid.y = context)
struct MapPtrs {
  const void *in[TRG_MAXB];
  const double *U[TRG_MAXB];
  void *out[TRG_MAXB];
};

template <typename InT, int OUT>
__global__ void __launch_bounds__(256)
map_kernel(MapPtrs ptrs, MapParams p) {
  extern __shared__ double Us[];
  const InT *__restrict__ in = static_cast<const InT *>(ptrs.in[blockIdx.y]);
  const double *__restrict__ Ug = ptrs.U[blockIdx.y];
  void *__restrict__ out = ptrs.out[blockIdx.y];
  const double *U = Ug;
  if (p.u_lds > 0) {
    // every thread of the block reaches this barrier (the bound check follows)
    for (int i = threadIdx.x; i < p.u_lds; i += 256) Us[i] = Ug[i];
    __syncthreads();
    U = Us;
  }
  const uint32_t idx = blockIdx.x * 256u + threadIdx.x;
  if (idx >= p.count) return;
  uint32_t q = idx;
  int64_t oo = 0, oi = 0, ou = 0;
#pragma unroll
  for (int j = MAP_MAXD - 1; j >= 0; --j) {
    if (j < p.ndims) {
      const uint32_t qd = fast_div(q, p.div[j]);
      const uint32_t r = q - qd * p.div[j].d;
      q = qd;
      oo += int64_t(r) * p.so[j];
      oi += int64_t(r) * p.si[j];
      ou += int64_t(r) * p.su[j];
    }
  }
  if (p.ni > 1) {
    // inner dim in registers; the same summation order as below per output
    double acc[MAP_MAXI];
#pragma unroll
    for (int k = 0; k < MAP_MAXI; ++k) acc[k] = 0.0;
    if (p.nsum == 0) {
      const double x = double(in[oi]);
#pragma unroll
      for (int k = 0; k < MAP_MAXI; ++k)
        if (k < p.ni) acc[k] = x * U[ou + k * p.isu];
    } else if (p.nsum == 1) {
      for (int a = 0; a < p.ssize[0]; ++a) {
        const double x = double(in[oi + a * p.ssi[0]]);
        const double *pu = U + ou + a * p.ssu[0];
#pragma unroll
        for (int k = 0; k < MAP_MAXI; ++k)
          if (k < p.ni) acc[k] += x * pu[k * p.isu];
      }
    } else {
      for (int a = 0; a < p.ssize[0]; ++a)
        for (int b = 0; b < p.ssize[1]; ++b) {
          const double x = double(in[oi + a * p.ssi[0] + b * p.ssi[1]]);
          const double *pu = U + ou + a * p.ssu[0] + b * p.ssu[1];
#pragma unroll
          for (int k = 0; k < MAP_MAXI; ++k)
            if (k < p.ni) acc[k] += x * pu[k * p.isu];
        }
    }
#pragma unroll
    for (int k = 0; k < MAP_MAXI; ++k)
      if (k < p.ni) map_store<OUT>(out, oo + k * p.iso, p.lo_plane, acc[k]);
    return;
  }
  double acc;
  if (p.nsum == 0) {
    acc = U ? double(in[oi]) * U[ou] : double(in[oi]);
  } else if (p.nsum == 1) {
    acc = 0.0;
    for (int a = 0; a < p.ssize[0]; ++a) acc += double(in[oi + a * p.ssi[0]]) * U[ou + a * p.ssu[0]];
  } else {
    acc = 0.0;
    for (int a = 0; a < p.ssize[0]; ++a) {
      const InT *pi = in + oi + a * p.ssi[0];
      const double *pu = U + ou + a * p.ssu[0];
      for (int b = 0; b < p.ssize[1]; ++b) acc += double(pi[b * p.ssi[1]]) * pu[b * p.ssu[1]];
    }
  }
  map_store<OUT>(out, oo, p.lo_plane, acc);
}

template <typename InT>
void launch_map(const MapPtrs &ptrs, int nb, int out_kind, MapParams &p, hipStream_t st) {
  const dim3 grid((p.count + 255) / 256, nb), block(256);
  const size_t lds = p.u_lds > 0 ? size_t(p.u_lds) * 8 : 0;
  switch (out_kind) {
    case OUT_F64: hipLaunchKernelGGL((map_kernel<InT, OUT_F64>), grid, block, lds, st, ptrs, p); break;
    case OUT_F32: hipLaunchKernelGGL((map_kernel<InT, OUT_F32>), grid, block, lds, st, ptrs, p); break;
    case OUT_BF16X2: hipLaunchKernelGGL((map_kernel<InT, OUT_BF16X2>), grid, block, lds, st, ptrs, p); break;
    case OUT_BF16X3: hipLaunchKernelGGL((map_kernel<InT, OUT_BF16X3>), grid, block, lds, st, ptrs, p); break;
    default: throw Error(-1, "tensor_map: bad output kind");
  }
  TRG_HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------------ padding ---
// Elem: an unsigned integer type of the element size, so that every store
// clears one whole element.
template <typename Elem>
__global__ void zero_pad_kernel(Elem *buf, int64_t rows, int64_t rows_pad, int64_t cols, int64_t ld, int planes,
                                int64_t plane_stride, int64_t batch_stride) {
  // grid.y = context (batch_stride elements apart); grid-stride over
  // (plane, row) pairs; each row clears [cols, ld) or all of it
  buf += int64_t(blockIdx.y) * batch_stride;
  const int64_t total = int64_t(planes) * rows_pad;
  for (int64_t rr = blockIdx.x; rr < total; rr += gridDim.x) {
    const int64_t plane = rr / rows_pad, row = rr % rows_pad;
    Elem *base = buf + plane * plane_stride + row * ld;
    const int64_t c0 = row < rows ? cols : 0;
    for (int64_t c = c0 + threadIdx.x; c < ld; c += blockDim.x) base[c] = Elem(0);
  }
}

__global__ void fill_zero_kernel(uint32_t *buf, size_t words) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < words; i += size_t(gridDim.x) * blockDim.x)
    buf[i] = 0u;
}

// ------------------------------------------------------------ reductions ---
__global__ void reduce_splits_kernel(const double *part, int splits, int64_t rows, int64_t cols,
                                     int64_t ldp, int64_t sstride, double *out, int64_t ldo) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int64_t r = i / cols, c = i % cols;
  double s = 0.0;
  for (int k = 0; k < splits; ++k) s += part[k * sstride + r * ldp + c];
  out[r * ldo + c] = s;
}

// The same sum with eight threads per output: thread (o, g) of a 32 x 8
// workgroup adds the splits k = g (mod 8) in increasing k, and the eight
// partial sums are added in a fixed tree, so the result is deterministic;
// 32 consecutive outputs read 256 contiguous bytes of a split.  For few
// outputs and many splits (the slabs of a tall-skinny Gram).
constexpr int RS_OUT = 32, RS_GROUPS = 8;

__global__ void __launch_bounds__(RS_OUT * RS_GROUPS)
reduce_splits_grouped_kernel(const double *part, int splits, int64_t rows, int64_t cols, int64_t ldp,
                             int64_t sstride, double *out, int64_t ldo) {
  __shared__ double sh[RS_GROUPS][RS_OUT];
  const int o = threadIdx.x % RS_OUT, g = threadIdx.x / RS_OUT;
  const int64_t i = int64_t(blockIdx.x) * RS_OUT + o;
  double s = 0.0;
  if (i < rows * cols) {
    const int64_t r = i / cols, c = i % cols;
    const double *p = part + r * ldp + c;
    for (int k = g; k < splits; k += RS_GROUPS) s += p[int64_t(k) * sstride];
  }
  sh[g][o] = s;
  __syncthreads();
  if (g == 0 && i < rows * cols) {
    const double t = ((sh[0][o] + sh[1][o]) + (sh[2][o] + sh[3][o])) + ((sh[4][o] + sh[5][o]) + (sh[6][o] + sh[7][o]));
    const int64_t r = i / cols, c = i % cols;
    out[r * ldo + c] = t;
  }
}

__global__ void gram_combine_kernel(const double *P, const double *Q, int dmu, int dn, double *G) {
  // G[(a,b),(a2,b2)] = sum_{i,i2} P[(i,a),(i2,a2)] Q[(i,b),(i2,b2)]
  const int n = dn * dn;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n) * n) return;
  const int row = int(t / n), col = int(t % n);
  const int a = row / dn, b = row % dn, a2 = col / dn, b2 = col % dn;
  const int R = dmu * dn;
  double s = 0.0;
  for (int i = 0; i < dmu; ++i)
    for (int i2 = 0; i2 < dmu; ++i2)
      s += P[(i * dn + a) * R + i2 * dn + a2] * Q[(i * dn + b) * R + i2 * dn + b2];
  G[t] = s;
}

constexpr int NORM_BLOCKS = 1024;

__device__ inline double block_sum(double v, double *sh) {
  // deterministic tree over 256 threads
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  return sh[0];
}

__global__ void __launch_bounds__(256) sumsq_kernel(NormBatch nbt, int64_t n, double *partial) {
  __shared__ double sh[256];
  // grid.y = context; its partial sums follow those of the contexts before it
  const double *x = nbt.x[blockIdx.y];
  partial += size_t(blockIdx.y) * gridDim.x;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t b = int64_t(blockIdx.x) * per;
  const int64_t e = b + per < n ? b + per : n;
  double s = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) s += x[i] * x[i];
  const double tot = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256)
norm_final_kernel(NormBatch nbt, const double *partial, int nb) {
  __shared__ double sh[256];
  // one workgroup per context, each with its own accumulator weight
  partial += size_t(blockIdx.x) * nb;
  const double weight = nbt.weight[blockIdx.x];
  double *scal = nbt.scal[blockIdx.x];
  double *acc = scal + 3;
  int *err = nbt.err[blockIdx.x];
  double *rec = nbt.rec[blockIdx.x];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += partial[i];
  const double tot = block_sum(s, sh);
  if (threadIdx.x == 0) {
    const double c = sqrt(tot);
    const bool ok = c > 0.0 && isfinite(c);
    scal[0] = c;
    scal[1] = ok ? 1.0 / c : 0.0;
    scal[2] = ok ? log(c) : 0.0;
    if (rec) rec[0] = scal[2];
    if (ok) acc[0] += weight * log(c);
    else *err |= 1;
  }
}

struct ScalePtrs {
  double *x[TRG_MAXB];
  const double *scal[TRG_MAXB];
};

__global__ void scale_kernel(ScalePtrs sp, int64_t n, double factor) {
  // grid.y = context
  double *x = sp.x[blockIdx.y];
  const double f = factor * sp.scal[blockIdx.y][1];
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    x[i] *= f;
}

struct TraceParams {
  const double *X[3];
  int count, d;
  int dims[4];
  int64_t diag_stride[4];
};

__global__ void __launch_bounds__(256) trace_kernel(TraceParams p, double *out) {
  __shared__ double sh[256];
  int64_t total = 1;
  for (int a = 0; a < p.d; ++a) total *= p.dims[a];
  for (int j = 0; j < p.count; ++j) {
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < total; t += 256) {
      int64_t q = t, off = 0;
      for (int a = p.d - 1; a >= 0; --a) {
        off += (q % p.dims[a]) * p.diag_stride[a];
        q /= p.dims[a];
      }
      s += p.X[j][off];
    }
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) out[j] = tot;
    __syncthreads();
  }
}

// Initial tensors from the closed form: n = number of legs at index 1,
// T0 = 2 c^a s^b g(bh), S_M = 2 c^a s^b g'(bh),
// S_E = 2 c^a s^b [(a tanh b + b coth b) g(bh) + h g'(bh)],
// c = cosh beta, s = sinh beta, a = (2d - n)/2, b = n/2, g = cosh (n even)
// or sinh (n odd), g' the other one.
__global__ void ising_kernel(double *T, double *SE, double *SM, int d, double beta, double h) {
  const int nl = 2 * d;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (1 << nl)) return;
  const int n = __popc(idx);
  const double a = 0.5 * (nl - n), b = 0.5 * n;
  const double ch = cosh(beta), sh = sinh(beta);
  const double base = 2.0 * pow(ch, a) * (n ? pow(sh, b) : 1.0);
  const bool even = (n & 1) == 0;
  const double g = even ? cosh(beta * h) : sinh(beta * h);
  const double gp = even ? sinh(beta * h) : cosh(beta * h);
  // leg l of the row-major index is bit (nl-1-l) of idx; the closed form
  // depends only on the count n, so the bit order does not matter
  if (T) T[idx] = base * g;
  if (SM) SM[idx] = base * gp;
  if (SE) {
    const double dlog = (n ? b / tanh(beta) : 0.0) + a * tanh(beta);
    SE[idx] = base * (dlog * g + h * gp);
  }
}

}  // namespace

// ------------------------------------------------------------- host side ---
void tensor_map(const void *in, int in_kind, const double *U, void *out, int out_kind,
                int64_t lo_plane, const MapDim *dims, int ndims, const MapSum *sums, int nsum,
                hipStream_t st) {
  tensor_map_batch(&in, in_kind, &U, &out, 1, out_kind, lo_plane, dims, ndims, sums, nsum, st);
}

void tensor_map_batch(const void *const *ins, int in_kind, const double *const *Us, void *const *outs, int nb,
                      int out_kind, int64_t lo_plane, const MapDim *dims, int ndims, const MapSum *sums,
                      int nsum, hipStream_t st) {
  TRG_REQUIRE(nb >= 1 && nb <= TRG_MAXB, "tensor_map: batch size out of range");
  TRG_REQUIRE(ndims >= 1 && ndims <= MAP_MAXD && nsum >= 0 && nsum <= 2, "tensor_map: bad rank");
  const double *U = Us[0];
  for (int b = 0; b < nb; ++b)
    TRG_REQUIRE((Us[b] != nullptr) == (U != nullptr), "tensor_map: every context needs a matrix or none");
  TRG_REQUIRE(nsum == 0 || U != nullptr, "tensor_map: summation needs a matrix");
  for (int i = 0; i < ndims; ++i)
    TRG_REQUIRE(dims[i].size >= 1 && dims[i].size < (int64_t(1) << 31), "tensor_map: bad dim");
  // inner dim: a matrix-only dim (absent from the input) of 2..MAP_MAXI
  // values, the one with the largest output stride
  int in_dim = -1;
  if (U)
    for (int i = 0; i < ndims; ++i)
      if (dims[i].si == 0 && dims[i].su != 0 && dims[i].size >= 2 && dims[i].size <= MAP_MAXI &&
          (in_dim < 0 || std::llabs(dims[i].so) > std::llabs(dims[in_dim].so)))
        in_dim = i;
  const MapDim idim = in_dim >= 0 ? dims[in_dim] : MapDim{1, 0, 0, 0};
  MapDim tdims[MAP_MAXD];
  int nt = 0;
  for (int i = 0; i < ndims; ++i)
    if (i != in_dim) tdims[nt++] = dims[i];
  if (nt == 0) tdims[nt++] = MapDim{1, 0, 0, 0};
  dims = tdims;
  ndims = nt;
  int64_t total = 1;
  for (int i = 0; i < ndims; ++i) total *= dims[i].size;
  // split the outermost dims into separate launches until a launch has < 2^32 - 256 elements
  int outer = 0;
  int64_t inner = total;
  while (inner >= (int64_t(1) << 32) - 256) {
    TRG_REQUIRE(outer + 1 < ndims, "tensor_map: cannot split launch");
    inner /= dims[outer].size;
    ++outer;
  }
  int64_t nouter = total / inner;
  MapParams p{};
  p.ndims = ndims - outer;
  p.nsum = nsum;
  for (int i = 0; i < p.ndims; ++i) {
    const MapDim &m = dims[outer + i];
    p.div[i] = make_fastdiv(uint32_t(m.size));
    p.so[i] = m.so;
    p.si[i] = m.si;
    p.su[i] = m.su;
  }
  for (int j = 0; j < nsum; ++j) {
    p.ssize[j] = int32_t(sums[j].size);
    p.ssi[j] = sums[j].si;
    p.ssu[j] = sums[j].su;
  }
  p.count = uint32_t(inner);
  p.lo_plane = lo_plane;
  p.ni = int32_t(idim.size);
  p.iso = idim.so;
  p.isu = idim.su;
  // matrix entries one launch can touch, from its base: stage them in LDS
  // when the register-held inner dim multiplies the matrix reads
  p.u_lds = 0;
  if (U && p.ni > 1) {
    bool nonneg = idim.su >= 0;
    int64_t span = 1 + (idim.size - 1) * idim.su;
    for (int i = outer; i < ndims; ++i) {
      nonneg = nonneg && dims[i].su >= 0;
      span += (dims[i].size - 1) * dims[i].su;
    }
    for (int j = 0; j < nsum; ++j) {
      nonneg = nonneg && sums[j].su >= 0;
      span += (sums[j].size - 1) * sums[j].su;
    }
    if (nonneg && span <= MAP_ULDS_MAX) p.u_lds = int32_t(span);
  }
  const int esz_in = in_kind == IN_F64 ? 8 : 4;
  const int esz_out = out_kind == OUT_F64 ? 8 : (out_kind == OUT_F32 ? 4 : 2);
  for (int64_t o = 0; o < nouter; ++o) {
    // offsets of this outer multi-index
    int64_t q = o, oo = 0, oi = 0, ou = 0;
    for (int i = outer - 1; i >= 0; --i) {
      const int64_t r = q % dims[i].size;
      q /= dims[i].size;
      oo += r * dims[i].so;
      oi += r * dims[i].si;
      ou += r * dims[i].su;
    }
    MapPtrs ptrs{};
    for (int b = 0; b < nb; ++b) {
      ptrs.in[b] = static_cast<const char *>(ins[b]) + oi * esz_in;
      ptrs.U[b] = Us[b] ? Us[b] + ou : nullptr;
      ptrs.out[b] = static_cast<char *>(outs[b]) + oo * esz_out;
    }
    if (in_kind == IN_F64)
      launch_map<double>(ptrs, nb, out_kind, p, st);
    else
      launch_map<float>(ptrs, nb, out_kind, p, st);
  }
}

void zero_pad(void *buf, int64_t rows, int64_t rows_pad, int64_t cols, int64_t ld, int elem_bytes,
              int planes, int64_t plane_stride, hipStream_t st, int nb, int64_t batch_stride) {
  if (cols == ld && rows == rows_pad) return;
  TRG_REQUIRE(nb >= 1 && nb <= 65535, "zero_pad: batch size out of range");
  const int64_t work = int64_t(planes) * rows_pad;
  const dim3 grid(uint32_t(work < 65536 ? work : 65536), uint32_t(nb));
  switch (elem_bytes) {
    case 2:
      hipLaunchKernelGGL(zero_pad_kernel<uint16_t>, grid, dim3(256), 0, st, static_cast<uint16_t *>(buf), rows,
                         rows_pad, cols, ld, planes, plane_stride, batch_stride);
      break;
    case 4:
      hipLaunchKernelGGL(zero_pad_kernel<uint32_t>, grid, dim3(256), 0, st, static_cast<uint32_t *>(buf), rows,
                         rows_pad, cols, ld, planes, plane_stride, batch_stride);
      break;
    case 8:
      hipLaunchKernelGGL(zero_pad_kernel<uint64_t>, grid, dim3(256), 0, st, static_cast<uint64_t *>(buf), rows,
                         rows_pad, cols, ld, planes, plane_stride, batch_stride);
      break;
    default:
      throw Error(-1, "zero_pad: element size must be 2, 4 or 8 bytes");
  }
  TRG_HIP_CHECK(hipGetLastError());
}

void fill_zero(void *buf, size_t bytes, hipStream_t st) {
  TRG_REQUIRE(bytes % 4 == 0, "fill_zero: size must be a multiple of 4");
  const size_t words = bytes / 4;
  if (!words) return;
  const size_t blocks = (words + 255) / 256;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(uint32_t(blocks < 65536 ? blocks : 65536)), dim3(256), 0, st,
                     static_cast<uint32_t *>(buf), words);
  TRG_HIP_CHECK(hipGetLastError());
}

void reduce_splits(const double *part, int splits, int64_t rows, int64_t cols, int64_t ldp,
                   int64_t split_stride, double *out, int64_t ldo, hipStream_t st) {
  const int64_t n = rows * cols;
  if (splits >= 2 * RS_GROUPS && n < int64_t(256) * 1024) {
    hipLaunchKernelGGL(reduce_splits_grouped_kernel, dim3(uint32_t((n + RS_OUT - 1) / RS_OUT)),
                       dim3(RS_OUT * RS_GROUPS), 0, st, part, splits, rows, cols, ldp, split_stride, out, ldo);
  } else {
    hipLaunchKernelGGL(reduce_splits_kernel, dim3(uint32_t((n + 255) / 256)), dim3(256), 0, st, part, splits,
                       rows, cols, ldp, split_stride, out, ldo);
  }
  TRG_HIP_CHECK(hipGetLastError());
}

void gram_combine(const double *P, const double *Q, int dmu, int dn, double *G, hipStream_t st) {
  const int64_t n2 = int64_t(dn) * dn * dn * dn;
  hipLaunchKernelGGL(gram_combine_kernel, dim3(uint32_t((n2 + 255) / 256)), dim3(256), 0, st, P, Q, dmu, dn, G);
  TRG_HIP_CHECK(hipGetLastError());
}

int norm_blocks() { return NORM_BLOCKS; }

void norm_and_accumulate(const double *x, int64_t n, double *partial, int nblocks, double *scal,
                         double *acc, double weight, int *err, hipStream_t st) {
  TRG_REQUIRE(acc == scal + 3, "norm: the accumulator is scal[3]");
  NormBatch b{};
  b.x[0] = x;
  b.scal[0] = scal;
  b.err[0] = err;
  b.rec[0] = nullptr;
  b.weight[0] = weight;
  norm_and_accumulate_batch(b, 1, n, partial, nblocks, st);
}

void norm_and_accumulate_batch(const NormBatch &b, int nb, int64_t n, double *partial, int nblocks,
                               hipStream_t st) {
  TRG_REQUIRE(nb >= 1 && nb <= TRG_MAXB, "norm: batch size out of range");
  hipLaunchKernelGGL(sumsq_kernel, dim3(nblocks, nb), dim3(256), 0, st, b, n, partial);
  TRG_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(norm_final_kernel, dim3(nb), dim3(256), 0, st, b, partial, nblocks);
  TRG_HIP_CHECK(hipGetLastError());
}

void scale_by_inverse(double *x, int64_t n, const double *scal, double factor, hipStream_t st) {
  scale_by_inverse_batch(&x, &scal, 1, n, factor, st);
}

void scale_by_inverse_batch(double *const *xs, const double *const *scals, int nb, int64_t n, double factor,
                            hipStream_t st) {
  TRG_REQUIRE(nb >= 1 && nb <= TRG_MAXB, "scale: batch size out of range");
  ScalePtrs sp{};
  for (int b = 0; b < nb; ++b) {
    sp.x[b] = xs[b];
    sp.scal[b] = scals[b];
  }
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(scale_kernel, dim3(uint32_t(blocks < 16384 ? blocks : 16384), nb), dim3(256), 0, st, sp, n,
                     factor);
  TRG_HIP_CHECK(hipGetLastError());
}

void periodic_traces(const double *const *X, int count, const int *dims, int d, double *out,
                     hipStream_t st) {
  TRG_REQUIRE(count >= 1 && count <= 3 && d >= 1 && d <= 4, "trace: bad arguments");
  TraceParams p{};
  p.count = count;
  p.d = d;
  for (int j = 0; j < count; ++j) p.X[j] = X[j];
  // row-major strides of the 2d legs
  int64_t stride[8];
  int64_t s = 1;
  for (int l = 2 * d - 1; l >= 0; --l) {
    stride[l] = s;
    s *= dims[l / 2];
  }
  for (int a = 0; a < d; ++a) {
    p.dims[a] = dims[a];
    p.diag_stride[a] = stride[2 * a] + stride[2 * a + 1];
  }
  hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(256), 0, st, p, out);
  TRG_HIP_CHECK(hipGetLastError());
}

namespace {

// Degeneracy indicator: M[a][a'] = T with the legs of `axis` open and every
// other axis' pair traced (one workgroup per entry, fixed reduction tree),
// then out = {Tr M, Tr(M M)} from one workgroup.
struct IndicatorParams {
  int n;                  // dims[axis]
  int64_t s0, s1;         // strides of the backward / forward leg of axis
  int nother;
  int odims[3];
  int64_t odiag[3];       // stride of the diagonal of each other axis
};

__global__ void __launch_bounds__(256) indicator_matrix_kernel(const double *T, IndicatorParams p, double *M) {
  __shared__ double sh[256];
  const int a = blockIdx.x / p.n, a2 = blockIdx.x % p.n;
  int64_t total = 1;
  for (int b = 0; b < p.nother; ++b) total *= p.odims[b];
  const double *base = T + int64_t(a) * p.s0 + int64_t(a2) * p.s1;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < total; i += 256) {
    int64_t q = i, off = 0;
    for (int b = p.nother - 1; b >= 0; --b) {
      off += (q % p.odims[b]) * p.odiag[b];
      q /= p.odims[b];
    }
    s += base[off];
  }
  const double r = block_sum(s, sh);
  if (threadIdx.x == 0) M[blockIdx.x] = r;
}

__global__ void __launch_bounds__(256) indicator_reduce_kernel(const double *M, int n, double *out) {
  __shared__ double sh[256];
  double tr = 0.0, tr2 = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) tr += M[i * n + i];
  for (int64_t ij = threadIdx.x; ij < int64_t(n) * n; ij += 256) {
    const int i = int(ij / n), j = int(ij % n);
    tr2 += M[i * n + j] * M[j * n + i];
  }
  const double a = block_sum(tr, sh);
  __syncthreads();
  const double b = block_sum(tr2, sh);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

}  // namespace

void indicator_traces(const double *T, const int *dims, int d, int axis, double *M, double *out, hipStream_t st) {
  TRG_REQUIRE(d >= 1 && d <= 4 && axis >= 0 && axis < d, "indicator: bad arguments");
  int64_t stride[8];
  int64_t s = 1;
  for (int l = 2 * d - 1; l >= 0; --l) {
    stride[l] = s;
    s *= dims[l / 2];
  }
  IndicatorParams p{};
  p.n = dims[axis];
  p.s0 = stride[2 * axis];
  p.s1 = stride[2 * axis + 1];
  for (int b = 0; b < d; ++b) {
    if (b == axis) continue;
    p.odims[p.nother] = dims[b];
    p.odiag[p.nother] = stride[2 * b] + stride[2 * b + 1];
    ++p.nother;
  }
  const int64_t nn = int64_t(p.n) * p.n;
  TRG_REQUIRE(nn < (int64_t(1) << 31), "indicator: leg too large");
  hipLaunchKernelGGL(indicator_matrix_kernel, dim3(uint32_t(nn)), dim3(256), 0, st, T, p, M);
  TRG_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(indicator_reduce_kernel, dim3(1), dim3(256), 0, st, M, p.n, out);
  TRG_HIP_CHECK(hipGetLastError());
}

void indicator_reduce(const double *M, int n, double *out, hipStream_t st) {
  hipLaunchKernelGGL(indicator_reduce_kernel, dim3(1), dim3(256), 0, st, M, n, out);
  TRG_HIP_CHECK(hipGetLastError());
}

void ising_init(double *T, double *SE, double *SM, int d, double beta, double h, hipStream_t st) {
  const int n = 1 << (2 * d);
  hipLaunchKernelGGL(ising_kernel, dim3((n + 255) / 256), dim3(256), 0, st, T, SE, SM, d, beta, h);
  TRG_HIP_CHECK(hipGetLastError());
}

}  // namespace trg
