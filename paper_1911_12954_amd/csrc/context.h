// Context of libtrg and host-side helpers shared by the HOTRG and ATRG engines.
#pragma once

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/trg.h"
#include "internal.h"

namespace trg {

struct Leg {
  std::string name;
  int64_t size, stride;
};
using View = std::vector<Leg>;

inline const Leg &find_leg(const View &v, const std::string &n) {
  for (const auto &l : v)
    if (l.name == n) return l;
  throw Error(-1, "internal: leg " + n + " not found");
}
inline bool has_leg(const View &v, const std::string &n) {
  for (const auto &l : v)
    if (l.name == n) return true;
  return false;
}

// row-major contiguous layout of the named legs (first = outermost)
inline View contiguous(const std::vector<std::pair<std::string, int64_t>> &legs, int64_t scale = 1) {
  View v;
  int64_t s = scale;
  for (int i = int(legs.size()) - 1; i >= 0; --i) {
    v.insert(v.begin(), Leg{legs[i].first, legs[i].second, s});
    s *= legs[i].second;
  }
  return v;
}

inline int64_t view_count(const View &v) {
  int64_t n = 1;
  for (const auto &l : v) n *= l.size;
  return n;
}

inline View rename(View v, const std::map<std::string, std::string> &m) {
  for (auto &l : v) {
    auto it = m.find(l.name);
    if (it != m.end()) l.name = it->second;
  }
  return v;
}

// out(legs of outv) = sum over `sums` of in(legs of inv) * U(u legs)
// u_strides gives the U stride of every U-side leg name (outputs and sums).
void apply_map(const void *in, int in_kind, const View &inv, const double *U,
               const std::map<std::string, int64_t> &u_strides, const std::vector<std::string> &sums,
               void *out, int out_kind, int64_t lo_plane, const View &outv, hipStream_t st);
// the same map for nb contexts in one launch (context i: ins[i], Us[i], outs[i])
void apply_map_batch(const void *const *ins, int in_kind, const View &inv, const double *const *Us,
                     const std::map<std::string, int64_t> &u_strides, const std::vector<std::string> &sums,
                     void *const *outs, int nb, int out_kind, int64_t lo_plane, const View &outv, hipStream_t st);

inline std::string nm(const char *p, int ax) { return std::string(p) + std::to_string(ax); }

struct Buffer {
  void *ptr = nullptr;
  size_t cap = 0;
};

}  // namespace trg

using trg::Buffer;
using trg::Error;

// Named scratch buffers of one or more contexts; freed with the allocator of
// the context that created the pool when the last user lets go of it.
struct WorkspacePool {
  std::map<std::string, Buffer> bufs;
  void (*free_fn)(void *, void *) = nullptr;
  void *user = nullptr;
  bool use_alloc = false;
  explicit WorkspacePool(const trg_config &cfg) : free_fn(cfg.free), user(cfg.alloc_user), use_alloc(cfg.alloc != nullptr) {}
  ~WorkspacePool() {
    for (auto &kv : bufs) {
      if (!kv.second.ptr) continue;
      if (use_alloc) {
        if (free_fn) free_fn(kv.second.ptr, user);
      } else {
        (void)hipFree(kv.second.ptr);
      }
    }
  }
};

struct trg_ctx {
  int d = 0;
  int dims[4] = {0, 0, 0, 0};
  int nsteps = 0;
  trg_config cfg{};
  hipStream_t st = nullptr;
  bool poisoned = false;
  std::string err;
  int nimp = 0;        // number of impure tensors
  int imp_kind[2] = {-1, -1};  // 0 = E, 1 = M
  bool has_e = false, has_m = false;

  Buffer T, Tn, S[2], Sn[2];
  Buffer dev_scalars;  // doubles: [0] c [1] 1/c [2] ln c [3] acc [4..6] traces [7] c0
  Buffer dev_err;      // int
  Buffer dev_rec;      // per-step device records
  int rec_cap = 0;
  std::vector<trg_step_rec> host_rec;  // host-known parts
  Buffer U[4], spec[4];
  int Un[4] = {0, 0, 0, 0}, Uk[4] = {0, 0, 0, 0};
  // join/scratch workspace; contexts stepped one after another on the same
  // stream may share one (trg_share_workspace)
  std::shared_ptr<WorkspacePool> pool;
  int force_side = -1;

  // ATRG: T = sum_l G[b, l] H[l, f] (G: n x r, H: r x n), last swap spectrum
  Buffer G, H, atrg_sigma;
  int imp_r[2] = {0, 0};  // ATRG: bond of impurity j's pieces S[j] (G_S) and Sn[j] (H_S)
  int r = 0;
  int atrg_nsig = 0;
  // ATRG Z2 mode: parity (0 even, 1 odd) of every leg index of each axis and
  // of every bond index; host staging of the parity tables a step uploads
  // (kept here so that they outlive the asynchronous copies)
  bool z2 = false;
  std::vector<int8_t> z2_legs[4], z2_bond;
  std::vector<int> z2_stage[4];

  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> join_events;
  double join_ms = 0.0, join_flops_done = 0.0, join_flops_pending = 0.0;
  long long join_launches = 0;

  void *alloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (cfg.alloc) {
      p = cfg.alloc(bytes, cfg.alloc_user);
      if (!p) throw Error(TRG_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        throw Error(TRG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
      }
    }
    return p;
  }
  void release(void *p) {
    if (!p) return;
    if (cfg.alloc) {
      if (cfg.free) cfg.free(p, cfg.alloc_user);
    } else {
      (void)hipFree(p);
    }
  }
  void ensure(Buffer &b, size_t bytes) {
    if (b.cap >= bytes && b.ptr) return;
    if (b.ptr) {
      // the stream may still read the old buffer: hipFree needs the wait, a
      // custom allocator is stream-ordered on st by contract
      if (!cfg.alloc) TRG_HIP_CHECK(hipStreamSynchronize(st));
      release(b.ptr);
      b.ptr = nullptr;
      b.cap = 0;
    }
    b.ptr = alloc(bytes);
    b.cap = bytes;
  }
  template <typename Tp>
  Tp *wsp(const std::string &name, size_t bytes) {
    if (!pool) pool = std::make_shared<WorkspacePool>(cfg);
    Buffer &b = pool->bufs[name];
    ensure(b, bytes);
    return static_cast<Tp *>(b.ptr);
  }
  size_t ws_held() const {
    size_t s = 0;
    if (pool)
      for (const auto &kv : pool->bufs) s += kv.second.cap;
    return s;
  }
  double *scal() { return static_cast<double *>(dev_scalars.ptr); }
  int *errp() { return static_cast<int *>(dev_err.ptr); }
  int64_t total() const {
    int64_t n = 1;
    for (int a = 0; a < d; ++a) n *= int64_t(dims[a]) * dims[a];
    return n;
  }
};

namespace trg {

// ATRG state and shared engine helpers (engine.hip / atrg.hip)
void atrg_init_ising(trg_ctx &c, double beta, double h);
void atrg_step_impl(trg_ctx &c, int mu, int dcut);
double atrg_trace(trg_ctx &c);
// Tr S_j = sum G_S[b, m] H_S[m, b] of ATRG impurity j (synchronises)
double atrg_impurity_trace(trg_ctx &c, int j);
// {Tr M, Tr(M M)} into out for M[x][x'] = sum_{l, other legs traced} G[.., x, .., l] H[l, .., x', ..]
void atrg_indicator_traces(trg_ctx &c, int axis, double *M, double *out);
void sync_check(trg_ctx &c);
double *rec_d(trg_ctx &c, int n);
int *rec_i(trg_ctx &c, int n);
void ensure_records(trg_ctx &c, int need);

// precision of the next HOTRG join: FP64 for the first cfg.fp64_steps steps
inline int join_precision(const trg_ctx &c) {
  return c.nsteps < c.cfg.fp64_steps ? int(TRG_FP64) : c.cfg.precision;
}

// arithmetic of the contraction that produced the current tensor: FP64 for
// the initial (or imported, or host-given) tensor of step 0 and for the steps
// joined in FP64, else the configured precision (HOTRG join or ATRG
// contraction GEMMs)
inline int producer_precision(const trg_ctx &c) {
  if (c.nsteps == 0) return TRG_FP64;
  if (c.cfg.method == TRG_ATRG) return c.cfg.precision == TRG_FP32 ? int(TRG_FP32) : int(TRG_FP64);
  return c.nsteps - 1 < c.cfg.fp64_steps ? int(TRG_FP64) : c.cfg.precision;
}

// C(out_names, contiguous) = sum over the legs shared by A and B of A * B,
// through packed, padded operands and the MFMA GEMM (prec FP64 or FP32).
void einsum2(trg_ctx &c, const double *A, const View &va, const double *B, const View &vb, double *C,
             const std::vector<std::string> &out_names, int prec, const std::string &tag);

}  // namespace trg
