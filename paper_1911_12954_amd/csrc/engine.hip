// HOTRG step engine and the C-ABI of libtrg.
//
// One step along axis mu (Sec. 2 and Fig. 1 of the paper):
//   1. Gram matrices of the two-site tensor for every transverse axis nu and
//      both leg pairs (backward, forward) from the one-site environments P
//      and Q (split-K FP64 MFMA products) and their FP64 combination.
//   2. Jacobi eigendecomposition on the device, truncation to k_nu =
//      min(d_nu^2, Dcut), side choice and canonical basis: the isometry U_nu.
//   3. The block-spin contraction: operands A (site 1, its backward pairs
//      along the first transverse axes compressed) and Bt (site 2, forward
//      pairs compressed) are built in the join precision, the join E = A Bt^T
//      runs on MFMA, and the remaining transverse pairs are compressed from E
//      into the new tensor.  Large steps are sliced over the outer legs x0
//      (of A) and x2 (of Bt) to fit the workspace.
//   4. Frobenius normalisation c_n and acc += 2^{-n} ln c_n in FP64; impure
//      tensors S' = [C(S,T) + C(T,S)] / (2 c_n) with the same isometries.
// All of it is enqueued on the context's stream; no host synchronisation.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "context.h"

using namespace trg;

namespace {

thread_local std::string g_thread_error;

}  // namespace

namespace trg {

void apply_map(const void *in, int in_kind, const View &inv, const double *U,
               const std::map<std::string, int64_t> &u_strides, const std::vector<std::string> &sums,
               void *out, int out_kind, int64_t lo_plane, const View &outv, hipStream_t st) {
  apply_map_batch(&in, in_kind, inv, &U, u_strides, sums, &out, 1, out_kind, lo_plane, outv, st);
}

void apply_map_batch(const void *const *ins, int in_kind, const View &inv, const double *const *Us,
                     const std::map<std::string, int64_t> &u_strides, const std::vector<std::string> &sums,
                     void *const *outs, int nb, int out_kind, int64_t lo_plane, const View &outv, hipStream_t st) {
  std::vector<MapDim> dims;
  for (const auto &o : outv) {
    MapDim m{o.size, o.stride, 0, 0};
    if (has_leg(inv, o.name)) m.si = find_leg(inv, o.name).stride;
    auto it = u_strides.find(o.name);
    if (it != u_strides.end()) m.su = it->second;
    if (!has_leg(inv, o.name) && it == u_strides.end())
      throw Error(-1, "internal: output leg " + o.name + " has no source");
    dims.push_back(m);
  }
  std::vector<MapSum> ss;
  for (const auto &n : sums) {
    const Leg &l = find_leg(inv, n);
    auto it = u_strides.find(n);
    if (it == u_strides.end()) throw Error(-1, "internal: summed leg without U stride");
    ss.push_back(MapSum{l.size, l.stride, it->second});
  }
  tensor_map_batch(ins, in_kind, Us, outs, nb, out_kind, lo_plane, dims.data(), int(dims.size()), ss.data(),
                   int(ss.size()), st);
}

}  // namespace trg

namespace trg {

// device step record layout (doubles first, then ints)
constexpr int REC_D = 1 + 8;        // ln c, eps[4][2]
constexpr int REC_I = 4 * 4;        // per axis: side, k, degenerate, sweeps
constexpr size_t REC_BYTES = REC_D * 8 + REC_I * 4;

double *rec_d(trg_ctx &c, int n) {
  return reinterpret_cast<double *>(static_cast<char *>(c.dev_rec.ptr) + size_t(n) * REC_BYTES);
}
int *rec_i(trg_ctx &c, int n) {
  return reinterpret_cast<int *>(static_cast<char *>(c.dev_rec.ptr) + size_t(n) * REC_BYTES + REC_D * 8);
}

void ensure_records(trg_ctx &c, int need) {
  if (need <= c.rec_cap) return;
  int cap = c.rec_cap ? c.rec_cap : 64;
  while (cap < need) cap *= 2;
  void *p = c.alloc(size_t(cap) * REC_BYTES);
  fill_zero(p, size_t(cap) * REC_BYTES, c.st);
  if (c.dev_rec.ptr) {
    TRG_HIP_CHECK(hipMemcpyAsync(p, c.dev_rec.ptr, size_t(c.rec_cap) * REC_BYTES, hipMemcpyDeviceToDevice, c.st));
    if (!c.cfg.alloc) TRG_HIP_CHECK(hipStreamSynchronize(c.st));
    c.release(c.dev_rec.ptr);
  }
  c.dev_rec.ptr = p;
  c.dev_rec.cap = size_t(cap) * REC_BYTES;
  c.rec_cap = cap;
}

std::vector<int64_t> canon_strides(const int *dims, int d) {
  std::vector<int64_t> s(2 * d);
  int64_t x = 1;
  for (int l = 2 * d - 1; l >= 0; --l) {
    s[l] = x;
    x *= dims[l / 2];
  }
  return s;
}

// ---------------------------------------------------------------- Grams ---
// Environment of one site keeping legs l1 (rows major) and l2: X[(l1,l2)][rest]
// then X X^T by split-K MFMA.  Result R x R (R = dim(l1) dim(l2)) in out.
void environment(trg_ctx &c, const double *T, int l1, int l2, double *out, const std::string &tag) {
  const int d = c.d;
  auto st_ = canon_strides(c.dims, d);
  const int64_t n1 = c.dims[l1 / 2], n2 = c.dims[l2 / 2];
  const int64_t R = n1 * n2, C = c.total() / R;
  const int64_t Rp = int64_t(round_up(R, 64));
  const int64_t tiles = (Rp / 64) * (Rp / 64);
  int64_t splits = (1024 + tiles - 1) / tiles;
  const int64_t kt = (C + 15) / 16;
  if (splits > kt) splits = kt;
  if (splits < 1) splits = 1;
  const int64_t kper = int64_t(round_up((C + splits - 1) / splits, 16));
  const int64_t Cp = kper * splits;
  double *X = c.wsp<double>("gram_X" + tag, size_t(Rp) * Cp * 8);
  double *part = c.wsp<double>("gram_part" + tag, size_t(splits) * Rp * Rp * 8);
  // X rows (l1, l2), columns: the other legs in canonical order
  View inv;
  for (int l = 0; l < 2 * d; ++l) inv.push_back(Leg{"l" + std::to_string(l), c.dims[l / 2], st_[l]});
  std::vector<std::pair<std::string, int64_t>> cols;
  for (int l = 0; l < 2 * d; ++l)
    if (l != l1 && l != l2) cols.push_back({"l" + std::to_string(l), c.dims[l / 2]});
  View outv = contiguous(cols);
  outv.insert(outv.begin(), Leg{"l" + std::to_string(l2), n2, Cp});
  outv.insert(outv.begin(), Leg{"l" + std::to_string(l1), n1, n2 * Cp});
  apply_map(T, IN_F64, inv, nullptr, {}, {}, X, OUT_F64, 0, outv, c.st);
  zero_pad(X, R, Rp, C, Cp, 8, 1, 0, c.st);
  gemm_nt_splitk_f64(X, X, part, uint64_t(Rp), uint64_t(Rp), uint64_t(Cp), uint64_t(Cp), uint64_t(Cp),
                     uint32_t(splits), uint64_t(kper), c.st);
  reduce_splits(part, int(splits), R, R, Rp, Rp * Rp, out, R, c.st);
}

// ------------------------------------------------------------ operands ---
// target GEMM rows of one join launch (x0 slices of A)
constexpr int64_t JOIN_ROWS = 32768;

struct StepShape {
  int mu;
  std::vector<int> others, pre, post;
  int nd[4];
  int64_t Mr, Kdim, Kpad;
  int prec;
};

// Operand of site 1 (A) or site 2 (Bt) for outer-leg values [o0, o0 + cnt):
// rows (outer, pair legs of post axes, compressed pre legs), columns
// (i, b_s..., a'_s...).  Written with row stride Kpad, rows padded to Mpad,
// in the join precision.  For the nb contexts of a batch at once: context b
// reads Xs[b] with its own isometries and writes out + b * out_slot bytes
// (temporaries in slots of tmp_slot bytes); every kernel is one launch.
void build_operand(std::vector<trg_ctx *> &cs, const StepShape &sh, const double *const *Xs, bool site1, int o0,
                   int cnt, char *out, size_t out_slot, int64_t Mpad, const std::string &tmp_tag) {
  trg_ctx &c = *cs[0];
  const int nb = int(cs.size());
  const int d = c.d, mu = sh.mu;
  auto st_ = canon_strides(c.dims, d);
  // view of X with names of the roles it plays
  View v;
  for (int ax = 0; ax < d; ++ax) {
    if (ax == mu) {
      if (site1) {
        v.push_back(Leg{"o", cnt, st_[2 * ax]});
        v.push_back(Leg{"i", c.dims[ax], st_[2 * ax + 1]});
      } else {
        v.push_back(Leg{"i", c.dims[ax], st_[2 * ax]});
        v.push_back(Leg{"o", cnt, st_[2 * ax + 1]});
      }
    } else {
      v.push_back(Leg{nm(site1 ? "a" : "b", ax), c.dims[ax], st_[2 * ax]});
      v.push_back(Leg{nm(site1 ? "ap" : "bp", ax), c.dims[ax], st_[2 * ax + 1]});
    }
  }
  std::vector<const void *> cur(nb);
  for (int b = 0; b < nb; ++b) cur[b] = Xs[b] + int64_t(o0) * (site1 ? st_[2 * mu] : st_[2 * mu + 1]);
  // final layout
  std::vector<std::pair<std::string, int64_t>> rows{{"o", cnt}}, cols{{"i", c.dims[mu]}};
  for (int r : sh.post) {
    rows.push_back({nm(site1 ? "a" : "b", r), c.dims[r]});
    rows.push_back({nm(site1 ? "ap" : "bp", r), c.dims[r]});
  }
  for (int s : sh.pre) rows.push_back({nm(site1 ? "K" : "L", s), sh.nd[s]});
  for (int s : sh.pre) cols.push_back({nm("b", s), c.dims[s]});
  for (int s : sh.pre) cols.push_back({nm("ap", s), c.dims[s]});
  View colv = contiguous(cols);
  View rowv = contiguous(rows, sh.Kpad);
  View finalv = rowv;
  finalv.insert(finalv.end(), colv.begin(), colv.end());
  const int64_t M = view_count(rowv);

  const int out_kind = sh.prec == TRG_FP64   ? OUT_F64
                       : sh.prec == TRG_FP32 ? OUT_F32
                       : sh.prec == TRG_BF16X3 ? OUT_BF16X2
                                               : OUT_BF16X3;
  const int esz = sh.prec == TRG_FP64 ? 8 : (sh.prec == TRG_FP32 ? 4 : 2);
  const int64_t lo_plane = Mpad * sh.Kpad;
  std::vector<void *> outs(nb);
  for (int b = 0; b < nb; ++b) outs[b] = out + size_t(b) * out_slot;

  View curv = v;
  for (size_t j = 0; j < sh.pre.size(); ++j) {
    const int s = sh.pre[j];
    const int64_t ds = c.dims[s], ks = sh.nd[s];
    // site 1 sums its backward leg a_s against U[a, b, K]; site 2 sums its
    // forward leg b'_s against U[a', b', L]
    std::map<std::string, int64_t> us;
    std::string summed;
    std::vector<std::pair<std::string, int64_t>> produced;
    if (site1) {
      summed = nm("a", s);
      us = {{summed, ds * ks}, {nm("b", s), ks}, {nm("K", s), 1}};
      produced = {{nm("b", s), ds}, {nm("K", s), ks}};
    } else {
      summed = nm("bp", s);
      us = {{nm("ap", s), ds * ks}, {summed, ks}, {nm("L", s), 1}};
      produced = {{nm("ap", s), ds}, {nm("L", s), ks}};
    }
    const bool last = j + 1 == sh.pre.size();
    std::vector<const double *> Us(nb);
    for (int b = 0; b < nb; ++b) Us[b] = static_cast<const double *>(cs[b]->U[s].ptr);
    if (last) {
      apply_map_batch(cur.data(), IN_F64, curv, Us.data(), us, {summed}, outs.data(), nb, out_kind, lo_plane, finalv,
                      c.st);
    } else {
      std::vector<std::pair<std::string, int64_t>> legs;
      for (const auto &l : curv) {
        if (l.name == summed) {
          for (auto &p : produced) legs.push_back(p);
        } else {
          legs.push_back({l.name, l.size});
        }
      }
      View tv = contiguous(legs);
      const size_t slot = size_t(view_count(tv)) * 8;
      char *tmp = c.wsp<char>("op_tmp" + tmp_tag, slot * nb);
      std::vector<void *> tmps(nb);
      for (int b = 0; b < nb; ++b) tmps[b] = tmp + size_t(b) * slot;
      apply_map_batch(cur.data(), IN_F64, curv, Us.data(), us, {summed}, tmps.data(), nb, OUT_F64, 0, tv, c.st);
      for (int b = 0; b < nb; ++b) cur[b] = tmps[b];
      curv = tv;
    }
  }
  zero_pad(out, M, Mpad, sh.Kdim, sh.Kpad, esz, operand_planes(sh.prec), lo_plane, c.st, nb,
           int64_t(out_slot / esz));
}

// Compress the post-axis pairs of a join block E (rows x0-block, cols
// x2-block) and write the new tensor's slab T'[x0a.., x2a..]: context b of
// the batch reads E + b * e_slot bytes and writes Touts[b].
void post_join(std::vector<trg_ctx *> &cs, const StepShape &sh, const char *E, size_t e_slot, int64_t ldc, int x0a,
               int c0, int x2a, int c2, double *const *Touts) {
  trg_ctx &c = *cs[0];
  const int nb = int(cs.size());
  const int d = c.d, mu = sh.mu;
  const int in_kind = sh.prec == TRG_FP64 ? IN_F64 : IN_F32;
  std::vector<std::pair<std::string, int64_t>> rows{{"o1", c0}}, cols{{"o2", c2}};
  for (int r : sh.post) {
    rows.push_back({nm("a", r), c.dims[r]});
    rows.push_back({nm("ap", r), c.dims[r]});
    cols.push_back({nm("b", r), c.dims[r]});
    cols.push_back({nm("bp", r), c.dims[r]});
  }
  for (int s : sh.pre) rows.push_back({nm("K", s), sh.nd[s]});
  for (int s : sh.pre) cols.push_back({nm("L", s), sh.nd[s]});
  View ev = contiguous(rows, ldc);
  View evc = contiguous(cols);
  ev.insert(ev.end(), evc.begin(), evc.end());
  // output: canonical layout of the new dims, offset to the slab
  auto nst = canon_strides(sh.nd, d);
  View outv;
  for (int ax = 0; ax < d; ++ax) {
    if (ax == mu) {
      outv.push_back(Leg{"o1", c0, nst[2 * ax]});
      outv.push_back(Leg{"o2", c2, nst[2 * ax + 1]});
    } else {
      outv.push_back(Leg{nm("K", ax), sh.nd[ax], nst[2 * ax]});
      outv.push_back(Leg{nm("L", ax), sh.nd[ax], nst[2 * ax + 1]});
    }
  }
  std::vector<const void *> ins(nb);
  std::vector<void *> dsts(nb);
  for (int b = 0; b < nb; ++b) {
    ins[b] = E + size_t(b) * e_slot;
    dsts[b] = Touts[b] + int64_t(x0a) * nst[2 * mu] + int64_t(x2a) * nst[2 * mu + 1];
  }
  if (sh.post.empty()) {
    std::vector<const double *> none(nb, nullptr);
    apply_map_batch(ins.data(), in_kind, ev, none.data(), {}, {}, dsts.data(), nb, OUT_F64, 0, outv, c.st);
    return;
  }
  if (sh.post.size() != 1) throw Error(-1, "internal: more than one post axis");
  const int r = sh.post[0];
  const int64_t dr = c.dims[r], kr = sh.nd[r];
  std::vector<const double *> Us(nb);
  for (int b = 0; b < nb; ++b) Us[b] = static_cast<const double *>(cs[b]->U[r].ptr);
  // (a_r, b_r) -> K_r into a contiguous temporary
  std::vector<std::pair<std::string, int64_t>> tl;
  for (const auto &l : ev)
    if (l.name != nm("a", r) && l.name != nm("b", r)) tl.push_back({l.name, l.size});
  tl.push_back({nm("K", r), kr});
  View tv = contiguous(tl);
  const size_t slot = size_t(view_count(tv)) * 8;
  char *tmp = c.wsp<char>("post_tmp", slot * nb);
  std::vector<void *> tmps(nb);
  std::vector<const void *> tmpin(nb);
  for (int b = 0; b < nb; ++b) {
    tmps[b] = tmp + size_t(b) * slot;
    tmpin[b] = tmps[b];
  }
  apply_map_batch(ins.data(), in_kind, ev, Us.data(), {{nm("a", r), dr * kr}, {nm("b", r), kr}, {nm("K", r), 1}},
                  {nm("a", r), nm("b", r)}, tmps.data(), nb, OUT_F64, 0, tv, c.st);
  // (a'_r, b'_r) -> L_r into the new tensor
  apply_map_batch(tmpin.data(), IN_F64, tv, Us.data(), {{nm("ap", r), dr * kr}, {nm("bp", r), kr}, {nm("L", r), 1}},
                  {nm("ap", r), nm("bp", r)}, dsts.data(), nb, OUT_F64, 0, outv, c.st);
}

void record_join(trg_ctx &c, hipEvent_t &a, hipEvent_t &b, bool begin) {
  if (!c.profiling) return;
  if (begin) {
    TRG_HIP_CHECK(hipEventCreate(&a));
    TRG_HIP_CHECK(hipEventCreate(&b));
    TRG_HIP_CHECK(hipEventRecord(a, c.st));
  } else {
    TRG_HIP_CHECK(hipEventRecord(b, c.st));
    c.join_events.push_back({a, b});
  }
}

// The join of nb contexts in one launch: product b reads A + b * a_slot and
// Bt + b * b_slot and writes E + b * e_slot (bytes).  A batched launch is
// timed and counted on the batch's first context.
void join(trg_ctx &c, int prec, const char *A, size_t a_slot, const char *Bt, size_t b_slot, char *E, size_t e_slot,
          int nb, int64_t Mpad, int64_t Npad, int64_t Kpad, bool accum) {
  hipEvent_t a{}, b{};
  record_join(c, a, b, true);
  const int ein = prec == TRG_FP64 ? 8 : (prec == TRG_FP32 ? 4 : 2);   // bytes of one element of one plane
  const int eout = prec == TRG_FP64 ? 8 : 4;
  gemm_nt(prec, A, Bt, E, uint64_t(Mpad), uint64_t(Npad), uint64_t(Kpad), uint64_t(Kpad), uint64_t(Kpad),
          uint64_t(Npad), accum, c.st, uint32_t(nb), a_slot / ein, b_slot / ein, e_slot / eout);
  record_join(c, a, b, false);
  c.join_launches += 1;
  c.join_flops_pending += 2.0 * double(Mpad) * double(Npad) * double(Kpad) * nb;
  // With TRG_PROGRESS set in the environment, wait for each join and report
  // it on stderr: a long step (minutes at Dcut 12 in FP64) then shows its
  // progress launch by launch.  Off by default (one cached getenv).
  static const bool progress = std::getenv("TRG_PROGRESS") != nullptr;
  if (progress) {
    TRG_HIP_CHECK(hipStreamSynchronize(c.st));
    std::fprintf(stderr, "[trg] join %lld done: %lld x %lld x %lld, %d product(s)\n",
                 static_cast<long long>(c.join_launches), static_cast<long long>(Mpad),
                 static_cast<long long>(Npad), static_cast<long long>(Kpad), nb);
    std::fflush(stderr);
  }
}

struct StepPrep {
  StepShape sh;
  int n_step;
  double *rd;
  int *ri;
};

StepPrep prepare_step(trg_ctx &c, int mu, int dcut) {
  const int d = c.d;
  StepPrep p;
  StepShape &sh = p.sh;
  sh.mu = mu;
  sh.prec = join_precision(c);
  for (int ax = 0; ax < d; ++ax)
    if (ax != mu) sh.others.push_back(ax);
  const size_t npre = (sh.others.size() + 1) / 2;
  for (size_t j = 0; j < sh.others.size(); ++j) (j < npre ? sh.pre : sh.post).push_back(sh.others[j]);
  for (int ax = 0; ax < d; ++ax) {
    const int64_t sq = int64_t(c.dims[ax]) * c.dims[ax];
    sh.nd[ax] = ax == mu ? c.dims[ax] : int(sq < dcut ? sq : dcut);
  }
  p.n_step = c.nsteps + 1;
  ensure_records(c, p.n_step + 1);
  p.rd = rec_d(c, p.n_step);
  p.ri = rec_i(c, p.n_step);
  return p;
}
// Gram matrices of every context into one buffer, one batched Jacobi launch
// for all of them, then each context's isometry selection.  Every matrix is
// processed by its own workgroup, so a batch gives the same bits as single
// contexts.
void isometries_batch(std::vector<trg_ctx *> &cs, std::vector<StepPrep> &ps, int mu) {
  trg_ctx &c0 = *cs[0];
  const int nc = int(cs.size());
  const std::vector<int> &others = ps[0].sh.others;
  const int nax = int(others.size());
  // every transverse axis first; axes of one order share one launch
  int nmax = 0;
  bool same_n = true;
  for (int ax : others) {
    nmax = std::max(nmax, c0.dims[ax] * c0.dims[ax]);
    same_n = same_n && c0.dims[ax] == c0.dims[others[0]];
  }
  const size_t per_ax = size_t(nc) * 2;  // matrices per axis
  double *G = c0.wsp<double>("gram_G", per_ax * nax * nmax * nmax * 8);
  double *W = c0.wsp<double>("gram_W", per_ax * nax * nmax * 8);
  double *V = c0.wsp<double>("gram_V", per_ax * nax * nmax * nmax * 8);
  int *sw = c0.wsp<int>("gram_sweeps", per_ax * nax * 4);
  // axis slot a holds per_ax matrices of order n_a, consecutive (stride
  // n_a^2, n_a for eigenvalues) from offset a * per_ax * nmax^2 (nmax); when
  // every order agrees the slots are contiguous: one batch of nax * per_ax
  const size_t slot_n = size_t(nmax);   // = every n_a when same_n
  auto gbase = [&](int a) { return size_t(a) * per_ax * slot_n * slot_n; };
  auto wbase = [&](int a) { return size_t(a) * per_ax * slot_n; };
  for (int a = 0; a < nax; ++a) {
    const int ax = others[a];
    const int dn = c0.dims[ax];
    const int n = dn * dn;
    const size_t ms = size_t(n) * n;   // matrix stride inside the slot
    const int dmu = c0.dims[mu];
    const int64_t R = int64_t(dmu) * dn;
    for (int i = 0; i < nc; ++i) {
      trg_ctx &c = *cs[i];
      double *PQ = c.wsp<double>("gram_PQ", size_t(2) * R * R * 8);
      const double *T = static_cast<const double *>(c.T.ptr);
      for (int side = 0; side < 2; ++side) {
        environment(c, T, 2 * mu + 1, 2 * ax + side, PQ, "");
        environment(c, T, 2 * mu, 2 * ax + side, PQ + R * R, "");
        gram_combine(PQ, PQ + R * R, dmu, dn, G + gbase(a) + (size_t(i) * 2 + side) * ms, c.st);
      }
    }
  }
  // every eigenvalue, and the eigenvectors of the kept columns plus a
  // cluster the cut splits (the widest window and most columns over the
  // batch, so that each context's selection finds what it reads)
  double rel = 0.0;
  std::vector<int> kmax(size_t(nax), 1);
  for (int i = 0; i < nc; ++i) {
    rel = std::max(rel, degeneracy_window(producer_precision(*cs[i])));
    for (int a = 0; a < nax; ++a) kmax[size_t(a)] = std::max(kmax[size_t(a)], ps[i].sh.nd[others[a]]);
  }
  if (same_n) {
    const int n = c0.dims[others[0]] * c0.dims[others[0]];
    const int kk = *std::max_element(kmax.begin(), kmax.end());
    double *work = n > JACOBI_MAX_N ? c0.wsp<double>("gram_top", eigh_top_work_doubles(n, int(per_ax) * nax) * 8)
                                    : nullptr;
    eigh_top_batched(G, W, V, sw, n, int(per_ax) * nax, kk, rel, work, c0.st);
  } else {
    for (int a = 0; a < nax; ++a) {
      const int n = c0.dims[others[a]] * c0.dims[others[a]];
      double *work = n > JACOBI_MAX_N ? c0.wsp<double>("gram_top" + std::to_string(a),
                                                       eigh_top_work_doubles(n, int(per_ax)) * 8)
                                      : nullptr;
      eigh_top_batched(G + gbase(a), W + wbase(a), V + gbase(a), sw + size_t(a) * per_ax, n, int(per_ax),
                       kmax[size_t(a)], rel, work, c0.st);
    }
  }
  for (int a = 0; a < nax; ++a) {
    const int ax = others[a];
    const int n = c0.dims[ax] * c0.dims[ax];
    for (int i = 0; i < nc; ++i) {
      trg_ctx &c = *cs[i];
      const int k = ps[i].sh.nd[ax];
      c.ensure(c.U[ax], size_t(n) * k * 8);
      c.ensure(c.spec[ax], size_t(n) * 8);
      c.Un[ax] = n;
      c.Uk[ax] = k;
      const size_t m = size_t(i) * 2;   // matrix index inside the slot
      SelectOut so{static_cast<double *>(c.U[ax].ptr), ps[i].rd + 1 + 2 * ax, ps[i].ri + 4 * ax,
                   static_cast<double *>(c.spec[ax].ptr)};
      select_isometry(W + wbase(a) + m * n, V + gbase(a) + m * n * n, sw + size_t(a) * per_ax + m, n, k,
                      c.force_side, degeneracy_window(producer_precision(c)), so, c.st);
    }
  }
}

// Block-spin contraction, normalisation and bookkeeping of one step for
// contexts of equal shape (d, dims, join precision, impurities), every kernel
// launched once for up to TRG_MAXB of them: the join plan (x0 slices of A,
// x2 slices of Bt) is that of one context, and the batch is cut into chunks
// whose join workspaces fit the budget together.  Context b of a chunk uses
// slot b of each operand buffer; the results do not depend on the chunking.
void contract_batch(std::vector<trg_ctx *> all, std::vector<StepPrep *> preps, int mu) {
  trg_ctx &c = *all[0];
  const int d = c.d;
  // the contexts share the shape of the step, not its number: each keeps its
  // own step count (accumulator weight 2^-n, records)
  StepShape &sh = preps[0]->sh;
  // ---- 3: block-spin contraction, sliced over x0 (A) and x2 (Bt)
  const GemmTile tile = gemm_tile(sh.prec);
  sh.Mr = 1;
  for (int r : sh.post) sh.Mr *= int64_t(c.dims[r]) * c.dims[r];
  for (int s : sh.pre) sh.Mr *= sh.nd[s];
  sh.Kdim = c.dims[mu];
  for (int s : sh.pre) sh.Kdim *= int64_t(c.dims[s]) * c.dims[s];
  sh.Kpad = int64_t(round_up(sh.Kdim, tile.k));
  for (auto *p : preps) {
    p->sh.Mr = sh.Mr;
    p->sh.Kdim = sh.Kdim;
    p->sh.Kpad = sh.Kpad;
  }
  const int esz = operand_bytes(sh.prec);  // per element, all planes
  const int esE = sh.prec == TRG_FP64 ? 8 : 4;
  const int nt = 1 + c.nimp;
  const int dmu = c.dims[mu];
  const int64_t total_old = c.total();
  int64_t ks1 = sh.pre.empty() ? 1 : sh.nd[sh.pre[0]];
  auto bytes_for = [&](int c0, int c2) {
    const double Mp = double(round_up(size_t(c0) * sh.Mr, tile.m));
    const double Np = double(round_up(size_t(c2) * sh.Mr, tile.n));
    double b = nt * (Mp + Np) * double(sh.Kpad) * esz;
    b += double(c0 > c2 ? c0 : c2) * double(total_old / dmu) * double(ks1) * 8.0;  // operand temp
    b += Mp * Np * esE;                                                             // E
    double e1 = double(c0) * c2;
    for (int r : sh.post) e1 *= double(c.dims[r]) * c.dims[r] * sh.nd[r];
    for (int s : sh.pre) e1 *= double(sh.nd[s]) * sh.nd[s];
    if (!sh.post.empty()) b += e1 * 8.0;
    return b;
  };
  // budget of the batch: every context brings its cfg.workspace_bytes (the
  // batched launches hold one slot per context); without a cap on some
  // context, 85 % of the free device memory
  double budget = 0.0;
  bool capped = true;
  for (auto *x : all) {
    capped = capped && x->cfg.workspace_bytes > 0;
    budget += double(x->cfg.workspace_bytes);
  }
  if (!capped) {
    size_t fr = 0, tot = 0;
    TRG_HIP_CHECK(hipMemGetInfo(&fr, &tot));
    budget = 0.85 * double(fr + c.ws_held()) - 2.0e9;
  }
  // natural plan, sized to one context's share: Bt whole, A in slices of
  // about JOIN_ROWS GEMM rows; the memory budget can only shrink it (the
  // slicing does not change any result)
  const double share = budget / double(all.size());
  int c2 = dmu;
  while (c2 > 1 && bytes_for(1, c2) > share) --c2;
  if (bytes_for(1, c2) > share) throw Error(TRG_ENOMEM, "join workspace does not fit the memory budget");
  const int c0_max = int(std::max<int64_t>(1, std::min<int64_t>(dmu, JOIN_ROWS / sh.Mr)));
  int c0 = 1;
  while (c0 < c0_max && bytes_for(c0 + 1, c2) <= share) ++c0;
  // contexts per launch
  const int fit = int(std::max(1.0, std::floor(budget / bytes_for(c0, c2))));
  const int chunk = std::min({fit, TRG_MAXB, int(all.size())});

  const int64_t cap_tensor = [&] {
    int64_t n = 1;
    for (int ax = 0; ax < d; ++ax) n *= int64_t(sh.nd[ax]) * sh.nd[ax];
    return n;
  }();
  const size_t a_slot = round_up(size_t(c0) * sh.Mr, tile.m) * size_t(sh.Kpad) * esz;
  const size_t b_slot = round_up(size_t(c2) * sh.Mr, tile.n) * size_t(sh.Kpad) * esz;
  const size_t e_slot = round_up(size_t(c0) * sh.Mr, tile.m) * round_up(size_t(c2) * sh.Mr, tile.n) * esE;

  for (size_t first = 0; first < all.size(); first += chunk) {
    std::vector<trg_ctx *> cs(all.begin() + first, all.begin() + std::min(all.size(), first + chunk));
    const int nb = int(cs.size());
    for (auto *x : cs) {
      x->ensure(x->Tn, size_t(cap_tensor) * 8);
      for (int j = 0; j < x->nimp; ++j) x->ensure(x->Sn[j], size_t(cap_tensor) * 8);
    }
    // sources and destinations per tensor kind t (pure, impurities) and context
    std::vector<std::vector<const double *>> src(nt, std::vector<const double *>(nb));
    std::vector<std::vector<double *>> dst(nt, std::vector<double *>(nb));
    for (int b = 0; b < nb; ++b) {
      src[0][b] = static_cast<const double *>(cs[b]->T.ptr);
      dst[0][b] = static_cast<double *>(cs[b]->Tn.ptr);
      for (int j = 0; j < c.nimp; ++j) {
        src[1 + j][b] = static_cast<const double *>(cs[b]->S[j].ptr);
        dst[1 + j][b] = static_cast<double *>(cs[b]->Sn[j].ptr);
      }
    }
    for (int x2a = 0; x2a < dmu; x2a += c2) {
      const int n2 = (dmu - x2a) < c2 ? (dmu - x2a) : c2;
      const int64_t Npad = int64_t(round_up(size_t(n2) * sh.Mr, tile.n));
      char *Bt[3];
      for (int t = 0; t < nt; ++t) {
        Bt[t] = c.wsp<char>("Bt" + std::to_string(t), b_slot * nb);
        build_operand(cs, sh, src[t].data(), false, x2a, n2, Bt[t], b_slot, Npad, "B");
      }
      for (int x0a = 0; x0a < dmu; x0a += c0) {
        const int n0 = (dmu - x0a) < c0 ? (dmu - x0a) : c0;
        const int64_t Mpad = int64_t(round_up(size_t(n0) * sh.Mr, tile.m));
        char *A[3];
        for (int t = 0; t < nt; ++t) {
          A[t] = c.wsp<char>("A" + std::to_string(t), a_slot * nb);
          build_operand(cs, sh, src[t].data(), true, x0a, n0, A[t], a_slot, Mpad, "A");
        }
        char *E = c.wsp<char>("E", e_slot * nb);
        // pure: E = A_T Bt_T
        join(c, sh.prec, A[0], a_slot, Bt[0], b_slot, E, e_slot, nb, Mpad, Npad, sh.Kpad, false);
        post_join(cs, sh, E, e_slot, Npad, x0a, n0, x2a, n2, dst[0].data());
        // impure: E = A_S Bt_T + A_T Bt_S
        for (int j = 0; j < c.nimp; ++j) {
          join(c, sh.prec, A[1 + j], a_slot, Bt[0], b_slot, E, e_slot, nb, Mpad, Npad, sh.Kpad, false);
          join(c, sh.prec, A[0], a_slot, Bt[1 + j], b_slot, E, e_slot, nb, Mpad, Npad, sh.Kpad, true);
          post_join(cs, sh, E, e_slot, Npad, x0a, n0, x2a, n2, dst[1 + j].data());
        }
      }
    }

    // ---- 4: normalisation (ln c_n also into each step record), accumulator,
    // impure scaling
    const int nblk = norm_blocks();
    double *partial = c.wsp<double>("norm_partial", size_t(nblk) * nb * 8);
    NormBatch nbt{};
    std::vector<const double *> scals(nb);
    for (int b = 0; b < nb; ++b) {
      nbt.x[b] = dst[0][b];
      nbt.scal[b] = cs[b]->scal();
      nbt.err[b] = cs[b]->errp();
      nbt.rec[b] = preps[first + b]->rd;
      nbt.weight[b] = std::ldexp(1.0, -preps[first + b]->n_step);
      scals[b] = cs[b]->scal();
    }
    norm_and_accumulate_batch(nbt, nb, cap_tensor, partial, nblk, c.st);
    scale_by_inverse_batch(dst[0].data(), scals.data(), nb, cap_tensor, 1.0, c.st);
    for (int j = 0; j < c.nimp; ++j) scale_by_inverse_batch(dst[1 + j].data(), scals.data(), nb, cap_tensor, 0.5, c.st);

    for (int b = 0; b < nb; ++b) {
      trg_ctx &x = *cs[b];
      const int n_step = preps[first + b]->n_step;
      std::swap(x.T, x.Tn);
      for (int j = 0; j < x.nimp; ++j) std::swap(x.S[j], x.Sn[j]);
      trg_step_rec hr{};
      hr.n = n_step;
      hr.axis = mu;
      hr.join_precision = sh.prec;
      for (int ax = 0; ax < 4; ++ax) {
        hr.dims[ax] = ax < d ? sh.nd[ax] : 0;
        hr.side[ax] = -1;
      }
      x.host_rec.push_back(hr);
      for (int ax = 0; ax < d; ++ax) x.dims[ax] = sh.nd[ax];
      x.nsteps = n_step;
    }
  }
}

void hotrg_step_batch_impl(std::vector<trg_ctx *> cs, int mu, int dcut) {
  std::vector<StepPrep> ps;
  for (auto *c : cs) ps.push_back(prepare_step(*c, mu, dcut));
  isometries_batch(cs, ps, mu);
  // contexts with the same impurities share the contraction launches
  std::vector<bool> done(cs.size(), false);
  for (size_t i = 0; i < cs.size(); ++i) {
    if (done[i]) continue;
    std::vector<trg_ctx *> group;
    std::vector<StepPrep *> preps;
    for (size_t j = i; j < cs.size(); ++j) {
      if (done[j] || cs[j]->nimp != cs[i]->nimp || cs[j]->imp_kind[0] != cs[i]->imp_kind[0]) continue;
      group.push_back(cs[j]);
      preps.push_back(&ps[j]);
      done[j] = true;
    }
    contract_batch(group, preps, mu);
  }
}

void hotrg_step_impl(trg_ctx &c, int mu, int dcut) { hotrg_step_batch_impl({&c}, mu, dcut); }

// ------------------------------------------------------------- helpers ---
int fail(trg_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  g_thread_error = msg;
  return code;
}

template <typename F>
int guarded(trg_ctx *c, F &&f) {
  try {
    if (c && c->poisoned) return fail(c, TRG_ESTATE, "context is poisoned by an earlier device error: " + c->err);
    return f();
  } catch (const Error &e) {
    if (c && (e.code == TRG_EHIP || e.code == TRG_ENUMERIC)) c->poisoned = true;
    return fail(c, e.code, e.what());
  } catch (const std::bad_alloc &) {
    return fail(c, TRG_ENOMEM, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(c, TRG_EHIP, e.what());
  }
}

// wait for the stream and check the device error flag
void sync_check(trg_ctx &c) {
  TRG_HIP_CHECK(hipStreamSynchronize(c.st));
  int e = 0;
  TRG_HIP_CHECK(hipMemcpy(&e, c.errp(), sizeof(int), hipMemcpyDeviceToHost));
  if (e) {
    c.poisoned = true;
    throw Error(TRG_ENUMERIC, (e & 1) ? "normalisation produced a zero or non-finite norm"
                                      : "device numeric error");
  }
  if (c.profiling) {
    for (auto &pr : c.join_events) {
      float ms = 0.f;
      TRG_HIP_CHECK(hipEventElapsedTime(&ms, pr.first, pr.second));
      c.join_ms += ms;
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    c.join_events.clear();
    c.join_flops_done += c.join_flops_pending;
    c.join_flops_pending = 0.0;
  }
}

trg_ctx *new_ctx(int d, const trg_config *cfg) {
  auto *c = new trg_ctx();
  c->d = d;
  if (cfg) c->cfg = *cfg;
  if (c->cfg.dcut <= 0) c->cfg.dcut = 8;
  c->st = static_cast<hipStream_t>(c->cfg.stream);
  c->z2 = c->cfg.z2 != 0;
  return c;
}

void init_common(trg_ctx &c) {
  c.ensure(c.dev_scalars, 16 * 8);
  c.ensure(c.dev_err, 64);
  fill_zero(c.dev_scalars.ptr, 16 * 8, c.st);
  fill_zero(c.dev_err.ptr, 64, c.st);
  ensure_records(c, 64);
}

void validate_cfg(const trg_config *cfg, int d) {
  TRG_REQUIRE(d >= 2 && d <= 4, "d must be 2, 3 or 4");
  if (!cfg) return;
  TRG_REQUIRE(cfg->precision >= TRG_FP64 && cfg->precision <= TRG_BF16X6, "unknown precision");
  TRG_REQUIRE(cfg->method == TRG_HOTRG || cfg->method == TRG_ATRG, "unknown method");
  TRG_REQUIRE(cfg->dcut >= 0 && cfg->dcut <= 1024, "dcut out of range");
  TRG_REQUIRE((cfg->impure & ~3u) == 0, "unknown impurity bits");
  TRG_REQUIRE(!cfg->alloc == !cfg->free, "alloc and free must be given together");
  TRG_REQUIRE(cfg->fp64_steps >= 0, "fp64_steps must be >= 0");
  TRG_REQUIRE(cfg->z2 == 0 || cfg->z2 == 1, "z2 must be 0 or 1");
  TRG_REQUIRE(!cfg->z2 || cfg->method == TRG_ATRG, "the Z2 mode is an ATRG mode");
}

// normalise the freshly written tensors: c_0 = ||T||, acc = ln c_0
void normalise_initial(trg_ctx &c) {
  const int64_t n = c.total();
  const int nb = norm_blocks();
  double *partial = c.wsp<double>("norm_partial", size_t(nb) * 8);
  norm_and_accumulate(static_cast<double *>(c.T.ptr), n, partial, nb, c.scal(), c.scal() + 3, 1.0, c.errp(),
                      c.st);
  scale_by_inverse(static_cast<double *>(c.T.ptr), n, c.scal(), 1.0, c.st);
  for (int j = 0; j < c.nimp; ++j) scale_by_inverse(static_cast<double *>(c.S[j].ptr), n, c.scal(), 1.0, c.st);
  TRG_HIP_CHECK(hipMemcpyAsync(rec_d(c, 0), c.scal() + 2, 8, hipMemcpyDeviceToDevice, c.st));
}

}  // namespace trg

// ------------------------------------------------ allocation-free scratch ---
// Device scratch of trg_indicator_x_noalloc: the partial-trace matrix M
// (up to NOALLOC_MAX_N^2 doubles) followed by the two traces.  Each GPU the
// library runs on holds its own copy until the process ends.  Host code uses
// the address hipGetSymbolAddress returns for the current device, never the
// array's name (which is a host-side stand-in).
constexpr int NOALLOC_MAX_N = 256;
constexpr size_t NOALLOC_M_BYTES = size_t(NOALLOC_MAX_N) * NOALLOC_MAX_N * 8;
constexpr size_t NOALLOC_SCRATCH_BYTES = NOALLOC_M_BYTES + 256;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of `scratch` on the current device (looked up once per device)
void *scratch_on_current_device() {
  int dev = -1;
  TRG_HIP_CHECK(hipGetDevice(&dev));
  TRG_REQUIRE(dev >= 0 && dev < NOALLOC_MAX_DEVICES, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    TRG_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    TRG_REQUIRE(ptr != nullptr, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

// =================================================================== C-ABI ==
extern "C" {

int trg_init_ising(trg_ctx **out, double beta, double h, int d, const trg_config *cfg) {
  if (!out) return fail(nullptr, TRG_EINVAL, "out is NULL");
  *out = nullptr;
  trg_ctx *c = nullptr;
  int rc = guarded(nullptr, [&]() -> int {
    validate_cfg(cfg, d);
    TRG_REQUIRE(std::isfinite(beta) && beta >= 0.0, "beta must be finite and >= 0");
    TRG_REQUIRE(std::isfinite(h), "h must be finite");
    const unsigned imp = cfg ? cfg->impure : 0u;
    TRG_REQUIRE(!(imp & TRG_IMPURE_E) || beta > 0.0, "the energy impurity needs beta > 0");
    const bool atrg = cfg && cfg->method == TRG_ATRG;
    TRG_REQUIRE(!atrg || cfg->precision <= TRG_FP32, "ATRG supports FP64 and FP32 contractions");
    TRG_REQUIRE(!(cfg && cfg->z2) || h == 0.0, "the Z2 mode needs h = 0 (the symmetric tensor)");
    c = new_ctx(d, cfg);
    for (int a = 0; a < d; ++a) c->dims[a] = 2;
    c->has_e = imp & TRG_IMPURE_E;
    c->has_m = imp & TRG_IMPURE_M;
    if (c->has_e) c->imp_kind[c->nimp++] = 0;
    if (c->has_m) c->imp_kind[c->nimp++] = 1;
    if (atrg) {
      init_common(*c);
      atrg_init_ising(*c, beta, h);
      return TRG_OK;
    }
    init_common(*c);
    const size_t bytes = size_t(c->total()) * 8;
    c->ensure(c->T, bytes);
    for (int j = 0; j < c->nimp; ++j) c->ensure(c->S[j], bytes);
    double *SE = c->has_e ? static_cast<double *>(c->S[0].ptr) : nullptr;
    double *SM = c->has_m ? static_cast<double *>(c->S[c->has_e ? 1 : 0].ptr) : nullptr;
    ising_init(static_cast<double *>(c->T.ptr), SE, SM, d, beta, h, c->st);
    normalise_initial(*c);
    return TRG_OK;
  });
  if (rc != TRG_OK) {
    if (c) trg_free(c);
    return rc;
  }
  *out = c;
  return TRG_OK;
}

int trg_init_tensor(trg_ctx **out, int d, const int *dims, const double *host_tensor, const trg_config *cfg) {
  if (!out || !dims || !host_tensor) return fail(nullptr, TRG_EINVAL, "NULL argument");
  *out = nullptr;
  trg_ctx *c = nullptr;
  int rc = guarded(nullptr, [&]() -> int {
    validate_cfg(cfg, d);
    TRG_REQUIRE(!cfg || cfg->impure == 0, "impurities need trg_init_ising");
    TRG_REQUIRE(!cfg || cfg->method == TRG_HOTRG, "ATRG contexts are not available in this build");
    for (int a = 0; a < d; ++a) TRG_REQUIRE(dims[a] >= 1 && dims[a] <= 1024, "bad leg dim");
    c = new_ctx(d, cfg);
    for (int a = 0; a < d; ++a) c->dims[a] = dims[a];
    init_common(*c);
    const size_t bytes = size_t(c->total()) * 8;
    c->ensure(c->T, bytes);
    TRG_HIP_CHECK(hipMemcpyAsync(c->T.ptr, host_tensor, bytes, hipMemcpyHostToDevice, c->st));
    normalise_initial(*c);
    sync_check(*c);
    return TRG_OK;
  });
  if (rc != TRG_OK) {
    if (c) trg_free(c);
    return rc;
  }
  *out = c;
  return TRG_OK;
}

int trg_hotrg_step(trg_ctx *ctx, int axis, int dcut) {
  if (!ctx) return fail(nullptr, TRG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() -> int {
    TRG_REQUIRE(axis >= 0 && axis < ctx->d, "axis out of range");
    TRG_REQUIRE(dcut >= 1 && dcut <= 1024, "dcut out of range");
    TRG_REQUIRE(ctx->cfg.method == TRG_HOTRG, "context method is not HOTRG");
    hotrg_step_impl(*ctx, axis, dcut);
    return TRG_OK;
  });
}

int trg_hotrg_step_batch(trg_ctx *const *ctxs, int n, int axis, int dcut) {
  if (!ctxs || n < 1) return fail(nullptr, TRG_EINVAL, "empty batch");
  // pointers first (no context is read before they are all distinct)
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return fail(nullptr, TRG_EINVAL, "NULL context in batch");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(nullptr, TRG_EINVAL, "a context appears twice in the batch");
  }
  for (int i = 0; i < n; ++i) {
    if (ctxs[i]->d != ctxs[0]->d || join_precision(*ctxs[i]) != join_precision(*ctxs[0]) ||
        producer_precision(*ctxs[i]) != producer_precision(*ctxs[0]) || ctxs[i]->st != ctxs[0]->st)
      return fail(nullptr, TRG_EINVAL, "batch contexts differ in d, join precision or stream");
    for (int a = 0; a < ctxs[0]->d; ++a)
      if (ctxs[i]->dims[a] != ctxs[0]->dims[a]) return fail(nullptr, TRG_EINVAL, "batch contexts differ in dims");
  }
  for (int i = 0; i < n; ++i)
    if (ctxs[i]->poisoned) return fail(ctxs[i], TRG_ESTATE, "context is poisoned by an earlier device error");
  if (axis < 0 || axis >= ctxs[0]->d || dcut < 1 || dcut > 1024) return fail(nullptr, TRG_EINVAL, "bad axis or dcut");
  for (int i = 0; i < n; ++i)
    if (ctxs[i]->cfg.method != TRG_HOTRG) return fail(nullptr, TRG_EINVAL, "batch contexts must be HOTRG");
  const int rc = guarded(nullptr, [&]() -> int {
    std::vector<trg_ctx *> cs(ctxs, ctxs + n);
    hotrg_step_batch_impl(cs, axis, dcut);
    return TRG_OK;
  });
  if (rc == TRG_EHIP || rc == TRG_ENUMERIC) {
    // the device state of every context of the batch is unknown
    for (int i = 0; i < n; ++i) {
      ctxs[i]->poisoned = true;
      ctxs[i]->err = g_thread_error;
    }
  } else if (rc != TRG_OK) {
    for (int i = 0; i < n; ++i) ctxs[i]->err = g_thread_error;
  }
  return rc;
}

int trg_atrg_step(trg_ctx *ctx, int axis, int dcut) {
  if (!ctx) return fail(nullptr, TRG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() -> int {
    TRG_REQUIRE(axis >= 0 && axis < ctx->d, "axis out of range");
    TRG_REQUIRE(dcut >= 1 && dcut <= 256, "dcut out of range for ATRG");
    if (ctx->cfg.method != TRG_ATRG) return fail(ctx, TRG_ESTATE, "context method is not ATRG");
    atrg_step_impl(*ctx, axis, dcut);
    return TRG_OK;
  });
}

int trg_init_factors(trg_ctx **out, int d, const int *dims, int r, const double *host_G, const double *host_H,
                     const trg_config *cfg) {
  if (!out || !dims || !host_G || !host_H) return fail(nullptr, TRG_EINVAL, "NULL argument");
  *out = nullptr;
  trg_ctx *c = nullptr;
  int rc = guarded(nullptr, [&]() -> int {
    validate_cfg(cfg, d);
    TRG_REQUIRE(cfg && cfg->method == TRG_ATRG, "factors need method TRG_ATRG");
    TRG_REQUIRE(cfg->impure == 0 && cfg->precision <= TRG_FP32, "unsupported ATRG configuration");
    TRG_REQUIRE(!cfg->z2, "the Z2 mode starts from trg_init_ising (its parities are known there)");
    TRG_REQUIRE(r >= 1 && r <= 512, "rank out of range");
    int64_t n = 1;
    for (int a = 0; a < d; ++a) {
      TRG_REQUIRE(dims[a] >= 1 && dims[a] <= 1024, "bad leg dim");
      n *= dims[a];
    }
    TRG_REQUIRE(n >= r, "pieces need at least r rows");
    c = new_ctx(d, cfg);
    for (int a = 0; a < d; ++a) c->dims[a] = dims[a];
    init_common(*c);
    c->r = r;
    c->ensure(c->G, size_t(n) * r * 8);
    c->ensure(c->H, size_t(n) * r * 8);
    TRG_HIP_CHECK(hipMemcpyAsync(c->G.ptr, host_G, size_t(n) * r * 8, hipMemcpyHostToDevice, c->st));
    TRG_HIP_CHECK(hipMemcpyAsync(c->H.ptr, host_H, size_t(n) * r * 8, hipMemcpyHostToDevice, c->st));
    sync_check(*c);
    return TRG_OK;
  });
  if (rc != TRG_OK) {
    if (c) trg_free(c);
    return rc;
  }
  *out = c;
  return TRG_OK;
}

int trg_atrg_spectrum(trg_ctx *ctx, double *out, int cap, int *n) {
  if (!ctx || !n) return fail(ctx, TRG_EINVAL, "NULL argument");
  return guarded(ctx, [&]() -> int {
    sync_check(*ctx);
    *n = ctx->atrg_nsig;
    if (out && ctx->atrg_nsig > 0) {
      TRG_REQUIRE(cap >= ctx->atrg_nsig, "capacity too small");
      TRG_HIP_CHECK(hipMemcpy(out, ctx->atrg_sigma.ptr, size_t(ctx->atrg_nsig) * 8, hipMemcpyDeviceToHost));
    }
    return TRG_OK;
  });
}

int trg_atrg_parities(trg_ctx *ctx, int *legs_out, size_t cap_legs, int *bond_out, size_t cap_bond, int *r_out) {
  if (!ctx) return fail(nullptr, TRG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() -> int {
    if (!ctx->z2) return fail(ctx, TRG_ESTATE, "not a Z2 context");
    sync_check(*ctx);
    if (r_out) *r_out = int(ctx->z2_bond.size());
    size_t nl = 0;
    for (int a = 0; a < ctx->d; ++a) nl += ctx->z2_legs[a].size();
    if (legs_out) {
      TRG_REQUIRE(cap_legs >= nl, "legs capacity too small");
      size_t e = 0;
      for (int a = 0; a < ctx->d; ++a)
        for (int8_t x : ctx->z2_legs[a]) legs_out[e++] = x;
    }
    if (bond_out) {
      TRG_REQUIRE(cap_bond >= ctx->z2_bond.size(), "bond capacity too small");
      for (size_t i = 0; i < ctx->z2_bond.size(); ++i) bond_out[i] = ctx->z2_bond[i];
    }
    return TRG_OK;
  });
}

int trg_get_factors(trg_ctx *ctx, double *host_G, size_t cap_G, double *host_H, size_t cap_H, int *r_out) {
  if (!ctx) return fail(nullptr, TRG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() -> int {
    if (ctx->cfg.method != TRG_ATRG) return fail(ctx, TRG_ESTATE, "not an ATRG context");
    sync_check(*ctx);
    int64_t n = 1;
    for (int a = 0; a < ctx->d; ++a) n *= ctx->dims[a];
    const size_t cnt = size_t(n) * size_t(ctx->r);
    if (r_out) *r_out = ctx->r;
    if (host_G) {
      TRG_REQUIRE(cap_G >= cnt, "G capacity too small");
      TRG_HIP_CHECK(hipMemcpy(host_G, ctx->G.ptr, cnt * 8, hipMemcpyDeviceToHost));
    }
    if (host_H) {
      TRG_REQUIRE(cap_H >= cnt, "H capacity too small");
      TRG_HIP_CHECK(hipMemcpy(host_H, ctx->H.ptr, cnt * 8, hipMemcpyDeviceToHost));
    }
    return TRG_OK;
  });
}

int trg_run(trg_ctx *ctx, long long L) {
  if (!ctx) return fail(nullptr, TRG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() -> int {
    TRG_REQUIRE(L >= 2 && (L & (L - 1)) == 0, "L must be a power of two >= 2");
    int m = 0;
    while ((1LL << m) < L) ++m;
    TRG_REQUIRE(ctx->nsteps <= ctx->d * m, "the context has already taken more steps than this lattice needs");
    // continues from the current step (a resumed checkpoint finishes its lattice)
    for (int n = ctx->nsteps + 1; n <= ctx->d * m; ++n) {
      if (ctx->cfg.method == TRG_ATRG)
        atrg_step_impl(*ctx, (n - 1) % ctx->d, ctx->cfg.dcut);
      else
        hotrg_step_impl(*ctx, (n - 1) % ctx->d, ctx->cfg.dcut);
    }
    sync_check(*ctx);
    return TRG_OK;
  });
}

static int traces(trg_ctx *ctx, double out[4]) {
  // out[0] = acc, out[1] = Tr T, out[2] = Tr S_E, out[3] = Tr S_M
  const double *X[3] = {static_cast<const double *>(ctx->T.ptr), nullptr, nullptr};
  for (int j = 0; j < ctx->nimp; ++j) X[1 + j] = static_cast<const double *>(ctx->S[j].ptr);
  periodic_traces(X, 1 + ctx->nimp, ctx->dims, ctx->d, ctx->scal() + 4, ctx->st);
  sync_check(*ctx);
  double h[4] = {0, 0, 0, 0};
  TRG_HIP_CHECK(hipMemcpy(h, ctx->scal() + 3, 4 * 8, hipMemcpyDeviceToHost));
  out[0] = h[0];
  out[1] = h[1];
  out[2] = out[3] = NAN;
  for (int j = 0; j < ctx->nimp; ++j) out[2 + ctx->imp_kind[j]] = h[2 + j];
  return TRG_OK;
}

int trg_free_energy(trg_ctx *ctx, double *lnz) {
  if (!ctx || !lnz) return fail(ctx, TRG_EINVAL, "NULL argument");
  return guarded(ctx, [&]() -> int {
    double t[4];
    if (ctx->cfg.method == TRG_ATRG) {
      t[1] = atrg_trace(*ctx);
      TRG_HIP_CHECK(hipMemcpy(&t[0], ctx->scal() + 3, 8, hipMemcpyDeviceToHost));
    } else {
      traces(ctx, t);
    }
    if (!(t[1] > 0.0) || !std::isfinite(t[1])) throw Error(TRG_ENUMERIC, "non-positive trace of the tensor");
    *lnz = t[0] + std::ldexp(1.0, -ctx->nsteps) * std::log(t[1]);
    return TRG_OK;
  });
}

int trg_indicator_x(trg_ctx *ctx, int axis, double *X) {
  if (!ctx || !X) return fail(ctx, TRG_EINVAL, "NULL argument");
  return guarded(ctx, [&]() -> int {
    TRG_REQUIRE(axis >= 0 && axis < ctx->d, "axis out of range");
    const int n = ctx->dims[axis];
    double *M = ctx->wsp<double>("xind_M", size_t(n) * n * 8);
    double *out = ctx->wsp<double>("xind_out", 2 * 8);
    if (ctx->cfg.method == TRG_ATRG)
      atrg_indicator_traces(*ctx, axis, M, out);
    else
      indicator_traces(static_cast<const double *>(ctx->T.ptr), ctx->dims, ctx->d, axis, M, out, ctx->st);
    sync_check(*ctx);
    double t[2];
    TRG_HIP_CHECK(hipMemcpy(t, out, 2 * 8, hipMemcpyDeviceToHost));
    if (!(t[1] > 0.0) || !std::isfinite(t[0])) throw Error(TRG_ENUMERIC, "indicator: vanishing two-site trace");
    *X = t[0] * t[0] / t[1];
    return TRG_OK;
  });
}

int trg_indicator_x_noalloc(trg_ctx *ctx, int axis, double *X) {
  if (!ctx || !X) return fail(ctx, TRG_EINVAL, "NULL argument");
  return guarded(ctx, [&]() -> int {
    TRG_REQUIRE(axis >= 0 && axis < ctx->d, "axis out of range");
    TRG_REQUIRE(ctx->cfg.method == TRG_HOTRG, "the allocation-free indicator takes HOTRG contexts");
    const int n = ctx->dims[axis];
    TRG_REQUIRE(n >= 1 && n <= NOALLOC_MAX_N, "leg dim of the axis exceeds the static scratch (at most 256)");
    char *base = static_cast<char *>(scratch_on_current_device());
    double *M = reinterpret_cast<double *>(base);
    double *out = reinterpret_cast<double *>(base + NOALLOC_M_BYTES);
    // both kernels overwrite every scratch entry they later read
    indicator_traces(static_cast<const double *>(ctx->T.ptr), ctx->dims, ctx->d, axis, M, out, ctx->st);
    sync_check(*ctx);
    double t[2];
    TRG_HIP_CHECK(hipMemcpy(t, out, 2 * 8, hipMemcpyDeviceToHost));
    if (!(t[1] > 0.0) || !std::isfinite(t[0])) throw Error(TRG_ENUMERIC, "indicator: vanishing two-site trace");
    *X = t[0] * t[0] / t[1];
    return TRG_OK;
  });
}

// Tr T and Tr S of the impurity of `kind` (0 E, 1 M)
static void impure_traces(trg_ctx *ctx, int kind, double *tT, double *tS) {
  if (ctx->cfg.method == TRG_ATRG) {
    int j = 0;
    while (j < ctx->nimp && ctx->imp_kind[j] != kind) ++j;
    *tT = atrg_trace(*ctx);
    *tS = atrg_impurity_trace(*ctx, j);
    return;
  }
  double t[4];
  traces(ctx, t);
  *tT = t[1];
  *tS = t[2 + kind];
}

int trg_impure_energy(trg_ctx *ctx, double *E) {
  if (!ctx || !E) return fail(ctx, TRG_EINVAL, "NULL argument");
  return guarded(ctx, [&]() -> int {
    if (!ctx->has_e) return fail(ctx, TRG_ESTATE, "energy impurity not enabled");
    double tT = 0.0, tS = 0.0;
    impure_traces(ctx, 0, &tT, &tS);
    *E = -tS / tT;
    return TRG_OK;
  });
}

int trg_impure_magnetization(trg_ctx *ctx, double *M) {
  if (!ctx || !M) return fail(ctx, TRG_EINVAL, "NULL argument");
  return guarded(ctx, [&]() -> int {
    if (!ctx->has_m) return fail(ctx, TRG_ESTATE, "magnetization impurity not enabled");
    double tT = 0.0, tS = 0.0;
    impure_traces(ctx, 1, &tT, &tS);
    *M = tS / tT;
    return TRG_OK;
  });
}

int trg_accumulator(trg_ctx *ctx, double *acc) {
  if (!ctx || !acc) return fail(ctx, TRG_EINVAL, "NULL argument");
  return guarded(ctx, [&]() -> int {
    sync_check(*ctx);
    TRG_HIP_CHECK(hipMemcpy(acc, ctx->scal() + 3, 8, hipMemcpyDeviceToHost));
    return TRG_OK;
  });
}

int trg_get_dims(const trg_ctx *ctx, int *dims, int *steps) {
  if (!ctx) return fail(nullptr, TRG_EINVAL, "ctx is NULL");
  if (dims)
    for (int a = 0; a < ctx->d; ++a) dims[a] = ctx->dims[a];
  if (steps) *steps = ctx->nsteps;
  return TRG_OK;
}

int trg_get_tensor(trg_ctx *ctx, int which, double *host_out, size_t cap) {
  if (!ctx || !host_out) return fail(ctx, TRG_EINVAL, "NULL argument");
  return guarded(ctx, [&]() -> int {
    if (ctx->cfg.method != TRG_HOTRG) return fail(ctx, TRG_ESTATE, "ATRG contexts hold factored tensors");
    const size_t n = size_t(ctx->total());
    TRG_REQUIRE(cap >= n, "output capacity too small");
    const void *src = nullptr;
    if (which == 0) src = ctx->T.ptr;
    for (int j = 0; j < ctx->nimp; ++j)
      if (which == 1 + ctx->imp_kind[j]) src = ctx->S[j].ptr;
    if (!src) return fail(ctx, TRG_ESTATE, "requested tensor not present");
    sync_check(*ctx);
    TRG_HIP_CHECK(hipMemcpy(host_out, src, n * 8, hipMemcpyDeviceToHost));
    return TRG_OK;
  });
}

int trg_get_isometry(trg_ctx *ctx, int nu, double *host_U, size_t capU, double *host_spectrum, size_t capS) {
  if (!ctx) return fail(nullptr, TRG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() -> int {
    TRG_REQUIRE(nu >= 0 && nu < ctx->d && ctx->Un[nu] > 0, "no isometry for that axis");
    sync_check(*ctx);
    const size_t n = size_t(ctx->Un[nu]), k = size_t(ctx->Uk[nu]);
    if (host_U) {
      TRG_REQUIRE(capU >= n * k, "U capacity too small");
      TRG_HIP_CHECK(hipMemcpy(host_U, ctx->U[nu].ptr, n * k * 8, hipMemcpyDeviceToHost));
    }
    if (host_spectrum) {
      TRG_REQUIRE(capS >= n, "spectrum capacity too small");
      TRG_HIP_CHECK(hipMemcpy(host_spectrum, ctx->spec[nu].ptr, n * 8, hipMemcpyDeviceToHost));
    }
    return TRG_OK;
  });
}

}  // extern "C"

// ------------------------------------------------------------ checkpoint ---
namespace {
struct StateHeader {
  char magic[8];
  uint32_t version, impure;
  int32_t d, method, precision, dcut, rsvd_p, rsvd_q, fp64_steps, nsteps, nimp, r, force_side;
  int32_t imp_kind[2], imp_r[2], dims[4];
  uint64_t seed, rec_bytes, nhost, ndoubles;
  int32_t z2, pad;   // z2: the leg and bond parity bytes follow the tensors
};
constexpr char STATE_MAGIC[8] = {'T', 'R', 'G', 'S', 'T', 'A', 'T', 'E'};
constexpr uint32_t STATE_VERSION = 2;

// bytes of the Z2 parity tables: every leg index of each axis, then the bond
size_t z2_table_bytes(int z2, int d, const int32_t *dims, int r) {
  if (!z2) return 0;
  size_t n = size_t(r);
  for (int a = 0; a < d; ++a) n += size_t(dims[a]);
  return n;
}

// the device buffers of the state, in blob order, with their sizes in doubles
std::vector<std::pair<void *, size_t>> state_tensors(trg_ctx &c) {
  std::vector<std::pair<void *, size_t>> v;
  if (c.cfg.method == TRG_ATRG) {
    int64_t n = 1;
    for (int a = 0; a < c.d; ++a) n *= c.dims[a];
    v.push_back({c.G.ptr, size_t(n) * c.r});
    v.push_back({c.H.ptr, size_t(n) * c.r});
    for (int j = 0; j < c.nimp; ++j) {
      v.push_back({c.S[j].ptr, size_t(n) * c.imp_r[j]});
      v.push_back({c.Sn[j].ptr, size_t(n) * c.imp_r[j]});
    }
  } else {
    v.push_back({c.T.ptr, size_t(c.total())});
    for (int j = 0; j < c.nimp; ++j) v.push_back({c.S[j].ptr, size_t(c.total())});
  }
  return v;
}
}  // namespace

extern "C" {

int trg_export_state(trg_ctx *ctx, void *host_buf, size_t cap, size_t *size) {
  if (!ctx || !size) return fail(ctx, TRG_EINVAL, "NULL argument");
  return guarded(ctx, [&]() -> int {
    sync_check(*ctx);
    const auto ten = state_tensors(*ctx);
    size_t nd = 0;
    for (const auto &t : ten) nd += t.second;
    const size_t rec_bytes = size_t(ctx->nsteps + 1) * REC_BYTES;
    int32_t dims32[4];
    for (int a = 0; a < 4; ++a) dims32[a] = ctx->dims[a];
    const size_t zb = z2_table_bytes(ctx->z2, ctx->d, dims32, ctx->r);
    const size_t total = sizeof(StateHeader) + 16 * 8 + rec_bytes + ctx->host_rec.size() * sizeof(trg_step_rec) +
                         nd * 8 + zb;
    *size = total;
    if (!host_buf) return TRG_OK;
    TRG_REQUIRE(cap >= total, "state buffer too small");
    StateHeader h{};
    std::memcpy(h.magic, STATE_MAGIC, 8);
    h.version = STATE_VERSION;
    h.impure = ctx->cfg.impure;
    h.d = ctx->d;
    h.method = ctx->cfg.method;
    h.precision = ctx->cfg.precision;
    h.dcut = ctx->cfg.dcut;
    h.rsvd_p = ctx->cfg.rsvd_p;
    h.rsvd_q = ctx->cfg.rsvd_q;
    h.fp64_steps = ctx->cfg.fp64_steps;
    h.nsteps = ctx->nsteps;
    h.nimp = ctx->nimp;
    h.r = ctx->r;
    h.force_side = ctx->force_side;
    for (int j = 0; j < 2; ++j) {
      h.imp_kind[j] = ctx->imp_kind[j];
      h.imp_r[j] = ctx->imp_r[j];
    }
    for (int a = 0; a < 4; ++a) h.dims[a] = ctx->dims[a];
    h.seed = ctx->cfg.seed;
    h.rec_bytes = rec_bytes;
    h.nhost = ctx->host_rec.size();
    h.ndoubles = nd;
    h.z2 = ctx->z2 ? 1 : 0;
    char *p = static_cast<char *>(host_buf);
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    TRG_HIP_CHECK(hipMemcpy(p, ctx->dev_scalars.ptr, 16 * 8, hipMemcpyDeviceToHost));
    p += 16 * 8;
    TRG_HIP_CHECK(hipMemcpy(p, ctx->dev_rec.ptr, rec_bytes, hipMemcpyDeviceToHost));
    p += rec_bytes;
    if (!ctx->host_rec.empty()) std::memcpy(p, ctx->host_rec.data(), ctx->host_rec.size() * sizeof(trg_step_rec));
    p += ctx->host_rec.size() * sizeof(trg_step_rec);
    for (const auto &t : ten) {
      TRG_HIP_CHECK(hipMemcpy(p, t.first, t.second * 8, hipMemcpyDeviceToHost));
      p += t.second * 8;
    }
    if (ctx->z2) {
      for (int a = 0; a < ctx->d; ++a) {
        TRG_REQUIRE(int(ctx->z2_legs[a].size()) == ctx->dims[a], "z2: leg parity table out of step");
        std::memcpy(p, ctx->z2_legs[a].data(), ctx->z2_legs[a].size());
        p += ctx->z2_legs[a].size();
      }
      TRG_REQUIRE(int(ctx->z2_bond.size()) == ctx->r, "z2: bond parity table out of step");
      std::memcpy(p, ctx->z2_bond.data(), ctx->z2_bond.size());
      p += ctx->z2_bond.size();
    }
    return TRG_OK;
  });
}

int trg_import_state(trg_ctx **out, const void *host_buf, size_t size, const trg_config *cfg) {
  if (!out || !host_buf) return fail(nullptr, TRG_EINVAL, "NULL argument");
  *out = nullptr;
  trg_ctx *c = nullptr;
  int rc = guarded(nullptr, [&]() -> int {
    TRG_REQUIRE(size >= sizeof(StateHeader), "state blob too short");
    StateHeader h{};
    std::memcpy(&h, host_buf, sizeof h);
    TRG_REQUIRE(std::memcmp(h.magic, STATE_MAGIC, 8) == 0, "not a state blob (bad magic)");
    TRG_REQUIRE(h.version == STATE_VERSION, "unsupported state blob version");
    TRG_REQUIRE(h.d >= 2 && h.d <= 4 && h.nsteps >= 0 && h.nimp >= 0 && h.nimp <= 2, "corrupt state header");
    TRG_REQUIRE(h.rec_bytes == size_t(h.nsteps + 1) * REC_BYTES, "corrupt state header (records)");
    for (int a = 0; a < h.d; ++a) TRG_REQUIRE(h.dims[a] >= 1 && h.dims[a] <= 1024, "corrupt state header (dims)");
    TRG_REQUIRE((h.z2 == 0 || h.z2 == 1) && (!h.z2 || h.method == TRG_ATRG), "corrupt state header (z2)");
    TRG_REQUIRE(h.r >= 0 && h.r <= 4096, "corrupt state header (bond)");
    const size_t need = sizeof(StateHeader) + 16 * 8 + h.rec_bytes + h.nhost * sizeof(trg_step_rec) +
                        h.ndoubles * 8 + z2_table_bytes(h.z2, h.d, h.dims, h.r);
    TRG_REQUIRE(size == need, "state blob size does not match its header");
    // the blob fixes the numerics; cfg may bring the stream, allocator and
    // workspace budget
    trg_config k = cfg ? *cfg : trg_config{};
    k.method = h.method;
    k.precision = h.precision;
    k.dcut = h.dcut;
    k.impure = h.impure;
    k.rsvd_p = h.rsvd_p;
    k.rsvd_q = h.rsvd_q;
    k.fp64_steps = h.fp64_steps;
    k.seed = h.seed;
    k.z2 = h.z2;
    validate_cfg(&k, h.d);
    c = new_ctx(h.d, &k);
    for (int a = 0; a < h.d; ++a) c->dims[a] = h.dims[a];
    c->nsteps = h.nsteps;
    c->nimp = h.nimp;
    c->r = h.r;
    c->force_side = h.force_side;
    for (int j = 0; j < 2; ++j) {
      c->imp_kind[j] = h.imp_kind[j];
      c->imp_r[j] = h.imp_r[j];
    }
    for (int j = 0; j < c->nimp; ++j) {
      TRG_REQUIRE(c->imp_kind[j] == 0 || c->imp_kind[j] == 1, "corrupt state header (impurity)");
      c->has_e = c->has_e || c->imp_kind[j] == 0;
      c->has_m = c->has_m || c->imp_kind[j] == 1;
    }
    init_common(*c);
    ensure_records(*c, h.nsteps + 2);
    auto ten = [&]() {
      std::vector<size_t> v;
      int64_t n = 1, tot = 1;
      for (int a = 0; a < h.d; ++a) {
        n *= h.dims[a];
        tot *= int64_t(h.dims[a]) * h.dims[a];
      }
      if (h.method == TRG_ATRG) {
        v.push_back(size_t(n) * h.r);
        v.push_back(size_t(n) * h.r);
        for (int j = 0; j < h.nimp; ++j) {
          v.push_back(size_t(n) * h.imp_r[j]);
          v.push_back(size_t(n) * h.imp_r[j]);
        }
      } else {
        for (int j = 0; j <= h.nimp; ++j) v.push_back(size_t(tot));
      }
      return v;
    }();
    size_t nd = 0;
    for (size_t x : ten) nd += x;
    TRG_REQUIRE(nd == h.ndoubles, "state blob tensor sizes do not match its header");
    if (h.method == TRG_ATRG) {
      c->ensure(c->G, ten[0] * 8);
      c->ensure(c->H, ten[1] * 8);
      for (int j = 0; j < c->nimp; ++j) {
        c->ensure(c->S[j], ten[2 + 2 * j] * 8);
        c->ensure(c->Sn[j], ten[3 + 2 * j] * 8);
      }
    } else {
      c->ensure(c->T, ten[0] * 8);
      for (int j = 0; j < c->nimp; ++j) c->ensure(c->S[j], ten[1 + j] * 8);
    }
    // the zero fills and allocations above are queued on the context's stream
    TRG_HIP_CHECK(hipStreamSynchronize(c->st));
    const char *p = static_cast<const char *>(host_buf) + sizeof h;
    TRG_HIP_CHECK(hipMemcpy(c->dev_scalars.ptr, p, 16 * 8, hipMemcpyHostToDevice));
    p += 16 * 8;
    TRG_HIP_CHECK(hipMemcpy(c->dev_rec.ptr, p, h.rec_bytes, hipMemcpyHostToDevice));
    p += h.rec_bytes;
    c->host_rec.resize(h.nhost);
    if (h.nhost) std::memcpy(c->host_rec.data(), p, h.nhost * sizeof(trg_step_rec));
    p += h.nhost * sizeof(trg_step_rec);
    for (const auto &t : state_tensors(*c)) {
      TRG_HIP_CHECK(hipMemcpy(t.first, p, t.second * 8, hipMemcpyHostToDevice));
      p += t.second * 8;
    }
    if (c->z2) {
      auto table = [&](size_t n) {
        std::vector<int8_t> v(reinterpret_cast<const int8_t *>(p), reinterpret_cast<const int8_t *>(p) + n);
        for (int8_t x : v) TRG_REQUIRE(x == 0 || x == 1, "corrupt state blob (parity)");
        p += n;
        return v;
      };
      for (int a = 0; a < h.d; ++a) c->z2_legs[a] = table(size_t(h.dims[a]));
      c->z2_bond = table(size_t(h.r));
    }
    return TRG_OK;
  });
  if (rc != TRG_OK) {
    if (c) trg_free(c);
    return rc;
  }
  *out = c;
  return TRG_OK;
}

int trg_step_log(trg_ctx *ctx, trg_step_rec *out, int cap, int *n) {
  if (!ctx || !n) return fail(ctx, TRG_EINVAL, "NULL argument");
  return guarded(ctx, [&]() -> int {
    sync_check(*ctx);
    const int cnt = int(ctx->host_rec.size());
    *n = cnt;
    if (!out) return TRG_OK;
    std::vector<char> raw(size_t(ctx->nsteps + 1) * REC_BYTES);
    TRG_HIP_CHECK(hipMemcpy(raw.data(), ctx->dev_rec.ptr, raw.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < cnt && i < cap; ++i) {
      trg_step_rec r = ctx->host_rec[i];
      const char *base = raw.data() + size_t(r.n) * REC_BYTES;
      const double *dd = reinterpret_cast<const double *>(base);
      const int *ii = reinterpret_cast<const int *>(base + REC_D * 8);
      r.ln_c = dd[0];
      for (int ax = 0; ax < 4; ++ax) {
        if (ax >= ctx->d || ax == r.axis) continue;
        r.eps[ax][0] = dd[1 + 2 * ax];
        r.eps[ax][1] = dd[2 + 2 * ax];
        r.side[ax] = ii[4 * ax];
        r.kept[ax] = ii[4 * ax + 1];
        r.degenerate_cut[ax] = ii[4 * ax + 2];
        r.sweeps[ax] = ii[4 * ax + 3];
      }
      out[i] = r;
    }
    return TRG_OK;
  });
}

size_t trg_resident_bytes(int d, int dcut, int precision, int method, unsigned impure) {
  (void)precision;
  if (d < 2 || d > 4 || dcut < 1) return 0;
  const double D = dcut;
  if (method == TRG_ATRG) {
    // G, H and their next copies; each impurity: two pieces of bond 2 Dcut
    // and their next copies
    const int ni = ((impure & 1u) ? 1 : 0) + ((impure & 2u) ? 1 : 0);
    return size_t((2.0 + 4.0 * ni) * 2.0 * std::pow(D, d + 1) * 8.0);
  }
  const int nt = 1 + ((impure & 1u) ? 1 : 0) + ((impure & 2u) ? 1 : 0);
  return size_t(2.0 * nt * std::pow(D, 2 * d) * 8.0);  // each tensor and its next-step buffer
}

size_t trg_workspace_bytes(int d, int dcut, int precision, int method, unsigned impure) {
  if (d < 2 || d > 4 || dcut < 1) return 0;
  const double D = dcut;
  if (method == TRG_ATRG) {
    // the D^{2d-1} contraction intermediate (GEMM output and its unpacked
    // copy) plus the randomized-SVD blocks (r = 5 Dcut columns); the
    // impurities' SVDs (rows up to 2 Dcut D^{d-1}) and new pieces on top
    const bool imp = (impure & 3u) != 0;
    return size_t(2.0 * std::pow(D, 2 * d - 1) * 8.0 + (imp ? 16.0 : 8.0) * std::pow(D, d) * 5.0 * D * 8.0 +
                  (imp ? 5.0 * std::pow(D, d + 1) * 8.0 : 0.0));
  }
  // steady-state join of the natural plan (every leg at Dcut)
  const int nt = 1 + ((impure & 1u) ? 1 : 0) + ((impure & 2u) ? 1 : 0);
  const int pre = d / 2, post = d - 1 - pre;
  const double Mr = std::pow(D, 2 * post + pre);
  const double K = std::pow(D, 1 + 2 * pre);
  const GemmTile tile = gemm_tile(precision);
  const double Kpad = double(round_up(size_t(K), tile.k));
  const double esz = operand_bytes(precision);
  const double esE = precision == TRG_FP64 ? 8.0 : 4.0;
  const double c0 = std::max(1.0, std::min(D, std::floor(double(JOIN_ROWS) / Mr)));
  const double Mp = double(round_up(size_t(c0 * Mr), tile.m)), Np = double(round_up(size_t(D * Mr), tile.n));
  double b = nt * (Mp + Np) * Kpad * esz;                 // operands
  b += D * std::pow(D, 2 * d - 1) * D * 8.0;              // operand build temporary
  b += Mp * Np * esE;                                     // join result
  if (post) b += c0 * D * std::pow(D, 2 * post + 2 * pre + post) * 8.0;  // post-join temporary
  b += 12.0 * std::pow(D, 2 * d) * 8.0 / 1.0;             // Gram packing, partials, eigensystems (bound)
  return size_t(b);
}

size_t trg_footprint_bytes(int d, int dcut, int precision, int method, unsigned impure) {
  return trg_resident_bytes(d, dcut, precision, method, impure) +
         trg_workspace_bytes(d, dcut, precision, method, impure);
}

int trg_share_workspace(trg_ctx *ctx, trg_ctx *donor) {
  if (!ctx || !donor) return fail(ctx, TRG_EINVAL, "NULL context");
  if (ctx->st != donor->st) return fail(ctx, TRG_EINVAL, "contexts sharing a workspace must share the stream");
  if ((ctx->cfg.alloc != nullptr) != (donor->cfg.alloc != nullptr))
    return fail(ctx, TRG_EINVAL, "contexts sharing a workspace must both use hipMalloc or both a custom allocator");
  return guarded(ctx, [&]() -> int {
    if (!donor->pool) donor->pool = std::make_shared<WorkspacePool>(donor->cfg);
    TRG_HIP_CHECK(hipStreamSynchronize(ctx->st));
    ctx->pool = donor->pool;
    return TRG_OK;
  });
}

int trg_sync(trg_ctx *ctx) {
  if (!ctx) return fail(nullptr, TRG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() -> int {
    sync_check(*ctx);
    return TRG_OK;
  });
}

void trg_free(trg_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->st);
  for (auto &pr : ctx->join_events) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  auto rel = [&](Buffer &b) {
    ctx->release(b.ptr);
    b.ptr = nullptr;
  };
  rel(ctx->T);
  rel(ctx->Tn);
  for (int j = 0; j < 2; ++j) {
    rel(ctx->S[j]);
    rel(ctx->Sn[j]);
  }
  rel(ctx->G);
  rel(ctx->H);
  rel(ctx->atrg_sigma);
  rel(ctx->dev_scalars);
  rel(ctx->dev_err);
  rel(ctx->dev_rec);
  for (int a = 0; a < 4; ++a) {
    rel(ctx->U[a]);
    rel(ctx->spec[a]);
  }
  ctx->pool.reset();
  delete ctx;
}

const char *trg_last_error(const trg_ctx *ctx) {
  if (ctx) return ctx->err.c_str();
  return g_thread_error.c_str();
}

// ------------------------------------------------- kernel-level entries ---
int trg_gemm(int precision, const void *A, const void *Bt, void *C, long long M, long long N, long long K,
             long long lda, long long ldb, long long ldc, int accumulate, void *stream) {
  return guarded(nullptr, [&]() -> int {
    TRG_REQUIRE(A && Bt && C && M >= 0 && N >= 0 && K >= 0, "bad gemm arguments");
    gemm_nt(precision, A, Bt, C, uint64_t(M), uint64_t(N), uint64_t(K), uint64_t(lda), uint64_t(ldb),
            uint64_t(ldc), accumulate != 0, static_cast<hipStream_t>(stream));
    return TRG_OK;
  });
}

int trg_gemm_tile(int precision, int *tile_m, int *tile_n, int *tile_k) {
  return guarded(nullptr, [&]() -> int {
    const GemmTile t = gemm_tile(precision);
    if (tile_m) *tile_m = t.m;
    if (tile_n) *tile_n = t.n;
    if (tile_k) *tile_k = t.k;
    return TRG_OK;
  });
}

int trg_eigh(double *A, double *w, double *V, int *sweeps, int n, int batch, void *stream) {
  return guarded(nullptr, [&]() -> int {
    TRG_REQUIRE(A && w && V && sweeps, "NULL argument");
    eigh_batched(A, w, V, sweeps, n, batch, static_cast<hipStream_t>(stream));
    return TRG_OK;
  });
}

int trg_eigh_top(double *A, double *w, double *V, int *sweeps, int n, int batch, int k, double cluster_rel,
                 void *work, void *stream) {
  return guarded(nullptr, [&]() -> int {
    TRG_REQUIRE(A && w && V && sweeps, "NULL argument");
    TRG_REQUIRE(n >= 1 && n <= 1024 && batch >= 1 && k >= 1, "eigh_top: bad sizes");
    TRG_REQUIRE(cluster_rel >= 0.0 && cluster_rel < 1.0, "eigh_top: cluster_rel outside [0, 1)");
    TRG_REQUIRE(work || n <= JACOBI_MAX_N, "eigh_top: workspace missing");
    eigh_top_batched(A, w, V, sweeps, n, batch, k, cluster_rel, static_cast<double *>(work),
                     static_cast<hipStream_t>(stream));
    return TRG_OK;
  });
}

size_t trg_eigh_top_work_bytes(int n, int batch) {
  if (n < 1 || n > 1024 || batch < 1) return 0;
  return eigh_top_work_doubles(n, batch) * 8;
}

int trg_set_profiling(trg_ctx *ctx, int on) {
  if (!ctx) return fail(nullptr, TRG_EINVAL, "ctx is NULL");
  ctx->profiling = on != 0;
  return TRG_OK;
}

int trg_join_profile(trg_ctx *ctx, double *ms, long long *launches, double *flops) {
  if (!ctx) return fail(nullptr, TRG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() -> int {
    sync_check(*ctx);
    if (ms) *ms = ctx->join_ms;
    if (launches) *launches = ctx->join_launches;
    if (flops) *flops = ctx->join_flops_done;
    ctx->join_ms = 0.0;
    ctx->join_launches = 0;
    ctx->join_flops_done = 0.0;
    return TRG_OK;
  });
}

int trg_set_force_side(trg_ctx *ctx, int side) {
  if (!ctx) return fail(nullptr, TRG_EINVAL, "ctx is NULL");
  if (side < -1 || side > 1) return fail(ctx, TRG_EINVAL, "side must be -1, 0 or 1");
  ctx->force_side = side;
  return TRG_OK;
}

}  // extern "C"
