// Hierarchical-matrix arithmetic on weak-admissibility (HODLR) plane blocks,
// batched over all planes of a cyclic-reduction level.
//
// The polymorphic operations of Eq. elim (A *_H B, A +_H B, A^{-H}, A *_H b)
// are realised as "exact structured result, then one truncation per produced
// block": every off-diagonal block of a result is first written as a stacked
// low-rank sum [U1 U2 ...][V1 V2 ...]^T that represents it exactly, then
// compressed by Householder QR of both stacks, a one-sided Jacobi SVD of the
// small core and truncation at the relative tolerance (Section 3.1: the
// accuracy is imposed on every block compression and every arithmetic
// operation).  Contributions that reach a block from its ancestors (diagonal
// low-rank terms) are accumulated top-down per segment and truncated at the
// inner tolerance eps * inner_eps_ratio: ratio 1 (the default) truncates them
// like every other operation result; smaller ratios approach one truncation
// per stored block, which indefinite operators need (their Schur complements
// amplify the extra truncation errors).
#include <algorithm>
#include <cstdio>

#include "hodlr.h"

namespace acr {

namespace {

template <class T>
GemmTask gt(const T* A, int64_t lda, int ta, const T* B, int64_t ldb, int tb, T* C, int64_t ldc, int m, int n,
            int k, double alpha, double beta) {
  GemmTask g{};
  g.A = A; g.B = B; g.C = C;
  g.lda = lda; g.ldb = ldb; g.ldc = ldc;
  g.m = m; g.n = n; g.k = k;
  g.ta = ta; g.tb = tb;
  g.alpha = alpha; g.beta = beta;
  return g;
}

template <class T>
CopyTask ctk(const T* src, int64_t lds, T* dst, int64_t ldd, int m, int n, double alpha, int acc,
             const T* rs = nullptr, const T* cs = nullptr) {
  CopyTask c;
  c.src = src; c.dst = dst; c.rs = rs; c.cs = cs;
  c.lds = lds; c.ldd = ldd;
  c.m = m; c.n = n;
  c.accumulate = acc;
  c.alpha = alpha;
  return c;
}

template <class T> struct CJob {
  T* Us;   // m x r stack (destroyed)
  T* Vs;   // n x r stack (destroyed)
  int m, n, r;
  LR<T>* out;
  Arena* arena = nullptr;   // where the truncated factors go (set by compress)
  int max_rank = 0;         // rank cap of this block (0: none)
};

// Householder path: QR of both stacks, Jacobi SVD of the core, Q [Z; 0].
template <class T>
void compress_householder(Exec& ex, std::vector<CJob<T>*>& live, double eps, Arena& tmp) {
  if (live.empty()) return;
  const auto mk = tmp.mark();
  const int nj = (int)live.size();
  std::vector<QrTask> qt;
  std::vector<SvdTask> st;
  int* d_rank = tmp.get_n<int>(nj);
  int* d_tv = tmp.get_n<int>(nj);
  qt.reserve(2 * nj);
  st.reserve(nj);
  std::vector<T*> tau_u(nj), tau_v(nj);
  std::vector<double*> Cw(nj), Yw(nj);
  for (int i = 0; i < nj; ++i) {
    const CJob<T>& j = *live[i];
    const int p = std::min(j.m, j.r), q = std::min(j.n, j.r);
    tau_u[i] = tmp.get_n<T>(p);
    tau_v[i] = tmp.get_n<T>(q);
    Cw[i] = tmp.get_n<double>(2 * (size_t)p * q);
    Yw[i] = tmp.get_n<double>(2 * (size_t)q * q);
    double* sig = tmp.get_n<double>(q);
    qt.push_back(QrTask{j.Us, tau_u[i], j.m, j.m, j.r});
    qt.push_back(QrTask{j.Vs, tau_v[i], j.n, j.n, j.r});
    SvdTask s{};
    s.Ru = j.Us; s.Rv = j.Vs; s.ldu = j.m; s.ldv = j.n;
    s.p = p; s.q = q; s.r = j.r;
    s.C = Cw[i]; s.Y = Yw[i]; s.sig = sig;
    s.rank_out = d_rank + i;
    s.max_rank = j.max_rank;
    s.mode = 0;
    s.perm = tmp.get_n<int>(q);
    s.t_out = d_tv + i;
    st.push_back(s);
  }
  ex.qr<T>(qt);
  ex.svd<T>(st, eps, d_tv);
  std::vector<int> ranks(nj);
  hip_check(hipMemcpyAsync(ranks.data(), d_rank, nj * sizeof(int), hipMemcpyDeviceToHost, ex.stream),
            "hipMemcpyAsync(ranks)");
  ex.sync();
  std::vector<ApplyQTask> at;
  at.reserve(2 * nj);
  for (int i = 0; i < nj; ++i) {
    CJob<T>& j = *live[i];
    const int p = std::min(j.m, j.r), q = std::min(j.n, j.r);
    const int k = ranks[i];
    LR<T> o;
    o.k = k;
    if (k > 0) {
      o.U = j.arena->template get_n<T>((size_t)j.m * k);
      o.V = j.arena->template get_n<T>((size_t)j.n * k);
      ApplyQTask a;
      a.Aq = j.Us; a.tau = tau_u[i]; a.Z = Cw[i] + (size_t)p * q; a.out = o.U;
      a.lda = j.m; a.ldz = p; a.ldo = j.m; a.m = j.m; a.p = p; a.k = k;
      at.push_back(a);
      ApplyQTask b;
      b.Aq = j.Vs; b.tau = tau_v[i]; b.Z = Yw[i] + (size_t)q * q; b.out = o.V;
      b.lda = j.n; b.ldz = q; b.ldo = j.n; b.m = j.n; b.p = q; b.k = k;
      at.push_back(b);
    }
    *j.out = o;
  }
  ex.applyq<T>(at);
  tmp.release(mk);
}

// Gram path for stacks too large for one workgroup (see gram.hip).
template <class T>
void compress_gram(Exec& ex, std::vector<CJob<T>*>& live, double eps, Arena& tmp) {
  if (live.empty()) return;
  const auto mk = tmp.mark();
  const int nj = (int)live.size();
  // directions of a stack below tau * its largest column norm are dropped: their
  // contribution to the block is below tau * ||U|| ||V||, far under eps * sigma_1
  const double tau = std::min(1e-6, 0.01 * eps);
  std::vector<GramTask> gt_;
  std::vector<PcholTask> pc;
  int* d_r1 = tmp.get_n<int>(2 * nj);
  auto chunk_rows = [](int m) { return std::max(256, ((m + 7) / 8 + 31) / 32 * 32); };
  for (int i = 0; i < nj; ++i) {
    const CJob<T>& j = *live[i];
    for (int side = 0; side < 2; ++side) {
      const int m = side ? j.n : j.m, r = j.r;
      GramTask g{};
      g.A = side ? j.Vs : j.Us;
      g.lda = m;
      g.m = m;
      g.r = r;
      g.rows_per_chunk = chunk_rows(m);
      const int nch = (m + g.rows_per_chunk - 1) / g.rows_per_chunk;
      g.part = tmp.get_n<double>((size_t)nch * r * r);
      g.G = tmp.get_n<double>((size_t)r * r);
      gt_.push_back(g);
      PcholTask p{};
      p.G = g.G;
      p.L = tmp.get_n<double>((size_t)r * r);
      p.perm = tmp.get_n<int>(r);
      p.d = tmp.get_n<double>(r);
      p.rank_out = d_r1 + 2 * i + side;
      p.r = r;
      pc.push_back(p);
    }
  }
  ex.gram<T>(gt_);
  ex.pchol(pc, tau * tau);
  std::vector<int> r1(2 * nj);
  hip_check(hipMemcpyAsync(r1.data(), d_r1, r1.size() * sizeof(int), hipMemcpyDeviceToHost, ex.stream),
            "hipMemcpyAsync(gram ranks)");
  ex.sync();
  std::vector<PcholTask> mat;
  std::vector<SvdTask> st;
  std::vector<int> idx;
  int* d_rank = tmp.get_n<int>(nj);
  int* d_tv = tmp.get_n<int>(nj);
  std::vector<double*> Cw(nj, nullptr), Yw(nj, nullptr);
  for (int i = 0; i < nj; ++i) {
    PcholTask& pu = pc[2 * i];
    PcholTask& pv = pc[2 * i + 1];
    pu.r1 = r1[2 * i];
    pv.r1 = r1[2 * i + 1];
    if (pu.r1 == 0 || pv.r1 == 0) continue;
    pu.R = tmp.get_n<double>((size_t)pu.r1 * pu.r);
    pv.R = tmp.get_n<double>((size_t)pv.r1 * pv.r);
    mat.push_back(pu);
    mat.push_back(pv);
    const int p = pu.r1, q = pv.r1;
    Cw[i] = tmp.get_n<double>(2 * (size_t)p * q);
    Yw[i] = tmp.get_n<double>(2 * (size_t)q * q);
    SvdTask s{};
    s.Ru = pu.R; s.Rv = pv.R; s.ldu = p; s.ldv = q;
    s.p = p; s.q = q; s.r = live[i]->r;
    s.C = Cw[i]; s.Y = Yw[i]; s.sig = tmp.get_n<double>(q);
    s.rank_out = d_rank + i;
    s.max_rank = live[i]->max_rank;
    s.mode = 1;
    s.perm = tmp.get_n<int>(q);
    s.t_out = d_tv + st.size();
    st.push_back(s);
    idx.push_back(i);
  }
  ex.materialize_r(mat);
  ex.svd<T>(st, eps, d_tv);
  std::vector<int> rk(nj, 0);
  if (!st.empty()) {
    hip_check(hipMemcpyAsync(rk.data(), d_rank, nj * sizeof(int), hipMemcpyDeviceToHost, ex.stream),
              "hipMemcpyAsync(ranks)");
    ex.sync();
  }
  std::vector<WtTask> wt;
  std::vector<GemmTask> gg;
  std::vector<T*> Wu(nj, nullptr), Wv(nj, nullptr);
  std::vector<char> is_live(nj, 0);
  for (int i : idx) is_live[i] = 1;
  for (int i = 0; i < nj; ++i) {
    CJob<T>& j = *live[i];
    const int k = is_live[i] ? rk[i] : 0;
    LR<T> o;
    o.k = k;
    if (k > 0) {
      const PcholTask& pu = pc[2 * i];
      const PcholTask& pv = pc[2 * i + 1];
      const int p = pu.r1, q = pv.r1, r = j.r;
      Wu[i] = tmp.get_n<T>((size_t)r * k);
      Wv[i] = tmp.get_n<T>((size_t)r * k);
      wt.push_back(WtTask{pu.L, pu.perm, Cw[i] + (size_t)p * q, p, Wu[i], r, p, k});
      wt.push_back(WtTask{pv.L, pv.perm, Yw[i] + (size_t)q * q, q, Wv[i], r, q, k});
      o.U = j.arena->template get_n<T>((size_t)j.m * k);
      o.V = j.arena->template get_n<T>((size_t)j.n * k);
      // the truncated factors are rebuilt in FP32 in every precision variant
      gg.push_back(gt<T>(j.Us, j.m, 0, Wu[i], r, 0, o.U, j.m, j.m, k, r, 1.0, 0.0));
      gg.back().lowp = -1;
      gg.push_back(gt<T>(j.Vs, j.n, 0, Wv[i], r, 0, o.V, j.n, j.n, k, r, 1.0, 0.0));
      gg.back().lowp = -1;
    }
    *j.out = o;
  }
  ex.wtilde<T>(wt);
  ex.gemm<T>(gg);
  tmp.release(mk);
}

// Truncated recompression of stacked low-rank sums (see file comment): the
// Gram path for eps >= 1e-4 (it drops directions below 0.01 eps of the stack
// norm and measured faster than Householder QR for LDS-sized stacks too);
// exact mode and smaller eps use Householder QR.
template <class T>
void compress(Exec& ex, std::vector<CJob<T>>& jobs, double eps, int max_rank, Arena& out, Arena& tmp) {
  std::vector<CJob<T>*> hh, gr;
  for (auto& j : jobs) {
    if (!j.arena) {
      j.arena = &out;
      j.max_rank = max_rank;
    }
    if (j.r == 0 || j.m == 0 || j.n == 0) {
      *j.out = LR<T>{};
      continue;
    }
    (ex.gram_ok && eps >= 1e-4 ? gr : hh).push_back(&j);
  }
  if (ex.trace) {
    int mm = 0, mr = 0;
    double w = 0;
    for (auto& j : jobs) {
      mm = std::max(mm, std::max(j.m, j.n));
      mr = std::max(mr, j.r);
      w += (double)j.r * j.r * (j.m + j.n);
    }
    std::fprintf(stderr, "[acr] compress %s n=%zu hh=%zu gram=%zu max_m=%d max_r=%d work=%.3g\n", ex.trace_tag,
                 jobs.size(), hh.size(), gr.size(), mm, mr, w);
  }
  compress_householder<T>(ex, hh, eps, tmp);
  compress_gram<T>(ex, gr, eps, tmp);
}

// Two independent sets of blocks (outputs to their own arenas, rank caps of
// their own): one compression batch when their tolerances agree, so that the
// pair costs one chain of launches and host round trips instead of two.
template <class T>
void compress2(Exec& ex, std::vector<CJob<T>>& a, double eps_a, int max_rank_a, Arena& out_a,
               std::vector<CJob<T>>& b, double eps_b, int max_rank_b, Arena& out_b, Arena& tmp) {
  if (eps_a != eps_b || a.empty() || b.empty()) {
    compress<T>(ex, a, eps_a, max_rank_a, out_a, tmp);
    compress<T>(ex, b, eps_b, max_rank_b, out_b, tmp);
    return;
  }
  std::vector<CJob<T>> all;
  all.reserve(a.size() + b.size());
  for (auto j : a) {
    j.arena = &out_a;
    j.max_rank = max_rank_a;
    all.push_back(j);
  }
  for (auto j : b) {
    j.arena = &out_b;
    j.max_rank = max_rank_b;
    all.push_back(j);
  }
  compress<T>(ex, all, eps_a, 0, tmp, tmp);
}

inline int nseg(int d) { return 1 << d; }

}  // namespace

template <class T> void hodlr_alloc_leaves(const Tree& tr, HMat<T>& H, Arena& out) {
  H.kind = HMat<T>::HODLR;
  H.diag = nullptr;
  H.leaf.assign(nseg(tr.L), nullptr);
  for (int s = 0; s < nseg(tr.L); ++s) H.leaf[s] = out.get_n<T>((size_t)tr.sz[tr.L][s] * tr.sz[tr.L][s]);
  H.blk.assign(tr.nblk(), LR<T>{});
}

// Y = alpha op(H_{>=dmin}) X + beta Y for every job, where H_{>=dmin} keeps the
// leaves and the blocks of depth >= dmin (the block diagonal of H at depth
// dmin), plus each job's optional diagonal low-rank terms corr[d][t] on the
// segments of depth d + 1 (d >= dmin).
template <class T>
void hodlr_multivec(Exec& ex, const Tree& tr, const std::vector<MVJob<T>>& jobs, bool trans, int dmin,
                    Arena& scratch) {
  const int L = tr.L;
  size_t tot = 0;
  for (auto& j : jobs) {
    if (j.H->kind != HMat<T>::HODLR) continue;
    for (int d = dmin; d < L; ++d)
      for (int s = 0; s < nseg(d + 1); ++s) tot += (size_t)j.H->blk[Tree::bid(d, s)].k * j.c;
    if (j.corr)
      for (int d = dmin; d < (int)j.corr->size(); ++d)
        for (auto& c : (*j.corr)[d]) tot += (size_t)c.k * j.c;
  }
  T* buf = scratch.get_n<T>(std::max<size_t>(tot, 1));
  // per job: pointer to the t of each block / correction
  std::vector<std::vector<T*>> tb(jobs.size());
  std::vector<std::vector<std::vector<T*>>> tcr(jobs.size());  // [job][depth][segment]
  std::vector<GemmTask> inner;
  size_t pos = 0;
  for (size_t ji = 0; ji < jobs.size(); ++ji) {
    const auto& j = jobs[ji];
    if (j.H->kind != HMat<T>::HODLR) continue;
    tb[ji].assign(tr.nblk(), nullptr);
    for (int d = dmin; d < L; ++d)
      for (int s = 0; s < nseg(d + 1); ++s) {
        const LR<T>& b = j.H->blk[Tree::bid(d, s)];
        if (b.k == 0) continue;
        T* t = buf + pos;
        pos += (size_t)b.k * j.c;
        tb[ji][Tree::bid(d, s)] = t;
        const int ro = tr.off[d + 1][s], rn = tr.sz[d + 1][s];
        const int co = tr.off[d + 1][s ^ 1], cn = tr.sz[d + 1][s ^ 1];
        if (!trans)
          inner.push_back(gt<T>(b.V, cn, 1, j.X + co, j.ldx, 0, t, b.k, b.k, j.c, cn, 1.0, 0.0));
        else
          inner.push_back(gt<T>(b.U, rn, 1, j.X + ro, j.ldx, 0, t, b.k, b.k, j.c, rn, 1.0, 0.0));
      }
    if (j.corr) {
      tcr[ji].assign(j.corr->size(), {});
      for (int d = dmin; d < (int)j.corr->size(); ++d)
        for (int s = 0; s < (int)(*j.corr)[d].size(); ++s) {
          const LR<T>& c = (*j.corr)[d][s];
          T* t = nullptr;
          if (c.k > 0) {
            t = buf + pos;
            pos += (size_t)c.k * j.c;
            const int so = tr.off[d + 1][s], sn = tr.sz[d + 1][s];
            inner.push_back(gt<T>(trans ? c.U : c.V, sn, 1, j.X + so, j.ldx, 0, t, c.k, c.k, j.c, sn, 1.0, 0.0));
          }
          tcr[ji][d].push_back(t);
        }
    }
  }
  // Inner products with a long inner dimension (the top blocks: rows = M/2)
  // and several right-hand sides are split into 512-row pieces whose partial
  // products are summed in a fixed order, so that the launch has enough tiles.
  {
    constexpr int kPiece = 512;
    std::vector<GemmTask> direct, pieces;
    std::vector<std::vector<CopyTask>> sums;
    for (const GemmTask& g : inner) {
      const int np = (g.k + kPiece - 1) / kPiece;
      if (np < 2 || g.n < 8 || g.beta != 0.0) {
        direct.push_back(g);
        continue;
      }
      T* part = scratch.get_n<T>((size_t)np * g.m * g.n);
      if ((int)sums.size() < np) sums.resize(np);
      for (int q = 0; q < np; ++q) {
        const int k0 = q * kPiece, kq = std::min(kPiece, g.k - k0);
        GemmTask h = g;
        h.A = static_cast<const T*>(g.A) + (g.ta ? (int64_t)k0 : (int64_t)k0 * g.lda);
        h.B = static_cast<const T*>(g.B) + (g.tb ? (int64_t)k0 * g.ldb : (int64_t)k0);
        h.k = kq;
        h.C = part + (size_t)q * g.m * g.n;
        h.ldc = g.m;
        h.alpha = 1.0;
        h.beta = 0.0;
        pieces.push_back(h);
        sums[q].push_back(ctk<T>(part + (size_t)q * g.m * g.n, g.m, static_cast<T*>(g.C), g.ldc, g.m, g.n,
                                 g.alpha, q > 0 ? 1 : 0));
      }
    }
    direct.insert(direct.end(), pieces.begin(), pieces.end());
    ex.gemm<T>(direct);
    for (auto& c : sums) ex.copy<T>(c);   // piece q added after piece q - 1: fixed order
  }
  // Without correction terms each leaf's rows of Y are formed in one pass: the
  // leaf times X plus every ancestor block's U-slice (V-slice transposed) times
  // its t, concatenated along the inner dimension (Y read and written once).
  bool seg = tr.L - dmin + 1 <= kMaxSeg;
  for (const auto& j : jobs) seg = seg && !j.corr && (j.beta == 0.0 || j.beta == 1.0);
  if (seg) {
    std::vector<SegGemmTask> sg;
    std::vector<CopyTask> dg;
    for (size_t ji = 0; ji < jobs.size(); ++ji) {
      const auto& j = jobs[ji];
      if (j.H->kind == HMat<T>::DIAG) {
        dg.push_back(ctk<T>(j.X, j.ldx, j.Y, j.ldy, tr.M, j.c, j.alpha, j.beta != 0.0, j.H->diag));
        continue;
      }
      if (j.H->kind == HMat<T>::ABSENT) {
        if (j.beta == 0.0) dg.push_back(ctk<T>(nullptr, 0, j.Y, j.ldy, tr.M, j.c, 0.0, 0));
        continue;
      }
      for (int s = 0; s < nseg(L); ++s) {
        const int o = tr.off[L][s], n = tr.sz[L][s];
        SegGemmTask g{};
        g.C = j.Y + o;
        g.ldc = j.ldy;
        g.m = n;
        g.n = j.c;
        g.alpha = j.alpha;
        g.beta = j.beta;
        g.A[0] = j.H->leaf[s];
        g.lda[0] = n;
        g.B[0] = j.X + o;
        g.ldb[0] = j.ldx;
        g.k[0] = n;
        g.ta = trans ? 1u : 0u;
        g.nseg = 1;
        for (int d = dmin; d < L; ++d) {
          // the leaf lies in segment sd of depth d + 1; its rows of H X come from
          // block (d, sd) (U rows) or, transposed, block (d, sd ^ 1) (V rows)
          const int sd = s >> (L - (d + 1));
          const int bs = trans ? (sd ^ 1) : sd;
          const LR<T>& b = j.H->blk[Tree::bid(d, bs)];
          if (b.k == 0) continue;
          const int so = tr.off[d + 1][sd], sn = tr.sz[d + 1][sd];
          g.A[g.nseg] = (trans ? b.V : b.U) + (o - so);
          g.lda[g.nseg] = sn;
          g.B[g.nseg] = tb[ji][Tree::bid(d, bs)];
          g.ldb[g.nseg] = b.k;
          g.k[g.nseg] = b.k;
          ++g.nseg;
        }
        sg.push_back(g);
      }
    }
    ex.seg_gemm<T>(sg);
    ex.copy<T>(dg);
    return;
  }
  std::vector<GemmTask> lv;
  std::vector<CopyTask> dg;
  for (const auto& j : jobs) {
    if (j.H->kind == HMat<T>::DIAG) {
      dg.push_back(ctk<T>(j.X, j.ldx, j.Y, j.ldy, tr.M, j.c, j.alpha, j.beta != 0.0, j.H->diag));
    } else if (j.H->kind == HMat<T>::ABSENT) {
      if (j.beta == 0.0) dg.push_back(ctk<T>(nullptr, 0, j.Y, j.ldy, tr.M, j.c, 0.0, 0));
    } else {
      for (int s = 0; s < nseg(L); ++s) {
        const int o = tr.off[L][s], n = tr.sz[L][s];
        lv.push_back(gt<T>(j.H->leaf[s], n, trans ? 1 : 0, j.X + o, j.ldx, 0, j.Y + o, j.ldy, n, j.c, n, j.alpha,
                           j.beta));
      }
    }
  }
  ex.gemm<T>(lv);
  ex.copy<T>(dg);
  for (int d = dmin; d < L; ++d) {
    std::vector<GemmTask> ap, apc;
    for (size_t ji = 0; ji < jobs.size(); ++ji) {
      const auto& j = jobs[ji];
      if (j.H->kind != HMat<T>::HODLR) continue;
      for (int s = 0; s < nseg(d + 1); ++s) {
        const LR<T>& b = j.H->blk[Tree::bid(d, s)];
        if (b.k == 0) continue;
        const T* t = tb[ji][Tree::bid(d, s)];
        const int ro = tr.off[d + 1][s], rn = tr.sz[d + 1][s];
        const int co = tr.off[d + 1][s ^ 1], cn = tr.sz[d + 1][s ^ 1];
        if (!trans)
          ap.push_back(gt<T>(b.U, rn, 0, t, b.k, 0, j.Y + ro, j.ldy, rn, j.c, b.k, j.alpha, 1.0));
        else
          ap.push_back(gt<T>(b.V, cn, 0, t, b.k, 0, j.Y + co, j.ldy, cn, j.c, b.k, j.alpha, 1.0));
      }
      if (j.corr && d < (int)j.corr->size()) {
        for (int s = 0; s < (int)(*j.corr)[d].size(); ++s) {
          const LR<T>& c = (*j.corr)[d][s];
          if (c.k == 0) continue;
          const int so = tr.off[d + 1][s], sn = tr.sz[d + 1][s];
          apc.push_back(gt<T>(trans ? c.V : c.U, sn, 0, tcr[ji][d][s], c.k, 0, j.Y + so, j.ldy, sn, j.c, c.k, j.alpha,
                              1.0));
        }
      }
    }
    ex.gemm<T>(ap);
    ex.gemm<T>(apc);
  }
}

// ---------------------------------------------------------------- inverse
//
// Bottom-up block inversion.  With B_{d+1} the block diagonal of D at depth
// d + 1 and O_d the off-diagonal blocks of depth d, each node satisfies
//   inv(B + U W^T) = inv(B) - inv(B) U (I + W^T inv(B) U)^{-1} W^T inv(B)
// (Sherman-Morrison-Woodbury), which yields per node the two new off-diagonal
// blocks and one low-rank correction on each child.  The corrections are
// pushed down into the deeper blocks and the leaves at the end.
template <class T>
void hodlr_inverse(Exec& ex, const Tree& tr, const std::vector<const HMat<T>*>& D,
                   const std::vector<HMat<T>*>& G, const Trunc& tc, Arena& out, Arena& work, Arena& tmp) {
  const int L = tr.L, M = tr.M;
  const int np = (int)D.size();
  const auto wmark = work.mark();
  // leaves
  {
    std::vector<CopyTask> cp;
    std::vector<InvTask> iv;
    for (int p = 0; p < np; ++p) {
      hodlr_alloc_leaves(tr, *G[p], out);
      for (int s = 0; s < nseg(L); ++s) {
        const int n = tr.sz[L][s];
        cp.push_back(ctk<T>(D[p]->leaf[s], n, G[p]->leaf[s], n, n, n, 1.0, 0));
        iv.push_back(InvTask{G[p]->leaf[s], n, n, 0});
      }
    }
    ex.copy<T>(cp);
    ex.inverse<T>(iv);
  }
  // state: off-diagonal blocks g (by block id) and corrections c[d][t]
  std::vector<std::vector<LR<T>>> g(np, std::vector<LR<T>>(tr.nblk()));
  std::vector<std::vector<std::vector<LR<T>>>> corr(np);
  for (int p = 0; p < np; ++p) {
    corr[p].assign(std::max(L - 1, 0), {});
    for (int d = 0; d + 1 < L; ++d) corr[p][d].assign(nseg(d + 1), LR<T>{});
  }
  std::vector<HMat<T>> cur(np);
  for (int p = 0; p < np; ++p) {
    cur[p].kind = HMat<T>::HODLR;
    cur[p].leaf = G[p]->leaf;
    cur[p].blk.assign(tr.nblk(), LR<T>{});
  }
  for (int d = L - 1; d >= 0; --d) {
    const auto tm = tmp.mark();
    // flat bases of depth d: Xu rows of s <- U_{d,s}; Xv rows of t <- V_{d,t^1}
    std::vector<int> K(np, 0);
    std::vector<T*> Xu(np), Xv(np), P(np), Q(np);
    std::vector<CopyTask> cp;
    std::vector<MVJob<T>> mv, mvt;
    for (int p = 0; p < np; ++p) {
      for (int s = 0; s < nseg(d + 1); ++s) K[p] = std::max(K[p], D[p]->blk[Tree::bid(d, s)].k);
      if (K[p] == 0) continue;
      Xu[p] = tmp.get_n<T>((size_t)M * K[p]);
      Xv[p] = tmp.get_n<T>((size_t)M * K[p]);
      P[p] = tmp.get_n<T>((size_t)M * K[p]);
      Q[p] = tmp.get_n<T>((size_t)M * K[p]);
      cp.push_back(ctk<T>(nullptr, 0, Xu[p], M, M, K[p], 0.0, 0));
      cp.push_back(ctk<T>(nullptr, 0, Xv[p], M, M, K[p], 0.0, 0));
    }
    ex.copy<T>(cp);
    cp.clear();
    for (int p = 0; p < np; ++p) {
      if (K[p] == 0) continue;
      for (int s = 0; s < nseg(d + 1); ++s) {
        const LR<T>& b = D[p]->blk[Tree::bid(d, s)];
        if (b.k == 0) continue;
        const int ro = tr.off[d + 1][s], rn = tr.sz[d + 1][s];
        const int co = tr.off[d + 1][s ^ 1], cn = tr.sz[d + 1][s ^ 1];
        cp.push_back(ctk<T>(b.U, rn, Xu[p] + ro, M, rn, b.k, 1.0, 0));
        cp.push_back(ctk<T>(b.V, cn, Xv[p] + co, M, cn, b.k, 1.0, 0));
      }
      mv.push_back(MVJob<T>{&cur[p], &corr[p], Xu[p], M, P[p], M, K[p], 1.0, 0.0});
      mvt.push_back(MVJob<T>{&cur[p], &corr[p], Xv[p], M, Q[p], M, K[p], 1.0, 0.0});
    }
    ex.copy<T>(cp);
    hodlr_multivec<T>(ex, tr, mv, false, d + 1, tmp);
    hodlr_multivec<T>(ex, tr, mvt, true, d + 1, tmp);
    // capacitance matrices per node
    struct Node { int p, b, k12, k21; T* K; };
    std::vector<Node> nodes;
    std::vector<CopyTask> eye;
    std::vector<GemmTask> kg;
    std::vector<InvTask> kinv;
    for (int p = 0; p < np; ++p) {
      if (K[p] == 0) continue;
      for (int b = 0; b < nseg(d); ++b) {
        const int s1 = 2 * b, s2 = 2 * b + 1;
        const LR<T>& B12 = D[p]->blk[Tree::bid(d, s1)];
        const LR<T>& B21 = D[p]->blk[Tree::bid(d, s2)];
        const int k12 = B12.k, k21 = B21.k, kk = k12 + k21;
        if (kk == 0) continue;
        T* Km = tmp.get_n<T>((size_t)kk * kk);
        nodes.push_back(Node{p, b, k12, k21, Km});
        eye.push_back(ctk<T>(nullptr, 0, Km, kk, kk, kk, 1.0, 0));
        const int o1 = tr.off[d + 1][s1], n1 = tr.sz[d + 1][s1];
        const int o2 = tr.off[d + 1][s2], n2 = tr.sz[d + 1][s2];
        if (k12 && k21) {
          kg.push_back(gt<T>(B12.V, n2, 1, P[p] + o2, M, 0, Km + (size_t)k12 * kk, kk, k12, k21, n2, 1.0, 0.0));
          kg.push_back(gt<T>(B21.V, n1, 1, P[p] + o1, M, 0, Km + k12, kk, k21, k12, n1, 1.0, 0.0));
        }
        kinv.push_back(InvTask{Km, kk, kk, 0});
      }
    }
    ex.copy<T>(eye);
    ex.gemm<T>(kg);
    ex.inverse<T>(kinv);
    // stacks of the new off-diagonal blocks and of the child corrections
    std::vector<CJob<T>> gj, cj;
    std::vector<GemmTask> sg;
    std::vector<CopyTask> sc;
    std::vector<GemmTask> leafupd;
    for (const Node& nd : nodes) {
      const int p = nd.p, s1 = 2 * nd.b, s2 = s1 + 1, k12 = nd.k12, k21 = nd.k21, kk = k12 + k21;
      const int o1 = tr.off[d + 1][s1], n1 = tr.sz[d + 1][s1];
      const int o2 = tr.off[d + 1][s2], n2 = tr.sz[d + 1][s2];
      T* Km = nd.K;
      // block (d, s1) = -P1 K11 Q2^T ; block (d, s2) = -P2 K22 Q1^T
      if (k12) {
        T* Us = tmp.get_n<T>((size_t)n1 * k12);
        T* Vs = tmp.get_n<T>((size_t)n2 * k12);
        sg.push_back(gt<T>(P[p] + o1, M, 0, Km, kk, 0, Us, n1, n1, k12, k12, -1.0, 0.0));
        sc.push_back(ctk<T>(Q[p] + o2, M, Vs, n2, n2, k12, 1.0, 0));
        gj.push_back(CJob<T>{Us, Vs, n1, n2, k12, &g[p][Tree::bid(d, s1)]});
      }
      if (k21) {
        T* Us = tmp.get_n<T>((size_t)n2 * k21);
        T* Vs = tmp.get_n<T>((size_t)n1 * k21);
        sg.push_back(gt<T>(P[p] + o2, M, 0, Km + k12 + (size_t)k12 * kk, kk, 0, Us, n2, n2, k21, k21, -1.0, 0.0));
        sc.push_back(ctk<T>(Q[p] + o1, M, Vs, n1, n1, k21, 1.0, 0));
        gj.push_back(CJob<T>{Us, Vs, n2, n1, k21, &g[p][Tree::bid(d, s2)]});
      }
      // corrections: on s1: -P1 K12 Q1^T (rank k21); on s2: -P2 K21 Q2^T (rank k12)
      if (k12 && k21) {
        T* U1 = tmp.get_n<T>((size_t)n1 * k21);
        T* V1 = tmp.get_n<T>((size_t)n1 * k21);
        sg.push_back(gt<T>(P[p] + o1, M, 0, Km + (size_t)k12 * kk, kk, 0, U1, n1, n1, k21, k12, -1.0, 0.0));
        sc.push_back(ctk<T>(Q[p] + o1, M, V1, n1, n1, k21, 1.0, 0));
        T* U2 = tmp.get_n<T>((size_t)n2 * k12);
        T* V2 = tmp.get_n<T>((size_t)n2 * k12);
        sg.push_back(gt<T>(P[p] + o2, M, 0, Km + k12, kk, 0, U2, n2, n2, k12, k21, -1.0, 0.0));
        sc.push_back(ctk<T>(Q[p] + o2, M, V2, n2, n2, k12, 1.0, 0));
        if (d == L - 1) {
          // children are leaves: add the corrections to the dense inverses directly
          leafupd.push_back(gt<T>(U1, n1, 0, V1, n1, 1, G[p]->leaf[s1], n1, n1, n1, k21, 1.0, 1.0));
          leafupd.push_back(gt<T>(U2, n2, 0, V2, n2, 1, G[p]->leaf[s2], n2, n2, n2, k12, 1.0, 1.0));
        } else {
          cj.push_back(CJob<T>{U1, V1, n1, n1, k21, &corr[p][d][s1]});
          cj.push_back(CJob<T>{U2, V2, n2, n2, k12, &corr[p][d][s2]});
        }
      }
    }
    ex.gemm<T>(sg);
    ex.copy<T>(sc);
    ex.gemm<T>(leafupd);
    // depth-0 blocks are final; deeper ones are intermediate until the push-down
    compress2<T>(ex, gj, d == 0 ? tc.eps : tc.eps_inner, d == 0 ? tc.max_rank : 0, d == 0 ? out : work, cj,
                 tc.eps_inner, 0, work, tmp);
    for (int p = 0; p < np; ++p)
      for (int s = 0; s < nseg(d + 1); ++s) cur[p].blk[Tree::bid(d, s)] = g[p][Tree::bid(d, s)];
    tmp.release(tm);
  }
  for (int p = 0; p < np; ++p)
    for (int s = 0; s < (L > 0 ? 2 : 0); ++s) G[p]->blk[Tree::bid(0, s)] = g[p][Tree::bid(0, s)];
  // push-down of the corrections: acc on segments of depth d (from corrections
  // of depths < d) joins the blocks of depth d and the next accumulator
  std::vector<std::vector<LR<T>>> acc(np);
  for (int p = 0; p < np; ++p)
    if (L >= 2) acc[p] = corr[p][0];
  for (int d = 1; d < L; ++d) {
    const auto tm = tmp.mark();
    std::vector<CJob<T>> bj, aj;
    std::vector<CopyTask> sc;
    std::vector<GemmTask> leafupd;
    std::vector<std::vector<LR<T>>> nacc(np);
    for (int p = 0; p < np; ++p) {
      if (d + 1 < L) nacc[p].assign(nseg(d + 1), LR<T>{});
      for (int s = 0; s < nseg(d + 1); ++s) {
        const int par = s >> 1;
        const LR<T>& a = acc[p][par];
        const LR<T>& gb = g[p][Tree::bid(d, s)];
        const int ro = tr.off[d + 1][s] - tr.off[d][par], rn = tr.sz[d + 1][s];
        const int co = tr.off[d + 1][s ^ 1] - tr.off[d][par], cn = tr.sz[d + 1][s ^ 1];
        const int pn = tr.sz[d][par];
        // final block (d, s)
        const int r = gb.k + a.k;
        if (r > 0) {
          T* Us = tmp.get_n<T>((size_t)rn * r);
          T* Vs = tmp.get_n<T>((size_t)cn * r);
          if (gb.k) {
            sc.push_back(ctk<T>(gb.U, rn, Us, rn, rn, gb.k, 1.0, 0));
            sc.push_back(ctk<T>(gb.V, cn, Vs, cn, cn, gb.k, 1.0, 0));
          }
          if (a.k) {
            sc.push_back(ctk<T>(a.U + ro, pn, Us + (size_t)rn * gb.k, rn, rn, a.k, 1.0, 0));
            sc.push_back(ctk<T>(a.V + co, pn, Vs + (size_t)cn * gb.k, cn, cn, a.k, 1.0, 0));
          }
          bj.push_back(CJob<T>{Us, Vs, rn, cn, r, &G[p]->blk[Tree::bid(d, s)]});
        } else {
          G[p]->blk[Tree::bid(d, s)] = LR<T>{};
        }
        if (d + 1 < L) {
          const LR<T>& c = corr[p][d][s];
          const int ra = c.k + a.k;
          if (ra > 0) {
            T* Us = tmp.get_n<T>((size_t)rn * ra);
            T* Vs = tmp.get_n<T>((size_t)rn * ra);
            if (c.k) {
              sc.push_back(ctk<T>(c.U, rn, Us, rn, rn, c.k, 1.0, 0));
              sc.push_back(ctk<T>(c.V, rn, Vs, rn, rn, c.k, 1.0, 0));
            }
            if (a.k) {
              sc.push_back(ctk<T>(a.U + ro, pn, Us + (size_t)rn * c.k, rn, rn, a.k, 1.0, 0));
              sc.push_back(ctk<T>(a.V + ro, pn, Vs + (size_t)rn * c.k, rn, rn, a.k, 1.0, 0));
            }
            aj.push_back(CJob<T>{Us, Vs, rn, rn, ra, &nacc[p][s]});
          }
        } else if (a.k) {
          leafupd.push_back(gt<T>(a.U + ro, pn, 0, a.V + ro, pn, 1, G[p]->leaf[s], rn, rn, rn, a.k, 1.0, 1.0));
        }
      }
    }
    ex.copy<T>(sc);
    ex.gemm<T>(leafupd);
    compress2<T>(ex, bj, tc.eps, tc.max_rank, out, aj, tc.eps_inner, 0, work, tmp);
    // the new accumulators live in `work`, so only the stacks are released
    tmp.release(tm);
    if (d + 1 < L) acc = std::move(nacc);
  }
  work.release(wmark);
}

// ---------------------------------------------------------------- product
//
// C = alpha A B.  With A, B in HODLR form, the block (d, s) of the product is
//   A[s,s] U^B_{d,s} V^B_{d,s}^T + U^A_{d,s} (B[s',s']^T V^A_{d,s})^T
//   + (terms from the ancestors' off-diagonal blocks),
// where the ancestor of depth d0 contributes on each child segment t the
// diagonal term U^A_{d0,t} (V^A_{d0,t}^T U^B_{d0,t'}) V^B_{d0,t'}^T.  A
// diagonal factor (the level-0 couplings) scales rows or columns instead.
template <class T>
void hodlr_product(Exec& ex, const Tree& tr, const std::vector<ProdJob<T>>& jobs, const Trunc& tc,
                   Arena& out, Arena& work, Arena& tmp) {
  const int L = tr.L, M = tr.M;
  const auto wmark = work.mark();
  std::vector<const ProdJob<T>*> gen, dia;
  for (auto& j : jobs) {
    if (j.A->absent() || j.B->absent()) {
      *j.C = HMat<T>{};
      continue;
    }
    if (j.A->kind == HMat<T>::DIAG && j.B->kind == HMat<T>::DIAG)
      throw Failure(ST_NOT_SUPPORTED, "product of two diagonal blocks");
    (j.A->kind == HMat<T>::DIAG || j.B->kind == HMat<T>::DIAG ? dia : gen).push_back(&j);
  }
  // -- diagonal factor: scaled copy, then truncation of every block
  if (!dia.empty()) {
    const auto tm = tmp.mark();
    std::vector<CopyTask> cp;
    std::vector<CJob<T>> cj;
    for (const auto* j : dia) {
      const bool left = j->A->kind == HMat<T>::DIAG;
      const HMat<T>& H = left ? *j->B : *j->A;
      const T* dv = left ? j->A->diag : j->B->diag;
      hodlr_alloc_leaves(tr, *j->C, out);
      for (int s = 0; s < nseg(L); ++s) {
        const int o = tr.off[L][s], n = tr.sz[L][s];
        cp.push_back(ctk<T>(H.leaf[s], n, j->C->leaf[s], n, n, n, j->alpha, 0, left ? dv + o : nullptr,
                            left ? nullptr : dv + o));
      }
      for (int d = 0; d < L; ++d)
        for (int s = 0; s < nseg(d + 1); ++s) {
          const LR<T>& b = H.blk[Tree::bid(d, s)];
          if (b.k == 0) continue;
          const int ro = tr.off[d + 1][s], rn = tr.sz[d + 1][s];
          const int co = tr.off[d + 1][s ^ 1], cn = tr.sz[d + 1][s ^ 1];
          T* Us = tmp.get_n<T>((size_t)rn * b.k);
          T* Vs = tmp.get_n<T>((size_t)cn * b.k);
          cp.push_back(ctk<T>(b.U, rn, Us, rn, rn, b.k, j->alpha, 0, left ? dv + ro : nullptr));
          cp.push_back(ctk<T>(b.V, cn, Vs, cn, cn, b.k, 1.0, 0, left ? nullptr : dv + co));
          cj.push_back(CJob<T>{Us, Vs, rn, cn, b.k, &j->C->blk[Tree::bid(d, s)]});
        }
    }
    ex.copy<T>(cp);
    compress<T>(ex, cj, tc.eps, tc.max_rank, out, tmp);
    tmp.release(tm);
  }
  if (gen.empty()) {
    work.release(wmark);
    return;
  }
  const int nj = (int)gen.size();
  // leaves: C_l = alpha A_l B_l
  {
    std::vector<GemmTask> lg;
    for (const auto* j : gen) {
      hodlr_alloc_leaves(tr, *j->C, out);
      for (int s = 0; s < nseg(L); ++s) {
        const int n = tr.sz[L][s];
        lg.push_back(gt<T>(j->A->leaf[s], n, 0, j->B->leaf[s], n, 0, j->C->leaf[s], n, n, n, n, j->alpha, 0.0));
        lg.back().lowp = ex.leaf_lowp;
      }
    }
    ex.gemm<T>(lg);
  }
  std::vector<std::vector<LR<T>>> acc(nj);  // accumulators on segments of depth d
  for (int d = 0; d < L; ++d) {
    const auto tm = tmp.mark();
    std::vector<int> Kb(nj, 0), Ka(nj, 0);
    std::vector<T*> Xu(nj, nullptr), Xv(nj, nullptr), PU(nj, nullptr), QV(nj, nullptr);
    std::vector<CopyTask> cp;
    for (int i = 0; i < nj; ++i) {
      for (int s = 0; s < nseg(d + 1); ++s) {
        Kb[i] = std::max(Kb[i], gen[i]->B->blk[Tree::bid(d, s)].k);
        Ka[i] = std::max(Ka[i], gen[i]->A->blk[Tree::bid(d, s)].k);
      }
      if (Kb[i]) {
        Xu[i] = tmp.get_n<T>((size_t)M * Kb[i]);
        PU[i] = tmp.get_n<T>((size_t)M * Kb[i]);
        cp.push_back(ctk<T>(nullptr, 0, Xu[i], M, M, Kb[i], 0.0, 0));
      }
      if (Ka[i]) {
        Xv[i] = tmp.get_n<T>((size_t)M * Ka[i]);
        QV[i] = tmp.get_n<T>((size_t)M * Ka[i]);
        cp.push_back(ctk<T>(nullptr, 0, Xv[i], M, M, Ka[i], 0.0, 0));
      }
    }
    ex.copy<T>(cp);
    cp.clear();
    std::vector<MVJob<T>> mu, mvv;
    for (int i = 0; i < nj; ++i) {
      for (int s = 0; s < nseg(d + 1); ++s) {
        const LR<T>& bb = gen[i]->B->blk[Tree::bid(d, s)];
        const LR<T>& ab = gen[i]->A->blk[Tree::bid(d, s)];
        const int ro = tr.off[d + 1][s], rn = tr.sz[d + 1][s];
        const int co = tr.off[d + 1][s ^ 1], cn = tr.sz[d + 1][s ^ 1];
        if (bb.k) cp.push_back(ctk<T>(bb.U, rn, Xu[i] + ro, M, rn, bb.k, 1.0, 0));
        if (ab.k) cp.push_back(ctk<T>(ab.V, cn, Xv[i] + co, M, cn, ab.k, 1.0, 0));
      }
      if (Kb[i]) mu.push_back(MVJob<T>{gen[i]->A, nullptr, Xu[i], M, PU[i], M, Kb[i], 1.0, 0.0});
      if (Ka[i]) mvv.push_back(MVJob<T>{gen[i]->B, nullptr, Xv[i], M, QV[i], M, Ka[i], 1.0, 0.0});
    }
    ex.copy<T>(cp);
    hodlr_multivec<T>(ex, tr, mu, false, d + 1, tmp);
    hodlr_multivec<T>(ex, tr, mvv, true, d + 1, tmp);
    // own stacks (+ accumulator of the parent segment) of the blocks of depth d,
    // and diagonal terms of depth d on the child segments
    std::vector<CJob<T>> bj, aj;
    std::vector<CopyTask> sc;
    std::vector<GemmTask> wg, zg, leafupd;
    std::vector<std::vector<LR<T>>> nacc(nj);
    for (int i = 0; i < nj; ++i) {
      const ProdJob<T>& j = *gen[i];
      if (d + 1 < L) nacc[i].assign(nseg(d + 1), LR<T>{});
      for (int s = 0; s < nseg(d + 1); ++s) {
        const LR<T>& bb = j.B->blk[Tree::bid(d, s)];
        const LR<T>& ab = j.A->blk[Tree::bid(d, s)];
        const int ro = tr.off[d + 1][s], rn = tr.sz[d + 1][s];
        const int co = tr.off[d + 1][s ^ 1], cn = tr.sz[d + 1][s ^ 1];
        LR<T> a{};
        int pro = 0, pco = 0, pn = 0;
        if (d > 0) {
          const int par = s >> 1;
          a = acc[i][par];
          pro = tr.off[d + 1][s] - tr.off[d][par];
          pco = tr.off[d + 1][s ^ 1] - tr.off[d][par];
          pn = tr.sz[d][par];
        }
        const int r = bb.k + ab.k + a.k;
        if (r > 0) {
          T* Us = tmp.get_n<T>((size_t)rn * r);
          T* Vs = tmp.get_n<T>((size_t)cn * r);
          int c0 = 0;
          if (bb.k) {
            sc.push_back(ctk<T>(PU[i] + ro, M, Us, rn, rn, bb.k, j.alpha, 0));
            sc.push_back(ctk<T>(bb.V, cn, Vs, cn, cn, bb.k, 1.0, 0));
            c0 += bb.k;
          }
          if (ab.k) {
            sc.push_back(ctk<T>(ab.U, rn, Us + (size_t)rn * c0, rn, rn, ab.k, j.alpha, 0));
            sc.push_back(ctk<T>(QV[i] + co, M, Vs + (size_t)cn * c0, cn, cn, ab.k, 1.0, 0));
            c0 += ab.k;
          }
          if (a.k) {
            sc.push_back(ctk<T>(a.U + pro, pn, Us + (size_t)rn * c0, rn, rn, a.k, 1.0, 0));
            sc.push_back(ctk<T>(a.V + pco, pn, Vs + (size_t)cn * c0, cn, cn, a.k, 1.0, 0));
          }
          bj.push_back(CJob<T>{Us, Vs, rn, cn, r, &j.C->blk[Tree::bid(d, s)]});
        } else {
          j.C->blk[Tree::bid(d, s)] = LR<T>{};
        }
        // diagonal term on segment s: U^A_{d,s} (V^A_{d,s}^T U^B_{d,s^1}) V^B_{d,s^1}^T
        const LR<T>& bs = j.B->blk[Tree::bid(d, s ^ 1)];
        const int kz = (ab.k && bs.k) ? bs.k : 0;
        const int ra = kz + a.k;
        if (ra == 0) continue;
        T* Zu = tmp.get_n<T>((size_t)rn * ra);
        T* Zv = tmp.get_n<T>((size_t)rn * ra);
        if (kz) {
          T* W = tmp.get_n<T>((size_t)ab.k * kz);
          wg.push_back(gt<T>(ab.V, cn, 1, bs.U, cn, 0, W, ab.k, ab.k, kz, cn, 1.0, 0.0));
          zg.push_back(gt<T>(ab.U, rn, 0, W, ab.k, 0, Zu, rn, rn, kz, ab.k, j.alpha, 0.0));
          sc.push_back(ctk<T>(bs.V, rn, Zv, rn, rn, kz, 1.0, 0));
        }
        if (a.k) {
          sc.push_back(ctk<T>(a.U + pro, pn, Zu + (size_t)rn * kz, rn, rn, a.k, 1.0, 0));
          sc.push_back(ctk<T>(a.V + pro, pn, Zv + (size_t)rn * kz, rn, rn, a.k, 1.0, 0));
        }
        if (d + 1 < L)
          aj.push_back(CJob<T>{Zu, Zv, rn, rn, ra, &nacc[i][s]});
        else
          leafupd.push_back(gt<T>(Zu, rn, 0, Zv, rn, 1, j.C->leaf[s], rn, rn, rn, ra, 1.0, 1.0));
      }
    }
    ex.gemm<T>(wg);
    ex.gemm<T>(zg);
    ex.copy<T>(sc);
    ex.gemm<T>(leafupd);
    compress2<T>(ex, bj, tc.eps, tc.max_rank, out, aj, tc.eps_inner, 0, work, tmp);
    tmp.release(tm);
    if (d + 1 < L) acc = std::move(nacc);
  }
  work.release(wmark);
}

// ---------------------------------------------------------------- sum
template <class T>
void hodlr_sum(Exec& ex, const Tree& tr, const std::vector<SumJob<T>>& jobs, const Trunc& tc, Arena& out,
               Arena& tmp) {
  const int L = tr.L;
  const auto tm = tmp.mark();
  // leaves: the first present term is copied, every further term is added in
  // a launch of its own (tasks of one launch must not share a destination)
  std::vector<CopyTask> cp;
  std::vector<std::vector<CopyTask>> ca;
  std::vector<CJob<T>> cj;
  for (const auto& j : jobs) {
    hodlr_alloc_leaves(tr, *j.C, out);
    int nth = 0;
    for (const auto& term : j.terms) {
      const HMat<T>* H = term.first;
      if (H->absent()) continue;
      if (H->kind != HMat<T>::HODLR) throw Failure(ST_NOT_SUPPORTED, "sum of a diagonal block");
      if (nth > 0 && (int)ca.size() < nth) ca.resize(nth);
      for (int s = 0; s < nseg(L); ++s) {
        const int n = tr.sz[L][s];
        const CopyTask t = ctk<T>(H->leaf[s], n, j.C->leaf[s], n, n, n, term.second, nth > 0 ? 1 : 0);
        if (nth == 0) cp.push_back(t); else ca[nth - 1].push_back(t);
      }
      ++nth;
    }
    if (nth == 0) throw Failure(ST_INVALID, "empty sum");
    for (int d = 0; d < L; ++d)
      for (int s = 0; s < nseg(d + 1); ++s) {
        int r = 0;
        for (const auto& term : j.terms)
          if (!term.first->absent()) r += term.first->blk[Tree::bid(d, s)].k;
        const int rn = tr.sz[d + 1][s], cn = tr.sz[d + 1][s ^ 1];
        if (r == 0) {
          j.C->blk[Tree::bid(d, s)] = LR<T>{};
          continue;
        }
        T* Us = tmp.get_n<T>((size_t)rn * r);
        T* Vs = tmp.get_n<T>((size_t)cn * r);
        int c0 = 0;
        for (const auto& term : j.terms) {
          if (term.first->absent()) continue;
          const LR<T>& b = term.first->blk[Tree::bid(d, s)];
          if (!b.k) continue;
          cp.push_back(ctk<T>(b.U, rn, Us + (size_t)rn * c0, rn, rn, b.k, term.second, 0));
          cp.push_back(ctk<T>(b.V, cn, Vs + (size_t)cn * c0, cn, cn, b.k, 1.0, 0));
          c0 += b.k;
        }
        cj.push_back(CJob<T>{Us, Vs, rn, cn, r, &j.C->blk[Tree::bid(d, s)]});
      }
  }
  ex.copy<T>(cp);
  for (auto& a : ca) ex.copy<T>(a);
  compress<T>(ex, cj, tc.eps, tc.max_rank, out, tmp);
  tmp.release(tm);
}

#define ACR_OPS_INST(T)                                                                                        \
  template void hodlr_alloc_leaves<T>(const Tree&, HMat<T>&, Arena&);                                           \
  template void hodlr_multivec<T>(Exec&, const Tree&, const std::vector<MVJob<T>>&, bool, int, Arena&);         \
  template void hodlr_inverse<T>(Exec&, const Tree&, const std::vector<const HMat<T>*>&,                        \
                                 const std::vector<HMat<T>*>&, const Trunc&, Arena&, Arena&, Arena&);           \
  template void hodlr_product<T>(Exec&, const Tree&, const std::vector<ProdJob<T>>&, const Trunc&, Arena&,      \
                                 Arena&, Arena&);                                                               \
  template void hodlr_sum<T>(Exec&, const Tree&, const std::vector<SumJob<T>>&, const Trunc&, Arena&, Arena&);
ACR_OPS_INST(float)
ACR_OPS_INST(double)
#undef ACR_OPS_INST

}  // namespace acr
