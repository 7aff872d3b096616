// Host construction of the H-IDBF (hierarchical interpolative decomposition
// butterfly factorisation) of the 2D TM_z EFIE impedance matrix.
//
//  * entries: paper Sec. 3.1 (off-diagonal Hankel entries with the source
//    segment length, closed-form self term), plus an optional diag(z);
//  * hierarchy (Algorithm 1): recursive 2x2 split down to leaves of n0;
//    every off-diagonal block of size N/2^v is compressed by an IDBF with
//    L = log2(N/n0) - v levels (weak admissibility, Sec. 3.2.1); L = 0 blocks
//    and the diagonal leaves stay dense;
//  * IDBF of one block (appendix): linear-scaling column/row IDs (pivoted QR
//    of a Mock-Chebyshev sample of the partner index set), LRCS, MSCS and the
//    recursive MSCS.  After d splits the row IDs pair row nodes of level
//    L-d+1 with column nodes of level d (and symmetrically for the column
//    IDs); the recursion runs d = 1..D, D = ceil(L/2), and the remaining
//    coupling factor holds dense blocks of the kernel restricted to the last
//    row and column skeletons.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <thread>

#include "hbf_internal.h"

namespace hbf {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;

void parallel_for(int64_t n, int nthreads, const std::function<void(int64_t)>& fn) {
  if (n <= 0) return;
  const int T = static_cast<int>(std::min<int64_t>(n, std::max(1, nthreads)));
  if (T == 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int64_t> next(0);
  std::vector<std::thread> th;
  std::exception_ptr err = nullptr;
  std::atomic<bool> failed(false);
  for (int t = 0; t < T; ++t) {
    th.emplace_back([&]() {
      try {
        for (;;) {
          if (failed.load()) return;
          const int64_t i = next.fetch_add(1);
          if (i >= n) return;
          fn(i);
        }
      } catch (...) {
        if (!failed.exchange(true)) err = std::current_exception();
      }
    });
  }
  for (auto& x : th) x.join();
  if (err) std::rethrow_exception(err);
}

// Sample of s indices of [lo, lo+n): the points of the uniform grid nearest
// to Chebyshev nodes (Mock-Chebyshev, appendix, linear-scaling ID), plus the
// four indices at each end of the range.  Along a geometrically ordered
// curve the ends of a partner range are where it can touch the candidate
// set, so the near-field rows/columns are always sampled.
void mock_cheb(int64_t lo, int64_t n, int s, std::vector<int32_t>& out) {
  out.clear();
  if (n <= s + 8) {
    for (int64_t i = 0; i < n; ++i) out.push_back(static_cast<int32_t>(lo + i));
    return;
  }
  std::vector<int64_t> idx;
  for (int64_t e = 0; e < 4; ++e) {
    idx.push_back(e);
    idx.push_back(n - 1 - e);
  }
  for (int a = 0; a < s; ++a) {
    const double t = 0.5 * (1.0 - std::cos(kPi * (a + 0.5) / s));
    idx.push_back(static_cast<int64_t>(std::llround(t * static_cast<double>(n - 1))));
  }
  std::sort(idx.begin(), idx.end());
  idx.erase(std::unique(idx.begin(), idx.end()), idx.end());
  for (int64_t i : idx) out.push_back(static_cast<int32_t>(lo + i));
}

// The real unknowns of the library range [lo, lo+n) in order (ghost
// entries of the matrix are zero, so samples are drawn from these only).
void real_indices(const Plan& P, int64_t lo, int64_t n, std::vector<int32_t>& out) {
  out.clear();
  for (int64_t i = lo; i < lo + n; ++i)
    if (!P.is_ghost(i)) out.push_back(static_cast<int32_t>(i));
}

struct IdRec {
  int k = 0;
  std::vector<int32_t> skel;   // global indices of the skeleton (k)
  std::vector<uint8_t> perm;   // pivot order over the candidates
  std::vector<cplx> T;         // k x (n_cand - k), row-major (i, t) at i*r + t
  int64_t seg = -1;            // arena offset of the skeleton vector
};

// Column ID of the s x n sample matrix M (column-major, M[c*s + a]) by
// Householder QR with column pivoting: M Lambda = Q [R1 R2], T = R1^{-1} R2,
// rank = first k with |R_{k+1,k+1}| <= eps |R_11| (appendix, linear-scaling
// ID; the pivot norms are recomputed exactly at every step).
void column_id(std::vector<cplx>& M, int s, int n, double eps, int kmax, IdRec& out) {
  std::vector<int> piv(n);
  for (int j = 0; j < n; ++j) piv[j] = j;
  std::vector<double> nrm(n);
  const int kcap = std::min({s, n, kmax});
  double ref = 0.0;
  int k = 0;
  std::vector<cplx> v(s);
  // column norms over the rows not yet reduced, downdated after each step and
  // recomputed when cancellation makes the downdate unreliable
  std::vector<double> nrm0(n);
  for (int j = 0; j < n; ++j) {
    const cplx* c = &M[static_cast<size_t>(j) * s];
    double acc = 0.0;
    for (int a = 0; a < s; ++a) acc += std::norm(c[a]);
    nrm[j] = nrm0[j] = acc;
  }
  for (int i = 0; i < kcap; ++i) {
    int p = i;
    double best = -1.0;
    for (int j = i; j < n; ++j) {
      if (nrm[j] < 1e-4 * nrm0[j]) {
        const cplx* c = &M[static_cast<size_t>(j) * s];
        double acc = 0.0;
        for (int a = i; a < s; ++a) acc += std::norm(c[a]);
        nrm[j] = nrm0[j] = acc;
      }
      if (nrm[j] > best) { best = nrm[j]; p = j; }
    }
    {  // exact norm of the chosen pivot
      const cplx* c = &M[static_cast<size_t>(p) * s];
      double acc = 0.0;
      for (int a = i; a < s; ++a) acc += std::norm(c[a]);
      best = acc;
    }
    const double pn = std::sqrt(best);
    if (i == 0) {
      ref = pn;
      if (ref == 0.0) break;
    } else if (pn <= eps * ref) {
      break;
    }
    if (p != i) {
      std::swap_ranges(&M[static_cast<size_t>(i) * s], &M[static_cast<size_t>(i) * s] + s,
                       &M[static_cast<size_t>(p) * s]);
      std::swap(piv[i], piv[p]);
      std::swap(nrm[i], nrm[p]);
      std::swap(nrm0[i], nrm0[p]);
    }
    // Householder vector for M[i:s, i]
    cplx* c = &M[static_cast<size_t>(i) * s];
    const double xn = pn;
    const double a0 = std::abs(c[i]);
    const cplx ph = (a0 > 0.0) ? c[i] / a0 : cplx(1.0, 0.0);
    const cplx alpha = -ph * xn;
    for (int a = i; a < s; ++a) v[a] = c[a];
    v[i] -= alpha;
    double vn2 = 0.0;
    for (int a = i; a < s; ++a) vn2 += std::norm(v[a]);
    c[i] = alpha;
    for (int a = i + 1; a < s; ++a) c[a] = 0.0;
    if (vn2 > 0.0) {
      const double inv = 2.0 / vn2;
      for (int j = i + 1; j < n; ++j) {
        cplx* cj = &M[static_cast<size_t>(j) * s];
        cplx dot = 0.0;
        for (int a = i; a < s; ++a) dot += std::conj(v[a]) * cj[a];
        dot *= inv;
        for (int a = i; a < s; ++a) cj[a] -= dot * v[a];
        nrm[j] = std::max(0.0, nrm[j] - std::norm(cj[i]));
      }
    }
    k = i + 1;
  }
  out.k = k;
  out.perm.resize(n);
  for (int j = 0; j < n; ++j) out.perm[j] = static_cast<uint8_t>(piv[j]);
  const int r = n - k;
  out.T.assign(static_cast<size_t>(k) * r, cplx(0.0));
  // back substitution R1 t = R2(:, c)
  std::vector<cplx> t(k);
  for (int cidx = 0; cidx < r; ++cidx) {
    const cplx* rc = &M[static_cast<size_t>(k + cidx) * s];
    for (int i = k - 1; i >= 0; --i) {
      cplx acc = rc[i];
      for (int j = i + 1; j < k; ++j) acc -= M[static_cast<size_t>(j) * s + i] * t[j];
      t[i] = acc / M[static_cast<size_t>(i) * s + i];
    }
    for (int i = 0; i < k; ++i) out.T[static_cast<size_t>(i) * r + cidx] = t[i];
  }
}

// ID of the candidate set `cand` against the partner range [plo, plo+pn):
// column ID of K(partner, cand) if partner_is_rows, else a row ID of
// K(cand, partner) computed as a column ID of its transpose.  The sample of
// partner indices starts as a Mock-Chebyshev subset; the ID is then checked
// on a pseudo-random probe of other partner indices and the sample grows
// until the probe residual is at the tolerance (or the sample is the whole
// partner set).
// The first sample and the first probe of compute_id for the same arguments
// (their index sets, in the same order), with room for their matrices, so a
// batch of IDs can have those matrices evaluated together beforehand.
struct IdPrefetch {
  std::vector<int32_t> samp, probe;
  std::vector<cplx> Ms, Mp;
  bool ready = false;
  // the column ID of the first sample, computed by the evaluator (id_ready)
  bool id_ready = false;
  int32_t k = 0;
  std::vector<uint8_t> perm;
  std::vector<cplx> T;
};

uint64_t id_seed(int64_t plo, const std::vector<int32_t>& cand) {
  return 0x9E3779B97F4A7C15ull ^ (static_cast<uint64_t>(plo) * 0xBF58476D1CE4E5B9ull) ^
         (static_cast<uint64_t>(cand[0]) << 20) ^ static_cast<uint64_t>(cand.size());
}

uint64_t id_rnd(uint64_t& seed) {
  seed ^= seed >> 30; seed *= 0xBF58476D1CE4E5B9ull;
  seed ^= seed >> 27; seed *= 0x94D049BB133111EBull;
  seed ^= seed >> 31;
  return seed;
}

constexpr int kProbe = 16;  // partner indices of a probe

void id_first_sets(const Plan& P, const std::vector<int32_t>& cand, int64_t plo, int64_t pn, IdPrefetch& pf) {
  const int n = static_cast<int>(cand.size());
  pf.samp.clear();
  pf.probe.clear();
  pf.ready = false;
  std::vector<int32_t> pos;
  const bool padded = !P.ghost.empty();
  if (padded) real_indices(P, plo, pn, pos);
  const int64_t pr = padded ? static_cast<int64_t>(pos.size()) : pn;
  if (pr == 0) return;
  auto to_partner = [&](std::vector<int32_t>& v) {
    if (padded)
      for (auto& x : v) x = pos[x];
    else
      for (auto& x : v) x += static_cast<int32_t>(plo);
  };
  const int s = static_cast<int>(std::min<int64_t>(pr, std::max(48, n / 2 + 16)));
  mock_cheb(0, pr, s, pf.samp);
  to_partner(pf.samp);
  uint64_t seed = id_seed(plo, cand);
  pf.probe.resize(kProbe);
  for (int a = 0; a < kProbe; ++a) pf.probe[a] = static_cast<int32_t>(id_rnd(seed) % pr);
  to_partner(pf.probe);
  pf.Mp.resize(pf.probe.size() * n);
}

void compute_id(const Plan& P, const std::vector<int32_t>& cand, int64_t plo, int64_t pn,
                bool partner_is_rows, double eps, IdRec& out, IdPrefetch* pf = nullptr) {
  const int n = static_cast<int>(cand.size());
  int s = static_cast<int>(std::min<int64_t>(pn, std::max(48, n / 2 + 16)));
  std::vector<int32_t> samp, probe;
  std::vector<cplx> M, Mp;
  auto fill = [&](const std::vector<int32_t>& pts, std::vector<cplx>& A) {
    const int ss = static_cast<int>(pts.size());
    A.resize(static_cast<size_t>(ss) * n);
    for (int c = 0; c < n; ++c)
      for (int a = 0; a < ss; ++a)
        A[static_cast<size_t>(c) * ss + a] = partner_is_rows ? P.entry(pts[a], cand[c]) : P.entry(cand[c], pts[a]);
  };
  uint64_t seed = id_seed(plo, cand);
  auto rnd = [&]() { return id_rnd(seed); };
  // prefetched matrices (same index sets as computed here) replace the host evaluation
  auto fill_or_take = [&](const std::vector<int32_t>& pts, std::vector<cplx>& A, const std::vector<int32_t>& pre,
                          std::vector<cplx>& preM) {
    if (pf && pf->ready && pts == pre && preM.size() == pts.size() * static_cast<size_t>(n)) A.swap(preM);
    else fill(pts, A);
  };
  // the partner set: its real unknowns, addressed by position pos[0..pr)
  std::vector<int32_t> pos;
  const bool padded = !P.ghost.empty();
  if (padded) real_indices(P, plo, pn, pos);
  const int64_t pr = padded ? static_cast<int64_t>(pos.size()) : pn;
  if (pr == 0) {  // nothing to interpolate against: every candidate is redundant with T = 0
    out.k = 0;
    out.perm.resize(n);
    for (int c = 0; c < n; ++c) out.perm[c] = c;
    out.T.assign(0, cplx(0.0));
    out.skel.clear();
    return;
  }
  auto to_partner = [&](std::vector<int32_t>& v) {
    if (padded)
      for (auto& x : v) x = pos[x];
    else
      for (auto& x : v) x += static_cast<int32_t>(plo);
  };
  s = static_cast<int>(std::min<int64_t>(pr, s));
  for (int attempt = 0; attempt < 8; ++attempt) {
    mock_cheb(0, pr, s, samp);
    to_partner(samp);
    const int ss = static_cast<int>(samp.size());
    if (pf && pf->id_ready && samp == pf->samp) {
      // the first sample's ID, computed with its matrix by the evaluator
      out.k = pf->k;
      out.perm.swap(pf->perm);
      out.T.assign(pf->T.begin(), pf->T.begin() + static_cast<size_t>(pf->k) * (n - pf->k));
      pf->id_ready = false;
    } else {
      if (pf) fill_or_take(samp, M, pf->samp, pf->Ms);
      else fill(samp, M);
      column_id(M, ss, n, eps, std::min(n, 127), out);
    }
    if (ss >= pr) break;
    const int need = 2 * out.k + 16;
    if (ss < need) {
      s = static_cast<int>(std::min<int64_t>(pr, need + 16));
      continue;
    }
    // probe: residual of K(probe, p) - K(probe, q) T relative to K(probe, cand)
    const int np = kProbe;
    probe.resize(np);
    for (int a = 0; a < np; ++a) probe[a] = static_cast<int32_t>(rnd() % pr);
    to_partner(probe);
    const int npr = np;
    if (pf) fill_or_take(probe, Mp, pf->probe, pf->Mp);
    else fill(probe, Mp);
    const int k = out.k, r = n - k;
    double rn = 0.0, an = 0.0;
    for (int c = 0; c < n; ++c)
      for (int a = 0; a < npr; ++a) an += std::norm(Mp[static_cast<size_t>(c) * npr + a]);
    for (int t = 0; t < r; ++t) {
      const int pc = out.perm[k + t];
      for (int a = 0; a < npr; ++a) {
        cplx acc = Mp[static_cast<size_t>(pc) * npr + a];
        for (int i = 0; i < k; ++i) acc -= Mp[static_cast<size_t>(out.perm[i]) * npr + a] * out.T[static_cast<size_t>(i) * r + t];
        rn += std::norm(acc);
      }
    }
    if (rn <= 4.0 * eps * eps * an) break;
    s = static_cast<int>(std::min<int64_t>(pr, 2 * ss));
  }
  out.skel.resize(out.k);
  for (int i = 0; i < out.k; ++i) out.skel[i] = cand[out.perm[i]];
}

inline int ilog2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << (l + 1)) <= x) ++l;
  return l;
}

int32_t push_unit(Plan& P, Unit u, const std::vector<cplx>& mats, const std::vector<uint8_t>& perms) {
  u.mat = static_cast<int64_t>(P.fac.size());
  int64_t len = static_cast<int64_t>(mats.size());
  u.mat_len = static_cast<int32_t>((len + 1) & ~int64_t(1));
  P.fac.insert(P.fac.end(), mats.begin(), mats.end());
  if (len & 1) P.fac.push_back(cplx(0.0));
  u.perm = static_cast<int64_t>(P.perm.size());
  P.perm.insert(P.perm.end(), perms.begin(), perms.end());
  P.units.push_back(u);
  return static_cast<int32_t>(P.units.size() - 1);
}

Unit blank_unit(uint8_t type) {
  Unit u;
  std::memset(&u, 0, sizeof(u));
  u.type = type;
  return u;
}

// ---------------------------------------------------------------------------
// IDBF of every off-diagonal block of one H-level (all blocks share L).
// ---------------------------------------------------------------------------
// IDs whose first sample and probe matrices are evaluated in one batch.
constexpr int64_t kIdBatch = 8192;

void build_level_blocks(Plan& P, int v, double eps, int nthreads, EntryEval* eval) {
  const int64_t N = P.n;
  const int64_t nv = N >> v;           // block size
  const int L = P.V - v;
  const int D = (L + 1) / 2;
  const int64_t npairs = int64_t(1) << (v - 1);
  const int64_t nb = 2 * npairs;        // blocks at this level
  const int n0 = P.n0;
  const int64_t m = int64_t(1) << L;    // leaves per block side

  const size_t b0 = P.blocks.size();
  for (int64_t p = 0; p < npairs; ++p) {
    for (int lower = 0; lower < 2; ++lower) {
      BlockInfo bi;
      bi.n = nv;
      bi.L = L;
      bi.D = D;
      bi.hlevel = v;
      bi.pair = p;
      bi.lower = lower;
      const int64_t base = p * 2 * nv;
      bi.row0 = lower ? base + nv : base;
      bi.col0 = lower ? base : base + nv;
      bi.lvl_begin.assign(2 * D + 1, 0);
      bi.lvl_end.assign(2 * D + 1, 0);
      P.blocks.push_back(bi);
    }
  }
  const int64_t nid = int64_t(2) * m;   // IDs per block per level per side
  // R[d] / C[d] for the current and previous level
  std::vector<IdRec> Rprev, Cprev, Rcur, Ccur;
  // arena segment offsets are assigned in a fixed order after each level

  auto leaf_range = [&](int64_t node, int level) { return std::make_pair(node * (nv >> level), nv >> level); };

  for (int d = 1; d <= D; ++d) {
    Rcur.assign(static_cast<size_t>(nb * nid), IdRec());
    Ccur.assign(static_cast<size_t>(nb * nid), IdRec());
    // one job per ID: its candidates (the IDs of the previous level's child
    // nodes, or the leaf rows/columns) and its partner range
    struct Job {
      std::vector<int32_t> cand;
      int64_t plo = 0, pn = 0;
      bool partner_rows = false;
      IdPrefetch pf;
    };
    const int64_t njobs = 2 * nb * nid;
    std::vector<Job> jobs(static_cast<size_t>(njobs));
    parallel_for(njobs, nthreads, [&](int64_t job) {
      const bool row_side = job < nb * nid;
      const int64_t jj = row_side ? job : job - nb * nid;
      const int64_t b = jj / nid;
      const int64_t id = jj % nid;
      const BlockInfo& bi = P.blocks[b0 + b];
      const int64_t a = id >> d;                 // node at level L-d+1 on the ID's own side
      const int64_t o = id & ((int64_t(1) << d) - 1);  // partner node at level d
      Job& J = jobs[job];
      const std::vector<IdRec>& prev = row_side ? Rprev : Cprev;
      const int64_t own0 = row_side ? bi.row0 : bi.col0;
      if (d == 1) {
        for (int i = 0; i < n0; ++i) J.cand.push_back(static_cast<int32_t>(own0 + a * n0 + i));
      } else {
        const int64_t op = o >> 1;
        for (int c = 0; c < 2; ++c) {
          const IdRec& ch = prev[b * nid + (((2 * a + c) << (d - 1)) + op)];
          J.cand.insert(J.cand.end(), ch.skel.begin(), ch.skel.end());
        }
      }
      auto pr = leaf_range(o, d);
      J.plo = (row_side ? bi.col0 : bi.row0) + pr.first;
      J.pn = pr.second;
      J.partner_rows = !row_side;  // row IDs sample the partner columns, column IDs the partner rows
    });
    auto run_ids = [&](int64_t j0, int64_t j1, bool pre) {
      parallel_for(j1 - j0, nthreads, [&](int64_t q) {
        const int64_t job = j0 + q;
        const bool row_side = job < nb * nid;
        const int64_t jj = row_side ? job : job - nb * nid;
        Job& J = jobs[job];
        IdRec& out = row_side ? Rcur[jj] : Ccur[jj];
        compute_id(P, J.cand, J.plo, J.pn, J.partner_rows, eps, out, pre ? &J.pf : nullptr);
        J.pf = IdPrefetch();
      });
    };
    if (!eval) {
      run_ids(0, njobs, false);
    } else {
      for (int64_t j0 = 0; j0 < njobs; j0 += kIdBatch) {
        const int64_t j1 = std::min(njobs, j0 + kIdBatch);
        parallel_for(j1 - j0, nthreads, [&](int64_t q) {
          Job& J = jobs[j0 + q];
          id_first_sets(P, J.cand, J.plo, J.pn, J.pf);
        });
        std::vector<EntryJob> ej;
        std::vector<IdJob> ids;
        ej.reserve(static_cast<size_t>(2 * (j1 - j0)));
        ids.reserve(static_cast<size_t>(j1 - j0));
        for (int64_t job = j0; job < j1; ++job) {
          Job& J = jobs[job];
          const int32_t nc = static_cast<int32_t>(J.cand.size());
          if (J.pf.samp.empty()) continue;
          const int32_t sw = J.partner_rows ? 0 : 1;
          // the first sample's matrix feeds the evaluator's ID only
          ids.push_back({static_cast<int32_t>(ej.size()), std::min(nc, 127), eps, &J.pf.k, nullptr, nullptr});
          ej.push_back({J.pf.samp.data(), static_cast<int32_t>(J.pf.samp.size()), J.cand.data(), nc, sw, nullptr});
          ej.push_back({J.pf.probe.data(), static_cast<int32_t>(J.pf.probe.size()), J.cand.data(), nc, sw,
                        J.pf.Mp.data()});
          J.pf.perm.resize(static_cast<size_t>(nc));
          J.pf.T.resize(static_cast<size_t>(nc) * nc / 4 + 1);
          ids.back().perm = J.pf.perm.data();
          ids.back().T = J.pf.T.data();
          J.pf.ready = true;
          J.pf.id_ready = true;
        }
        eval->eval(ej, ids);
        run_ids(j0, j1, true);
      }
    }
    // arena segments and statistics
    for (auto* vec : {&Ccur, &Rcur}) {
      for (auto& r : *vec) {
        r.seg = P.arena_rows;
        P.arena_rows += r.k;
        P.max_rank = std::max(P.max_rank, r.k);
        P.sum_rank += r.k;
        P.n_ids += 1;
      }
    }
    // ---- units of level d: V side (GATHER) and U side (SCATTER) ----
    for (int64_t b = 0; b < nb; ++b) {
      BlockInfo& bi = P.blocks[b0 + b];
      const int fl = d - 1;  // forward level of the V units
      bi.lvl_begin[fl] = static_cast<int32_t>(P.units.size());
      const int64_t nsig = int64_t(1) << (L - d + 1);
      const int64_t ntp = int64_t(1) << (d - 1);
      for (int64_t sg = 0; sg < nsig; ++sg) {
        for (int64_t tp = 0; tp < ntp; ++tp) {
          Unit u = blank_unit(UNIT_GATHER);
          const IdRec& ia = Ccur[b * nid + ((sg << d) + 2 * tp)];
          const IdRec& ib = Ccur[b * nid + ((sg << d) + 2 * tp + 1)];
          int nsrc;
          if (d == 1) {
            u.in_buf = BUF_X;
            u.in_off[0] = static_cast<int32_t>(bi.col0 + sg * n0);
            u.in_len[0] = static_cast<int16_t>(n0);
            nsrc = n0;
          } else {
            const IdRec& c0 = Cprev[b * nid + (((2 * sg) << (d - 1)) + tp)];
            const IdRec& c1 = Cprev[b * nid + (((2 * sg + 1) << (d - 1)) + tp)];
            u.in_buf = BUF_ARENA;
            u.in_off[0] = static_cast<int32_t>(c0.seg);
            u.in_len[0] = static_cast<int16_t>(c0.k);
            u.in_off[1] = static_cast<int32_t>(c1.seg);
            u.in_len[1] = static_cast<int16_t>(c1.k);
            nsrc = c0.k + c1.k;
          }
          u.out_buf = BUF_ARENA;
          u.out_off[0] = static_cast<int32_t>(ia.seg);
          u.out_len[0] = static_cast<int16_t>(ia.k);
          u.out_off[1] = static_cast<int32_t>(ib.seg);
          u.out_len[1] = static_cast<int16_t>(ib.k);
          u.k[0] = static_cast<int16_t>(ia.k);
          u.k[1] = static_cast<int16_t>(ib.k);
          std::vector<cplx> mats;
          std::vector<uint8_t> perms;
          for (const IdRec* r : {&ia, &ib}) {
            const int rr = nsrc - r->k;
            // column-major k x rr
            for (int t = 0; t < rr; ++t)
              for (int i = 0; i < r->k; ++i) mats.push_back(r->T[static_cast<size_t>(i) * rr + t]);
            perms.insert(perms.end(), r->perm.begin(), r->perm.end());
          }
          push_unit(P, u, mats, perms);
        }
      }
      bi.lvl_end[fl] = static_cast<int32_t>(P.units.size());
    }
    for (int64_t b = 0; b < nb; ++b) {
      BlockInfo& bi = P.blocks[b0 + b];
      const int fl = 2 * D - (d - 1);  // forward level of the U units
      bi.lvl_begin[fl] = static_cast<int32_t>(P.units.size());
      const int64_t ntau = int64_t(1) << (L - d + 1);
      const int64_t nsp = int64_t(1) << (d - 1);
      for (int64_t ta = 0; ta < ntau; ++ta) {
        for (int64_t sp = 0; sp < nsp; ++sp) {
          Unit u = blank_unit(UNIT_SCATTER);
          const IdRec& ia = Rcur[b * nid + ((ta << d) + 2 * sp)];
          const IdRec& ib = Rcur[b * nid + ((ta << d) + 2 * sp + 1)];
          u.in_buf = BUF_ARENA;
          u.in_off[0] = static_cast<int32_t>(ia.seg);
          u.in_len[0] = static_cast<int16_t>(ia.k);
          u.in_off[1] = static_cast<int32_t>(ib.seg);
          u.in_len[1] = static_cast<int16_t>(ib.k);
          u.k[0] = static_cast<int16_t>(ia.k);
          u.k[1] = static_cast<int16_t>(ib.k);
          int ndst;
          if (d == 1) {
            u.out_buf = BUF_Y;
            u.out_off[0] = static_cast<int32_t>(bi.row0 + ta * n0);
            u.out_len[0] = static_cast<int16_t>(n0);
            ndst = n0;
          } else {
            const IdRec& r0 = Rprev[b * nid + (((2 * ta) << (d - 1)) + sp)];
            const IdRec& r1 = Rprev[b * nid + (((2 * ta + 1) << (d - 1)) + sp)];
            u.out_buf = BUF_ARENA;
            u.out_off[0] = static_cast<int32_t>(r0.seg);
            u.out_len[0] = static_cast<int16_t>(r0.k);
            u.out_off[1] = static_cast<int32_t>(r1.seg);
            u.out_len[1] = static_cast<int16_t>(r1.k);
            ndst = r0.k + r1.k;
          }
          std::vector<cplx> mats;
          std::vector<uint8_t> perms;
          for (const IdRec* r : {&ia, &ib}) {
            const int rr = ndst - r->k;
            // row-major k x rr
            mats.insert(mats.end(), r->T.begin(), r->T.end());
            std::vector<uint8_t> inv(ndst);
            for (int j = 0; j < ndst; ++j) inv[r->perm[j]] = static_cast<uint8_t>(j);
            perms.insert(perms.end(), inv.begin(), inv.end());
            (void)rr;
          }
          push_unit(P, u, mats, perms);
        }
      }
      bi.lvl_end[fl] = static_cast<int32_t>(P.units.size());
    }
    // free the transfer matrices of the finished level, keep skeletons
    for (auto* vec : {&Ccur, &Rcur})
      for (auto& r : *vec) { std::vector<cplx>().swap(r.T); }
    Rprev.swap(Rcur);
    Cprev.swap(Ccur);
  }
  // ---- middle coupling units (dense kernel blocks on the last skeletons) ----
  const bool odd = (L & 1) != 0;
  std::vector<std::vector<cplx>> mid_mats(static_cast<size_t>(nb * (odd ? 2 * m : m)));
  const int64_t nD = int64_t(1) << D;
  auto mid_sets = [&](int64_t b, int64_t ta, int64_t sg, std::vector<const IdRec*>& rs,
                      std::vector<const IdRec*>& cs) {
    rs.clear();
    cs.clear();
    if (odd) {
      rs.push_back(&Rprev[b * nid + ((ta << D) + sg)]);
      cs.push_back(&Cprev[b * nid + ((sg << D) + ta)]);
    } else {
      rs.push_back(&Rprev[b * nid + (((2 * ta) << D) + sg)]);
      rs.push_back(&Rprev[b * nid + (((2 * ta + 1) << D) + sg)]);
      cs.push_back(&Cprev[b * nid + (((2 * sg) << D) + ta)]);
      cs.push_back(&Cprev[b * nid + (((2 * sg + 1) << D) + ta)]);
    }
  };
  const int64_t nmid = nb * nD * nD;
  std::vector<std::vector<int32_t>> mid_rows(static_cast<size_t>(nmid)), mid_cols(static_cast<size_t>(nmid));
  parallel_for(nmid, nthreads, [&](int64_t job) {
    const int64_t b = job / (nD * nD);
    const int64_t ta = (job / nD) % nD;
    const int64_t sg = job % nD;
    std::vector<const IdRec*> rs, cs;
    mid_sets(b, ta, sg, rs, cs);
    std::vector<int32_t>& rows = mid_rows[job];
    std::vector<int32_t>& cols = mid_cols[job];
    for (auto* r : rs) rows.insert(rows.end(), r->skel.begin(), r->skel.end());
    for (auto* c : cs) cols.insert(cols.end(), c->skel.begin(), c->skel.end());
    std::vector<cplx>& M = mid_mats[job];
    M.resize(rows.size() * cols.size());
    // column-major n_dst x n_src
    if (!eval)
      for (size_t t = 0; t < cols.size(); ++t)
        for (size_t i = 0; i < rows.size(); ++i) M[t * rows.size() + i] = P.entry(rows[i], cols[t]);
  });
  if (eval) {
    for (int64_t j0 = 0; j0 < nmid; j0 += 8 * kIdBatch) {
      std::vector<EntryJob> ej;
      for (int64_t job = j0; job < std::min(nmid, j0 + 8 * kIdBatch); ++job)
        if (!mid_mats[job].empty())
          ej.push_back({mid_rows[job].data(), static_cast<int32_t>(mid_rows[job].size()), mid_cols[job].data(),
                        static_cast<int32_t>(mid_cols[job].size()), 0, mid_mats[job].data()});
      eval->eval(ej);
    }
  }
  for (int64_t b = 0; b < nb; ++b) {
    BlockInfo& bi = P.blocks[b0 + b];
    bi.lvl_begin[D] = static_cast<int32_t>(P.units.size());
    for (int64_t ta = 0; ta < nD; ++ta) {
      for (int64_t sg = 0; sg < nD; ++sg) {
        std::vector<const IdRec*> rs, cs;
        mid_sets(b, ta, sg, rs, cs);
        Unit u = blank_unit(UNIT_DENSE);
        u.in_buf = BUF_ARENA;
        u.out_buf = BUF_ARENA;
        for (size_t i = 0; i < cs.size(); ++i) {
          u.in_off[i] = static_cast<int32_t>(cs[i]->seg);
          u.in_len[i] = static_cast<int16_t>(cs[i]->k);
        }
        for (size_t i = 0; i < rs.size(); ++i) {
          u.out_off[i] = static_cast<int32_t>(rs[i]->seg);
          u.out_len[i] = static_cast<int16_t>(rs[i]->k);
        }
        std::vector<cplx>& M = mid_mats[(b * nD + ta) * nD + sg];
        push_unit(P, u, M, {});
        std::vector<cplx>().swap(M);
      }
    }
    bi.lvl_end[D] = static_cast<int32_t>(P.units.size());
  }
}

// A dense n0 x n0 block A[r0 + i, c0 + t], M column-major (M[t n0 + i]).
int32_t dense_block_unit(Plan& P, int64_t r0, int64_t c0, int n0, uint8_t in_buf, uint8_t out_buf,
                         const std::vector<cplx>& M) {
  Unit u = blank_unit(UNIT_DENSE);
  u.in_buf = in_buf;
  u.out_buf = out_buf;
  u.in_off[0] = static_cast<int32_t>(c0);
  u.in_len[0] = static_cast<int16_t>(n0);
  u.out_off[0] = static_cast<int32_t>(r0);
  u.out_len[0] = static_cast<int16_t>(n0);
  return push_unit(P, u, M, {});
}

int32_t dense_unit(Plan& P, int64_t r0, int64_t c0, int n0, uint8_t in_buf, uint8_t out_buf) {
  std::vector<cplx> M(static_cast<size_t>(n0) * n0);
  for (int t = 0; t < n0; ++t)
    for (int i = 0; i < n0; ++i) M[static_cast<size_t>(t) * n0 + i] = P.entry(r0 + i, c0 + t);
  return dense_block_unit(P, r0, c0, n0, in_buf, out_buf, M);
}

Launch make_launch(const Plan& P, int direct, int first, int count, int acc, int kind) {
  Launch l;
  l.direct = direct;
  l.first = first;
  l.count = count;
  l.max_src = l.max_dst = l.max_mat = 0;
  l.out_leaf = acc;
  l.kind = kind;
  auto visit = [&](int32_t uid) {
    const Unit& u = P.units[uid];
    const int a = u.in_len[0] + u.in_len[1];
    const int b = u.out_len[0] + u.out_len[1];
    l.max_src = std::max({l.max_src, a, b});
    l.max_dst = std::max({l.max_dst, a, b});
    l.max_in = std::max(l.max_in, a);
    l.max_out = std::max(l.max_out, b);
    l.max_mat = std::max<int32_t>(l.max_mat, u.mat_len);
  };
  l.single = 1;
  for (int g = first; g < first + count; ++g) {
    if (direct) {
      visit(g);
    } else {
      if (P.group_off[g + 1] - P.group_off[g] != 1) l.single = 0;
      for (int32_t q = P.group_off[g]; q < P.group_off[g + 1]; ++q) visit(P.group_units[q]);
    }
  }
  return l;
}

}  // namespace

void column_id_into(std::vector<cplx>& M, int s, int n, double eps, int kmax, int32_t* k, uint8_t* perm, cplx* T) {
  IdRec r;
  column_id(M, s, n, eps, kmax, r);
  *k = r.k;
  std::copy(r.perm.begin(), r.perm.end(), perm);
  std::copy(r.T.begin(), r.T.end(), T);
}

int32_t add_group(Plan& p, const std::vector<int32_t>& unit_ids) {
  if (p.group_off.empty()) p.group_off.push_back(0);
  p.group_units.insert(p.group_units.end(), unit_ids.begin(), unit_ids.end());
  p.group_off.push_back(static_cast<int32_t>(p.group_units.size()));
  return static_cast<int32_t>(p.group_off.size() - 2);
}

int build_threads(const hbf_build_opts* opts) {
  if (opts && opts->nthreads > 0) return opts->nthreads;
  const unsigned hc = std::thread::hardware_concurrency();
  return hc ? static_cast<int>(hc) : 8;
}

cplx Plan::self_entry(int64_t i) const {
  if (is_ghost(i)) return cplx(1.0, 0.0);
  // Sec. 3.1 closed form: (kappa eta0 w_i / 4) [1 - i (2/pi) ln(gamma kappa w_i / (4 e))]
  const double g = std::exp(kEulerGamma);
  const double c = kappa * eta0 * w[i] / 4.0;
  cplx d(c, -c * (2.0 / kPi) * std::log(g * kappa * w[i] / (4.0 * std::exp(1.0))));
  if (!z.empty()) d += z[i];
  return d;
}

cplx Plan::entry(int64_t i, int64_t j) const {
  if (i == j) return self_entry(i);
  if (is_ghost(i) || is_ghost(j)) return cplx(0.0, 0.0);
  const double r = std::hypot(cx[i] - cx[j], cy[i] - cy[j]);
  return (kappa * eta0 * w[j] / 4.0) * hankel2_0(kappa * r);
}

void build_plan(Plan& P, const hbf_curve* curve, double kappa, int leaf, double tol,
                const hbf_build_opts* opts, EntryEval* eval) {
  auto t0 = std::chrono::steady_clock::now();
  if (!curve || curve->ncurves < 1 || !curve->node_off || !curve->xy)
    throw std::invalid_argument("hbf_build: empty curve");
  if (!(kappa > 0.0) || !std::isfinite(kappa)) throw std::invalid_argument("hbf_build: kappa must be > 0");
  if (leaf < 2 || leaf > 128) throw std::invalid_argument("hbf_build: leaf must be in [2, 128]");
  if (!(tol > 0.0) || tol >= 1.0) throw std::invalid_argument("hbf_build: tol must be in (0, 1)");
  // geometry: segment i is the chord between consecutive nodes of a curve
  P.cx.clear();
  P.cy.clear();
  P.w.clear();
  for (int c = 0; c < curve->ncurves; ++c) {
    const int64_t a = curve->node_off[c], b = curve->node_off[c + 1];
    if (b - a < 2) throw std::invalid_argument("hbf_build: a curve needs at least 2 nodes");
    for (int64_t k = a; k + 1 < b; ++k) {
      const double x0 = curve->xy[2 * k], y0 = curve->xy[2 * k + 1];
      const double x1 = curve->xy[2 * k + 2], y1 = curve->xy[2 * k + 3];
      if (!std::isfinite(x0 + y0 + x1 + y1)) throw std::invalid_argument("hbf_build: non-finite node");
      P.cx.push_back(0.5 * (x0 + x1));
      P.cy.push_back(0.5 * (y0 + y1));
      const double wl = std::hypot(x1 - x0, y1 - y0);
      if (!(wl > 0.0)) throw std::invalid_argument("hbf_build: zero-length segment");
      P.w.push_back(wl);
    }
  }
  P.n_real = static_cast<int64_t>(P.w.size());
  P.n0 = leaf;
  if (P.n_real <= leaf) throw std::invalid_argument("hbf_build: N must exceed the leaf size");
  if (P.n_real >= (int64_t(1) << 29)) throw std::invalid_argument("hbf_build: N too large");
  {
    // leaf partition: bisect [0, N) while a piece has more than n0 unknowns,
    // first half ceil(m/2); a leaf at depth d and index j of that tree owns
    // library leaf j 2^(V - d), V the deepest level
    struct Leaf { int64_t lo, hi; int depth; int64_t index; };
    std::vector<Leaf> leaves;
    std::function<void(int64_t, int64_t, int, int64_t)> rec = [&](int64_t lo, int64_t hi, int d, int64_t j) {
      if (hi - lo <= leaf) {
        leaves.push_back({lo, hi, d, j});
        return;
      }
      const int64_t mid = lo + (hi - lo + 1) / 2;
      rec(lo, mid, d + 1, 2 * j);
      rec(mid, hi, d + 1, 2 * j + 1);
    };
    rec(0, P.n_real, 0, 0);
    int V = 0;
    for (const Leaf& l : leaves) V = std::max(V, l.depth);
    P.V = V;
    P.n = static_cast<int64_t>(leaf) << V;
    P.lib_of.clear();
    P.ghost.clear();
    if (P.n != P.n_real) {
      P.lib_of.assign(P.n_real, -1);
      P.ghost.assign(P.n, 1);
      std::vector<double> cx(P.n, 0.0), cy(P.n, 0.0), w(P.n, 1.0);
      for (const Leaf& l : leaves) {
        const int64_t base = (l.index << (V - l.depth)) * leaf;
        for (int64_t i = l.lo; i < l.hi; ++i) {
          const int64_t q = base + (i - l.lo);
          P.lib_of[i] = static_cast<int32_t>(q);
          P.ghost[q] = 0;
          cx[q] = P.cx[i];
          cy[q] = P.cy[i];
          w[q] = P.w[i];
        }
      }
      P.cx.swap(cx);
      P.cy.swap(cy);
      P.w.swap(w);
    }
  }
  const int64_t nl = P.n / leaf;
  P.kappa = kappa;
  P.eta0 = (opts && opts->eta0 > 0.0) ? opts->eta0 : 376.730313668;
  P.tol = tol;
  P.z.clear();
  if (opts && opts->z) {
    P.z.assign(P.n, cplx(0.0, 0.0));
    for (int64_t i = 0; i < P.n_real; ++i) P.z[P.lib(i)] = cplx(opts->z[2 * i], opts->z[2 * i + 1]);
  }
  const int nthreads = build_threads(opts);
  // the ID tolerance: a fraction of tol, so the accumulated error over the
  // factor chain and the sum over blocks stays at the level of tol
  const double eps = 0.5 * tol;

  P.units.clear();
  P.fac.clear();
  P.perm.clear();
  P.blocks.clear();
  P.group_off.clear();
  P.group_units.clear();
  P.arena_rows = 0;
  P.max_rank = 0;
  P.sum_rank = 0;
  P.n_ids = 0;

  if (eval) eval->prepare(P);
  // diagonal leaves and the dense L = 0 blocks of the last level, in this order
  const int64_t npl = nl / 2;
  std::vector<std::pair<int64_t, int64_t>> dense_rc;  // (first row, first column)
  for (int64_t b = 0; b < nl; ++b) dense_rc.push_back({b * leaf, b * leaf});
  for (int64_t p = 0; p < npl; ++p) {
    dense_rc.push_back({(2 * p + 1) * leaf, 2 * p * leaf});
    dense_rc.push_back({2 * p * leaf, (2 * p + 1) * leaf});
  }
  std::vector<int32_t> dense_ids(dense_rc.size(), -1);
  if (!eval) {
    for (size_t q = 0; q < dense_rc.size(); ++q)
      dense_ids[q] = dense_unit(P, dense_rc[q].first, dense_rc[q].second, leaf, BUF_X, BUF_Y);
  } else {
    constexpr size_t kDenseBatch = 4096;
    const size_t bs = static_cast<size_t>(leaf) * leaf;
    std::vector<int32_t> idx;
    std::vector<cplx> M;
    for (size_t q0 = 0; q0 < dense_rc.size(); q0 += kDenseBatch) {
      const size_t q1 = std::min(dense_rc.size(), q0 + kDenseBatch);
      idx.assign(2 * leaf * (q1 - q0), 0);
      M.assign(bs * (q1 - q0), cplx(0.0));
      std::vector<EntryJob> ej;
      for (size_t q = q0; q < q1; ++q) {
        int32_t* rows = &idx[2 * leaf * (q - q0)];
        int32_t* cols = rows + leaf;
        for (int i = 0; i < leaf; ++i) {
          rows[i] = static_cast<int32_t>(dense_rc[q].first + i);
          cols[i] = static_cast<int32_t>(dense_rc[q].second + i);
        }
        ej.push_back({rows, leaf, cols, leaf, 0, &M[bs * (q - q0)]});
      }
      eval->eval(ej);
      for (size_t q = q0; q < q1; ++q) {
        std::vector<cplx> Mq(M.begin() + bs * (q - q0), M.begin() + bs * (q - q0 + 1));
        dense_ids[q] = dense_block_unit(P, dense_rc[q].first, dense_rc[q].second, leaf, BUF_X, BUF_Y, Mq);
      }
    }
  }
  P.diag_unit.assign(nl, -1);
  P.l0_lower_unit.assign(npl, -1);
  P.l0_upper_unit.assign(npl, -1);
  for (int64_t b = 0; b < nl; ++b) P.diag_unit[b] = dense_ids[b];
  for (int64_t p = 0; p < npl; ++p) {
    P.l0_lower_unit[p] = dense_ids[nl + 2 * p];
    P.l0_upper_unit[p] = dense_ids[nl + 2 * p + 1];
  }
  const int64_t dense_end = static_cast<int64_t>(P.fac.size());
  // butterfly blocks, H-level by H-level
  const bool verbose = opts && opts->verbose;
  for (int v = 1; v < P.V; ++v) {
    build_level_blocks(P, v, eps, nthreads, eval);
    if (verbose) {
      const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      std::fprintf(stderr, "[hbf] H-level %d of %d compressed: %zu units, %.2f GB of factors (%.1f s)\n", v, P.V - 1,
                   P.units.size(), static_cast<double>(P.fac.size()) * 16e-9, sec);
      std::fflush(stderr);
    }
  }
  P.bytes_dense_c128 = dense_end * 16;
  P.bytes_butterfly_c128 = (static_cast<int64_t>(P.fac.size()) - dense_end) * 16;

  // scale factor a = 1 / A[i*, i*], i* = argmax |A_ii| over the real
  // unknowns (lowest index on ties)
  {
    int64_t ib = 0;
    double best = -1.0;
    for (int64_t i = 0; i < P.n_real; ++i) {
      const double a = std::abs(P.self_entry(P.lib(i)));
      if (a > best) { best = a; ib = P.lib(i); }
    }
    P.scale = 1.0 / P.self_entry(ib);
  }

  // Super-leaf solve units.  The diagonal tree is cut at super-leaves of
  // 2^sl leaves; inside one, the block substitution of Algorithms 3 / 4 is
  // replaced by the inverse of that diagonal block of L~ (or U~), formed in
  // FP64 from the exact entries.  Each leaf row block of the inverse is split
  // into slabs of sl_slab rows, one unit each (reading the super-leaf's input
  // rows the row block depends on), so that the solve of one super-leaf is
  // spread over many independent units.  Four sets: forward (L inverse),
  // backward (U inverse), and the conjugate transposes of the U and L
  // inverses for the adjoint sweeps (those are applied in forward mode).
  // Matrices live in a region after the factors and are filled by the leaf
  // factorisation.
  const hbf_prec prec = opts ? opts->prec : HBF_PREC_BLOCK_LU;
  const int sl_req = (opts && opts->superleaf > 0) ? opts->superleaf : 2;
  if (sl_req < 2 || sl_req > 3) throw std::invalid_argument("hbf_build: superleaf must be 2 or 3");
  P.sl = std::min(sl_req, P.V);
  P.sl_slab = (leaf % 8 == 0) ? 8 : leaf;
  const int s_leaves = 1 << P.sl;
  const int slabs = leaf / P.sl_slab;
  P.sl_units = s_leaves * slabs;
  const int64_t ns = static_cast<int64_t>(leaf) << P.sl;
  const int64_t nsl = P.n / ns;
  for (auto* v : {&P.sl_fwd, &P.sl_bwd, &P.sl_adj_fwd, &P.sl_adj_bwd}) v->clear();
  P.leaf_fac_begin = static_cast<int64_t>(P.fac.size());
  P.leaf_fac_len = 0;
  if (prec != HBF_PREC_NONE) {
    int64_t off = P.leaf_fac_begin;
    // set 0: lower-shaped forward, 1: upper-shaped backward, 2: lower-shaped
    // adjoint-forward, 3: upper-shaped adjoint-backward
    for (int set = 0; set < 4; ++set) {
      std::vector<int32_t>& dst = set == 0 ? P.sl_fwd : set == 1 ? P.sl_bwd : set == 2 ? P.sl_adj_fwd : P.sl_adj_bwd;
      const bool lower_shape = (set == 0 || set == 2);
      for (int64_t S = 0; S < nsl; ++S) {
        dst.push_back(static_cast<int32_t>(P.units.size()));
        for (int i = 0; i < s_leaves; ++i) {
          const int c0 = lower_shape ? 0 : i;                 // first leaf column of the row block
          const int c1 = lower_shape ? i + 1 : s_leaves;      // end leaf column
          for (int j = 0; j < slabs; ++j) {
            Unit u = blank_unit(UNIT_DENSE);
            u.in_buf = (set < 2) ? BUF_Y : BUF_X;
            u.out_buf = (set < 2) ? BUF_X : BUF_Y;
            u.in_off[0] = static_cast<int32_t>(S * ns + static_cast<int64_t>(c0) * leaf);
            u.in_len[0] = static_cast<int16_t>((c1 - c0) * leaf);
            u.out_off[0] = static_cast<int32_t>(S * ns + static_cast<int64_t>(i) * leaf + j * P.sl_slab);
            u.out_len[0] = static_cast<int16_t>(P.sl_slab);
            u.mat_len = static_cast<int32_t>(static_cast<int64_t>(P.sl_slab) * leaf * (c1 - c0));
            u.mat = off;
            off += u.mat_len;
            u.perm = 0;
            P.units.push_back(u);
          }
        }
      }
    }
    P.leaf_fac_len = off - P.leaf_fac_begin;
  }
  (void)ns;

  // ---- matvec schedules ----
  int Dmax = 0;
  for (auto& bi : P.blocks) Dmax = std::max(Dmax, bi.D);
  const int F = 2 * Dmax;
  // forward stages 0..F-1 of single-unit groups, stage F = per-row-leaf sums
  std::vector<std::vector<int32_t>> fstage(F + 1), astage(F + 1);
  for (auto& bi : P.blocks) {
    const int D = bi.D;
    // forward stage of each block level: V levels 0..D-1 at 0..D-1, middle at F-D,
    // U levels D+1..2D-1 at F-D+1..F-1, U leaf at F (handled by row groups)
    for (int l = 0; l < 2 * D; ++l) {
      const int fs = (l < D) ? l : F - 2 * D + l;
      const int as = (l < D) ? F - l : 2 * D - l;  // adjoint stage (mirror)
      for (int32_t u = bi.lvl_begin[l]; u < bi.lvl_end[l]; ++u) {
        fstage[fs].push_back(u);
        if (l > 0) astage[as].push_back(u);
      }
    }
    for (int32_t u = bi.lvl_begin[2 * D]; u < bi.lvl_end[2 * D]; ++u) astage[0].push_back(u);
  }
  P.mv_fwd.clear();
  P.mv_adj.clear();
  for (int s = 0; s < F; ++s) {
    if (fstage[s].empty()) continue;
    const int g0 = static_cast<int>(P.group_off.empty() ? 0 : P.group_off.size() - 1);
    for (int32_t u : fstage[s]) add_group(P, {u});
    P.mv_fwd.push_back(make_launch(P, 0, g0, static_cast<int>(fstage[s].size()), 0, 0));
  }
  {
    // row-leaf groups: diag + L0 neighbour + U-leaf units of every block
    std::vector<std::vector<int32_t>> rows(nl);
    for (int64_t b = 0; b < nl; ++b) rows[b].push_back(P.diag_unit[b]);
    for (int64_t p = 0; p < npl; ++p) {
      rows[2 * p + 1].push_back(P.l0_lower_unit[p]);
      rows[2 * p].push_back(P.l0_upper_unit[p]);
    }
    for (auto& bi : P.blocks)
      for (int32_t u = bi.lvl_begin[2 * bi.D]; u < bi.lvl_end[2 * bi.D]; ++u)
        rows[P.units[u].out_off[0] / leaf].push_back(u);
    const int g0 = static_cast<int>(P.group_off.empty() ? 0 : P.group_off.size() - 1);
    for (int64_t b = 0; b < nl; ++b) add_group(P, rows[b]);
    P.mv_fwd.push_back(make_launch(P, 0, g0, static_cast<int>(nl), 0, 0));
  }
  for (int s = 0; s < F; ++s) {
    if (astage[s].empty()) continue;
    const int g0 = static_cast<int>(P.group_off.size() - 1);
    for (int32_t u : astage[s]) add_group(P, {u});
    P.mv_adj.push_back(make_launch(P, 0, g0, static_cast<int>(astage[s].size()), 0, 0));
  }
  {
    std::vector<std::vector<int32_t>> cols(nl);
    for (int64_t b = 0; b < nl; ++b) cols[b].push_back(P.diag_unit[b]);
    for (int64_t p = 0; p < npl; ++p) {
      cols[2 * p].push_back(P.l0_lower_unit[p]);
      cols[2 * p + 1].push_back(P.l0_upper_unit[p]);
    }
    for (auto& bi : P.blocks)
      for (int32_t u = bi.lvl_begin[0]; u < bi.lvl_end[0]; ++u) cols[P.units[u].in_off[0] / leaf].push_back(u);
    const int g0 = static_cast<int>(P.group_off.size() - 1);
    for (int64_t b = 0; b < nl; ++b) add_group(P, cols[b]);
    P.mv_adj.push_back(make_launch(P, 0, g0, static_cast<int>(nl), 0, 0));
  }
  P.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace hbf
