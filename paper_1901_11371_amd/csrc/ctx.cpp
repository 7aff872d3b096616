// Device context: construction upload, leaf factorisation, and the matvec /
// preconditioner entry points of the C ABI.
#include "ctx.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <atomic>
#include <thread>
#include <stdexcept>
#include <string>

using namespace hbf;

namespace {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError(std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
void dmalloc(T** p, size_t bytes, const char* what) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  const hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    throw std::bad_alloc();
  }
  (void)what;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

void free_graphs(hbf_ctx* c) {
  for (auto& kv : c->pc_graphs) (void)hipGraphExecDestroy(kv.second);
  c->pc_graphs.clear();
  for (auto& kv : c->step_graphs) (void)hipGraphExecDestroy(kv.second);
  c->step_graphs.clear();
}

void free_device(hbf_ctx* c) {
  free_graphs(c);
  dfree(c->d_pz);
  c->d_pz = nullptr;
  dfree(c->d_fac);
  dfree(c->d_perm);
  dfree(c->d_units);
  dfree(c->d_gofs);
  dfree(c->d_gunits);
  dfree(c->d_steps);
  dfree(c->d_punits);
  dfree(c->d_lunits);
  dfree(c->d_lwaves);
  dfree(c->d_lmap);
  dfree(c->d_lrole);
  c->d_lwaves = nullptr;
  c->d_lmap = nullptr;
  c->d_lrole = nullptr;
  dfree(c->d_arena);
  dfree(c->d_vin);
  dfree(c->d_vout);
  dfree(c->d_u);
  dfree(c->d_t);
  dfree(c->d_diag64);
  dfree(c->d_flag);
  dfree(c->d_krylov);
  dfree(c->d_w);
  dfree(c->d_x64);
  dfree(c->d_red);
  dfree(c->d_small);
  dfree(c->d_real_of);
  dfree(c->d_lib_of);
  c->d_real_of = c->d_lib_of = nullptr;
  c->vmap = hbf::VecMap{};
  if (c->h_flags) (void)hipHostFree(c->h_flags);
  c->h_flags = nullptr;
  for (auto& e : c->ev_step)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
  c->d_fac = c->d_arena = c->d_vin = c->d_vout = c->d_u = c->d_t = nullptr;
  c->d_krylov = c->d_w = c->d_x64 = nullptr;
}

// Upload host complex128 entries [begin, end) of P.fac as the storage dtype.
void upload_factors(hbf_ctx* c, int64_t begin, int64_t end, hipStream_t s) {
  const size_t chunk = size_t(1) << 22;  // entries per staging transfer
  void* stage = nullptr;
  hip_check(hipHostMalloc(&stage, chunk * c->elt, hipHostMallocDefault), "hipHostMalloc");
  try {
    for (int64_t e = begin; e < end; e += static_cast<int64_t>(chunk)) {
      const int64_t m = std::min<int64_t>(static_cast<int64_t>(chunk), end - e);
      if (c->dtype == HBF_C64) {
        float* f = static_cast<float*>(stage);
        for (int64_t i = 0; i < m; ++i) {
          f[2 * i] = static_cast<float>(c->P.fac[e + i].real());
          f[2 * i + 1] = static_cast<float>(c->P.fac[e + i].imag());
        }
      } else {
        std::memcpy(stage, &c->P.fac[e], m * 16);
      }
      hip_check(hipMemcpyAsync(static_cast<char*>(c->d_fac) + e * c->elt, stage, m * c->elt,
                               hipMemcpyHostToDevice, s),
                "upload factors");
      hip_check(hipStreamSynchronize(s), "upload sync");
    }
  } catch (...) {
    (void)hipHostFree(stage);
    throw;
  }
  (void)hipHostFree(stage);
}

// Exact FP64 diagonal blocks of the super-leaves without z (row-major ns x ns),
// cached on the host for refactoring.
void superleaf_entries(hbf_ctx* c, EntryEval* ev) {
  const Plan& P = c->P;
  const int64_t ns = static_cast<int64_t>(P.n0) << P.sl;
  const int64_t nsl = P.n / ns;
  c->sl_noz.assign(static_cast<size_t>(nsl * ns * ns), cd{0, 0});
  if (ev) {
    // row-major blocks: out[i ns + j] = A(S ns + i, S ns + j) is the job's
    // column-major product with rows = columns = the super-leaf's indices, swapped
    static_assert(sizeof(cd) == sizeof(cplx), "complex layouts");
    constexpr int64_t kBatch = 512;
    std::vector<std::vector<int32_t>> sets(static_cast<size_t>(std::min(nsl, kBatch)));
    for (int64_t S0 = 0; S0 < nsl; S0 += kBatch) {
      const int64_t S1 = std::min(nsl, S0 + kBatch);
      std::vector<EntryJob> jobs;
      for (int64_t S = S0; S < S1; ++S) {
        std::vector<int32_t>& v = sets[S - S0];
        v.resize(static_cast<size_t>(ns));
        for (int64_t i = 0; i < ns; ++i) v[i] = static_cast<int32_t>(S * ns + i);
        jobs.push_back({v.data(), static_cast<int32_t>(ns), v.data(), static_cast<int32_t>(ns), 1,
                        reinterpret_cast<cplx*>(&c->sl_noz[static_cast<size_t>(S * ns * ns)])});
      }
      ev->eval(jobs);
    }
    if (!P.z.empty())
      for (int64_t S = 0; S < nsl; ++S)
        for (int64_t i = 0; i < ns; ++i) {
          cd& d = c->sl_noz[static_cast<size_t>((S * ns + i) * ns + i)];
          d.x -= P.z[S * ns + i].real();
          d.y -= P.z[S * ns + i].imag();
        }
    return;
  }
  const int T = std::max(1, build_threads(nullptr));
  std::vector<std::thread> th;
  std::atomic<int64_t> next(0);
  for (int t = 0; t < T; ++t)
    th.emplace_back([&]() {
      for (;;) {
        const int64_t S = next.fetch_add(1);
        if (S >= nsl) return;
        for (int64_t i = 0; i < ns; ++i)
          for (int64_t j = 0; j < ns; ++j) {
            cplx v = (i == j) ? P.self_entry(S * ns + i) : P.entry(S * ns + i, S * ns + j);
            if (i == j && !P.z.empty()) v -= P.z[S * ns + i];
            c->sl_noz[(S * ns + i) * ns + j] = cd{v.real(), v.imag()};
          }
      }
    });
  for (auto& x : th) x.join();
}

// Super-leaf inverses with the current impedance, computed on the device in FP64.
void factor_leaves(hbf_ctx* c, hipStream_t s) {
  if (c->prec == HBF_PREC_NONE || c->P.sl_fwd.empty()) return;
  const Plan& P = c->P;
  const int n0 = P.n0;
  const int64_t ns = static_cast<int64_t>(n0) << P.sl;
  const int64_t nsl = P.n / ns;
  const int64_t blk = ns * ns;
  // one workgroup factors one super-leaf; a batch of up to 2 GiB of blocks and
  // workspace (4 blocks per super-leaf) keeps every CU busy
  const int64_t batch = std::min<int64_t>(nsl, std::max<int64_t>(64, (int64_t(2) << 30) / (4 * blk * 16)));
  SuperleafOut so;
  const int64_t per = static_cast<int64_t>(n0) * n0 * (1 << P.sl) * ((1 << P.sl) + 1) / 2;
  so.per_superleaf = per;
  so.slab = P.sl_slab;
  for (int set = 0; set < 4; ++set) so.base[set] = P.leaf_fac_begin + set * nsl * per;
  cd* dA = nullptr;
  cd* work = nullptr;
  hip_check(hipMemsetAsync(c->d_flag, 0, sizeof(int), s), "memset flag");
  dmalloc(&dA, static_cast<size_t>(batch * blk) * sizeof(cd), "superleaf blocks");
  try {
    dmalloc(&work, static_cast<size_t>(batch * 3 * blk) * sizeof(cd), "superleaf work");
    std::vector<cd> H(static_cast<size_t>(batch * blk));
    const int mode = (c->prec == HBF_PREC_PAPER_TRI) ? 1 : 0;
    for (int64_t S0 = 0; S0 < nsl; S0 += batch) {
      const int64_t nb = std::min(batch, nsl - S0);
      std::memcpy(H.data(), &c->sl_noz[S0 * blk], static_cast<size_t>(nb * blk) * sizeof(cd));
      if (!P.z.empty())
        for (int64_t b = 0; b < nb; ++b)
          for (int64_t i = 0; i < ns; ++i) {
            cd& d = H[b * blk + i * ns + i];
            d.x += P.z[(S0 + b) * ns + i].real();
            d.y += P.z[(S0 + b) * ns + i].imag();
          }
      hip_check(hipMemcpyAsync(dA, H.data(), static_cast<size_t>(nb * blk) * sizeof(cd), hipMemcpyHostToDevice, s),
                "upload superleaf");
      hip_check(launch_superleaf_factor(dA, S0, nb, static_cast<int>(ns), n0, mode, P.scale.real(), P.scale.imag(),
                                        c->d_fac, c->dtype == HBF_C128, so, c->d_flag, work, s),
                "superleaf factor");
      hip_check(hipStreamSynchronize(s), "superleaf sync");
    }
    int flag = 0;
    hip_check(hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s), "flag");
    hip_check(hipStreamSynchronize(s), "leaf sync");
    dfree(work);
    dfree(dA);
    work = nullptr;
    dA = nullptr;
    if (flag) throw std::domain_error("a leaf block is singular to working precision");
  } catch (...) {
    dfree(work);
    dfree(dA);
    throw;
  }
}

// One-entry process cache of a host factorisation (factor entries included),
// keyed by everything the construction depends on.
struct PlanCache {
  std::mutex mu;
  bool valid = false;
  uint64_t key = 0;
  Plan plan;
};
PlanCache& plan_cache() {
  static PlanCache c;
  return c;
}

uint64_t plan_key(const hbf_curve* curve, double kappa, int leaf, double tol, const hbf_build_opts* opts) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
  };
  mix(&curve->ncurves, sizeof(curve->ncurves));
  mix(curve->node_off, sizeof(int64_t) * (curve->ncurves + 1));
  mix(curve->xy, sizeof(double) * 2 * curve->node_off[curve->ncurves]);
  mix(&kappa, sizeof(kappa));
  mix(&leaf, sizeof(leaf));
  mix(&tol, sizeof(tol));
  const int prec = opts ? opts->prec : 0;
  mix(&prec, sizeof(prec));
  const double eta0 = opts ? opts->eta0 : 0.0;
  mix(&eta0, sizeof(eta0));
  const int sl = opts ? opts->superleaf : 0;
  mix(&sl, sizeof(sl));
  if (opts && opts->z) {
    const int64_t n = curve->node_off[curve->ncurves] - curve->ncurves;
    mix(opts->z, sizeof(double) * 2 * n);
  }
  return h;
}

hbf_status fail(hbf_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

}  // namespace

namespace hbf {

// Build the sweep schedules for the context's settings and upload their step
// tables and unit copies (throws on allocation or copy failure).
// Lane tables of the one-RHS forward matvec launches of single units (the
// direct launches of c->mv_fwd): a wave takes a run of consecutive units
// whose lanes fill at most 64, or a 64-row slice of a unit of more than 64
// outputs; lane l of wave w computes the output
// lmap[64 w + l] = (unit - wfirst[w]) << 8 | row (0xffff: idle) in the role
// lrole[64 w + l].  With lane_scatter_split, a SCATTER unit whose rows fit one
// wave gives each row redundant in both IDs two adjacent lanes (the owner runs
// the first ID's dot product, its partner the second's), so every lane runs at
// most one loop.  Replaces the context's tables.
void build_lane_tables(hbf_ctx* c) {
  const Plan& P = c->P;
  std::vector<int32_t> lw;
  std::vector<uint16_t> lm, lr;
  for (size_t li = 0; li < c->mv_fwd.size(); ++li) {
    Launch& l = c->mv_fwd[li];
    l.lw_first = l.lw_count = l.lw_mean = l.lw_split = 0;
    if (!l.direct || l.count <= 0) continue;
    // the launch's units in order (for launch-order copies: the first unit of
    // each group of the plan's launch)
    const Launch& pl = P.mv_fwd[li];
    auto unit = [&](int32_t u) -> const Unit& {
      return l.ucopy ? P.units[P.group_units[P.group_off[pl.first + (u - l.first)]]] : P.units[u];
    };
    int64_t ent = 0;
    for (int32_t u = l.first; u < l.first + l.count; ++u) ent += unit(u).mat_len;
    l.lw_mean = static_cast<int32_t>(ent / l.count);
    l.lw_first = static_cast<int32_t>(lw.size());
    auto open_wave = [&](int32_t u) {
      lw.push_back(u);
      lm.resize(lw.size() * 64, 0xffff);
      lr.resize(lw.size() * 64, 0);
    };
    std::vector<std::pair<uint16_t, uint16_t>> items;  // (row, role) of one unit
    int32_t run = -1;  // first unit of the open run (-1: none)
    int fill = 0;
    for (int32_t u = l.first; u < l.first + l.count; ++u) {
      const Unit& U = unit(u);
      const int n = U.out_len[0] + U.out_len[1];
      if (n > 64) {
        for (int o0 = 0; o0 < n; o0 += 64) {
          open_wave(u);
          for (int o = o0; o < std::min(n, o0 + 64); ++o) {
            lm[(lw.size() - 1) * 64 + (o - o0)] = static_cast<uint16_t>(o);
            lr[(lw.size() - 1) * 64 + (o - o0)] = kLaneWhole;
          }
        }
        run = -1;
        continue;
      }
      items.clear();
      if (c->lane_scatter_split && U.type == UNIT_SCATTER) {
        const uint8_t* pp = P.perm.data() + U.perm;
        for (int o = 0; o < n; ++o) {
          const bool d0 = pp[o] >= U.k[0], d1 = pp[n + o] >= U.k[1];
          if (d0 && d1) {
            items.push_back({static_cast<uint16_t>(o), kLaneSplit | kLaneOwner | kLaneDot0 | kLanePartner});
            items.push_back({static_cast<uint16_t>(o), kLaneSplit | kLaneDot1});
          } else {
            items.push_back({static_cast<uint16_t>(o),
                             static_cast<uint16_t>(kLaneSplit | kLaneOwner | (d0 ? kLaneDot0 : 0) |
                                                   (d1 ? kLaneDot1 : 0))});
          }
        }
      }
      if (items.empty() || items.size() > 64) {
        items.clear();
        for (int o = 0; o < n; ++o) items.push_back({static_cast<uint16_t>(o), kLaneWhole});
      }
      const int ni = static_cast<int>(items.size());
      if (run < 0 || fill + ni > 64 || u - run > 255) {
        run = u;
        fill = 0;
        open_wave(u);
      }
      for (int i = 0; i < ni; ++i) {
        const size_t e = (lw.size() - 1) * 64 + fill + i;
        lm[e] = static_cast<uint16_t>(((u - run) << 8) | items[i].first);
        uint16_t role = items[i].second;
        if (role & kLanePartner) role = static_cast<uint16_t>(role | ((fill + i + 1) << 8));  // the next lane
        if (role & kLaneSplit) l.lw_split = 1;
        lr[e] = role;
      }
      fill += ni;
    }
    l.lw_count = static_cast<int32_t>(lw.size()) - l.lw_first;
  }
  dfree(c->d_lwaves);
  dfree(c->d_lmap);
  dfree(c->d_lrole);
  c->d_lwaves = nullptr;
  c->d_lmap = nullptr;
  c->d_lrole = nullptr;
  dmalloc(&c->d_lwaves, std::max<size_t>(lw.size(), 1) * sizeof(int32_t), "units");
  dmalloc(&c->d_lmap, std::max<size_t>(lm.size(), 1) * sizeof(uint16_t), "units");
  dmalloc(&c->d_lrole, std::max<size_t>(lr.size(), 1) * sizeof(uint16_t), "units");
  if (!lw.empty()) {
    hip_check(hipMemcpy(c->d_lwaves, lw.data(), lw.size() * sizeof(int32_t), hipMemcpyHostToDevice), "units");
    hip_check(hipMemcpy(c->d_lmap, lm.data(), lm.size() * sizeof(uint16_t), hipMemcpyHostToDevice), "units");
    hip_check(hipMemcpy(c->d_lrole, lr.data(), lr.size() * sizeof(uint16_t), hipMemcpyHostToDevice), "units");
  }
}

void rebuild_sweeps(hbf_ctx* c, int prog_levels) {
  // LDS-resident programs exist only for the pipelined program kernel
  const int lds_rows = (c->prog_lds && c->prog_pipe)
                           ? prog_lds_rows_budget(static_cast<int>(c->elt), static_cast<int>(c->elt))
                           : 0;
  build_sweeps(c->P, c->S, prog_levels, lds_rows);
  dfree(c->d_steps);
  c->d_steps = nullptr;
  dfree(c->d_punits);
  c->d_punits = nullptr;
  dmalloc(&c->d_steps, std::max<size_t>(c->S.steps.size(), 1) * sizeof(int32_t), "steps");
  if (!c->S.steps.empty())
    hip_check(hipMemcpy(c->d_steps, c->S.steps.data(), c->S.steps.size() * sizeof(int32_t), hipMemcpyHostToDevice),
              "steps");
  dmalloc(&c->d_punits, std::max<size_t>(c->S.punits.size(), 1) * sizeof(Unit), "program units");
  if (!c->S.punits.empty())
    hip_check(hipMemcpy(c->d_punits, c->S.punits.data(), c->S.punits.size() * sizeof(Unit), hipMemcpyHostToDevice),
              "program units");
}

hipError_t run_launches(hbf_ctx* c, const std::vector<Launch>& L, bool adjoint, void* X, void* Y, int R,
                        bool vec_c128, double alpha_re, double alpha_im, hipStream_t s, bool sweep, void* arena) {
  void* const ar = arena ? arena : c->d_arena;
  const size_t szA = (vec_c128 || c->dtype == HBF_C128) ? 16 : 8;
  const size_t szF = c->elt;
  const int ch_cap = static_cast<int>(32768 / szF);
  for (const Launch& l : L) {
    if (l.prog) {
      // one workgroup per RHS chunk; each wave is a pipelined team
      StageArgs a;
      const bool lv = l.lv_rows > 0;
      a.units = lv ? c->d_punits : c->d_units;
      a.lv_rows = lv ? l.lv_rows : 0;
      a.prow0 = l.prow0;
      a.prows = l.prows;
      a.gofs = c->d_gofs;
      a.gunits = c->d_gunits;
      a.fac = c->d_fac;
      a.perm = c->d_perm;
      a.buf[BUF_X] = X;
      a.buf[BUF_Y] = Y;
      a.buf[BUF_ARENA] = ar;
      a.first = 0;
      a.direct = 1;
      a.R = R;
      const int mx = std::max({1, l.max_dst, l.max_src});
      const int rc = std::min(R, std::max(1, 256 / mx));
      a.rc = rc;
      a.nchunks = (R + rc - 1) / rc;
      a.acc = 0;
      a.alpha_re = alpha_re;
      a.alpha_im = alpha_im;
      a.src_cap = 0;
      a.ch = 0;
      a.split = c->lane_split ? 1 : 0;
      hipError_t e;
      if (c->prog_pipe) {
        e = (c->dtype == HBF_C128) ? launch_prog_pipe_c128(a, c->d_steps, l.first, l.first + l.count, adjoint, s)
                                   : launch_prog_pipe_c64(a, c->d_steps, l.first, l.first + l.count, adjoint, s);
      } else {
        const int mdo = std::max(1, l.max_dst);
        int rc2 = std::min(R, std::max(1, (64 * kProgOutPerThread) / mdo));
        const int wave_lds = 8192;
        while (rc2 > 1 && static_cast<size_t>(l.max_src) * rc2 * szA > 2048) --rc2;
        a.rc = rc2;
        a.nchunks = (R + rc2 - 1) / rc2;
        a.src_cap = std::max(1, l.max_src * rc2);
        int ch = static_cast<int>((wave_lds - 1024 - static_cast<size_t>(a.src_cap) * szA) / szF);
        ch &= ~1;
        ch = std::min(ch, (l.max_mat + 1) & ~1);
        if (ch < 2) ch = 2;
        a.ch = ch;
        e = (c->dtype == HBF_C128) ? launch_program_c128(a, c->d_steps, l.first, l.first + l.count, wave_lds, adjoint, s)
                                   : launch_program_c64(a, c->d_steps, l.first, l.first + l.count, wave_lds, adjoint, s);
      }
      if (e != hipSuccess) return e;
      continue;
    }
    StageArgs a;
    a.units = l.ucopy ? c->d_lunits : c->d_units;
    a.gofs = c->d_gofs;
    a.gunits = c->d_gunits;
    a.fac = c->d_fac;
    a.perm = c->d_perm;
    a.buf[BUF_X] = X;
    a.buf[BUF_Y] = Y;
    a.buf[BUF_ARENA] = ar;
    a.first = l.first;
    a.direct = l.direct;
    a.R = R;
    const int md = std::max(1, l.max_dst);
    const bool adj = adjoint && !l.force_fwd;
    const int mxp = std::max({1, l.max_dst, l.max_src});
    if (c->mfma && c->dtype == HBF_C64 && !vec_c128 && R >= c->mfma_min_r) {
      a.rc = R;
      a.nchunks = 1;
      a.acc = l.out_leaf;
      a.alpha_re = alpha_re;
      a.alpha_im = alpha_im;
      a.src_cap = 0;
      a.ch = 0;
      // a launch of few waves (groups x RHS chunks) gives every 16-row output
      // tile of a group a wave of its own: its chain of dependent steps is
      // then one tile long; a launch that fills the device keeps one wave per
      // group, which reads the group's sources once for all its tiles
      const int tiles = sweep ? c->sweep_mfma_tiles : c->mfma_tiles;
      const int64_t gw = static_cast<int64_t>(l.count) * ((R + 16 * tiles - 1) / (16 * tiles));
      const int mtiles = gw < c->mfma_split_rows ? std::max(1, ((adj ? l.max_in : l.max_out) + 15) / 16) : 1;
      const hipError_t e = launch_stage_mfma_c64(a, l.count, tiles, mtiles, adj, s);
      if (e != hipSuccess) return e;
      continue;
    }
    // launches of big units (the leaf transfers of 64-row sources, the middle
    // couplings) stay with the wave-per-unit kernels, which stream a unit's
    // matrix with whole-wave loads
    if (R == 1 && !sweep && !adj && c->lane_units && l.lw_count > 0 && l.lw_mean <= c->lane_max_entries) {
      a.rc = 1;
      a.nchunks = 1;
      a.acc = l.out_leaf;
      a.alpha_re = alpha_re;
      a.alpha_im = alpha_im;
      const int32_t* wf = c->d_lwaves + l.lw_first;
      const uint16_t* lmap = c->d_lmap + static_cast<int64_t>(l.lw_first) * 64;
      const uint16_t* lrole = l.lw_split ? c->d_lrole + static_cast<int64_t>(l.lw_first) * 64 : nullptr;
      hipError_t e;
      if (c->dtype == HBF_C128) e = launch_lanes_c128(a, wf, lmap, lrole, l.lw_count, s);
      else if (vec_c128) e = launch_lanes_c64_hi(a, wf, lmap, lrole, l.lw_count, s);
      else e = launch_lanes_c64(a, wf, lmap, lrole, l.lw_count, s);
      if (e != hipSuccess) return e;
      continue;
    }
    const int pmr = sweep ? c->sweep_pipe_max_r : c->pipe_max_r;
    const bool rc1 = sweep && c->sweep_rc1 && R > pmr;
    if ((R <= pmr || rc1) && mxp <= 256) {
      const int rc = rc1 ? 1 : std::min(R, std::max(1, 256 / mxp));
      a.rc = rc;
      a.nchunks = (R + rc - 1) / rc;
      a.acc = l.out_leaf;
      a.alpha_re = alpha_re;
      a.alpha_im = alpha_im;
      a.src_cap = 0;
      a.ch = 0;
      a.split = c->lane_split ? 1 : 0;
      a.single = l.single;
      hipError_t e;
      if (c->dtype == HBF_C128) e = launch_pipe_c128(a, l.count, a.nchunks, adj, c->r1_max_blocks, s);
      else if (vec_c128) e = launch_pipe_c64_hi(a, l.count, a.nchunks, adj, c->r1_max_blocks, s);
      else e = launch_pipe_c64(a, l.count, a.nchunks, adj, c->r1_max_blocks, s);
      if (e != hipSuccess) return e;
      continue;
    }
    if (c->wave_units && md * std::min(R, 2) <= 64 * kWaveOutPerThread && R <= 2) {
      // small groups: one wave per group
      a.rc = R;
      a.nchunks = 1;
      a.acc = l.out_leaf;
      a.alpha_re = alpha_re;
      a.alpha_im = alpha_im;
      a.src_cap = std::max(1, l.max_src * R);
      const int wave_lds = 8192;
      int ch = static_cast<int>((wave_lds - 1024 - static_cast<size_t>(a.src_cap) * szA) / szF);
      ch &= ~1;
      ch = std::min(ch, (l.max_mat + 1) & ~1);
      if (ch < 2) ch = 2;
      a.ch = ch;
      hipError_t e;
      if (c->dtype == HBF_C128) e = launch_stage_wave_c128(a, l.count, wave_lds, adj, s);
      else if (vec_c128) e = launch_stage_wave_c64_hi(a, l.count, wave_lds, adj, s);
      else e = launch_stage_wave_c64(a, l.count, wave_lds, adj, s);
      if (e != hipSuccess) return e;
      continue;
    }
    int rc = std::min(R, std::max(1, (kStageThreads * kOutPerThread) / md));
    while (rc > 1 && static_cast<size_t>(l.max_src) * rc * szA > 24576) --rc;
    a.rc = rc;
    a.nchunks = (R + rc - 1) / rc;
    a.acc = l.out_leaf;
    a.alpha_re = alpha_re;
    a.alpha_im = alpha_im;
    int ch = std::min(ch_cap, (l.max_mat + 1) & ~1);
    if (ch < 2) ch = 2;
    a.ch = ch;
    a.src_cap = std::max(1, l.max_src * rc);
    const size_t lds = static_cast<size_t>(a.src_cap) * szA + static_cast<size_t>(ch) * szF + 1024;
    hipError_t e;
    if (c->dtype == HBF_C128) e = launch_stage_c128(a, l.count, adj, lds, s);
    else if (vec_c128) e = launch_stage_c64_hi(a, l.count, adj, lds, s);
    else e = launch_stage_c64(a, l.count, adj, lds, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hbf_status matvec_internal(hbf_ctx* c, void* xin, void* yout, int R, bool vec_c128, bool adjoint, hipStream_t s,
                           void* arena) {
  hipError_t e;
  const std::vector<Launch>& fw = c->mv_direct ? c->mv_fwd : c->P.mv_fwd;
  const std::vector<Launch>& bw = c->mv_direct ? c->mv_adj : c->P.mv_adj;
  if (!adjoint) e = run_launches(c, fw, false, xin, yout, R, vec_c128, 1.0, 0.0, s, false, arena);
  else e = run_launches(c, bw, true, yout, xin, R, vec_c128, 1.0, 0.0, s, false, arena);
  if (e != hipSuccess) return fail(HBF_EHIP, std::string("matvec launch: ") + hipGetErrorString(e));
  return HBF_OK;
}

// The two sweeps of the preconditioner (input in d_u, output in zout).
hipError_t enqueue_sweeps(hbf_ctx* c, void* zout, int R, bool adjoint, hipStream_t s) {
  const bool paper = c->prec == HBF_PREC_PAPER_TRI;
  const double are = paper ? c->P.scale.real() : 1.0, aim = paper ? c->P.scale.imag() : 0.0;
  const bool v128 = c->dtype == HBF_C128;
  hipError_t e;
  if (!adjoint) {
    e = run_launches(c, c->S.fwd, false, c->d_t, c->d_u, R, v128, -are, -aim, s, true);
    if (e == hipSuccess && !paper) e = run_launches(c, c->S.diag, false, c->d_t, c->d_u, R, v128, 1.0, 0.0, s, true);
    if (e == hipSuccess) {
      void* mid = paper ? c->d_t : c->d_u;
      e = run_launches(c, c->S.bwd, false, zout, mid, R, v128, -1.0, 0.0, s, true);
    }
  } else {
    e = run_launches(c, c->S.adj_fwd, true, c->d_u, c->d_t, R, v128, -1.0, 0.0, s, true);
    if (e == hipSuccess && !paper) e = run_launches(c, c->S.diag, true, c->d_u, c->d_t, R, v128, 1.0, 0.0, s, true);
    if (e == hipSuccess) {
      void* mid = paper ? c->d_t : c->d_u;
      e = run_launches(c, c->S.adj_bwd, true, mid, zout, R, v128, -are, aim, s, true);
    }
  }
  return e;
}

// z = P^{-1} r (or P^{-H} r); r, z internal layout, vector dtype = context dtype.
// The sweep launches are captured once per (nrhs, adjoint) into a HIP graph and
// replayed; the graph reads d_u and writes d_pz, copied in and out around it.
hbf_status precond_internal(hbf_ctx* c, const void* rin, void* zout, int R, bool adjoint, hipStream_t s) {
  const size_t bytes = static_cast<size_t>(c->n) * R * c->elt;
  hipError_t e = hipMemcpyAsync(c->d_u, rin, bytes, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return fail(HBF_EHIP, "precond copy");
  if (c->prec == HBF_PREC_NONE) {
    e = hipMemcpyAsync(zout, c->d_u, bytes, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? HBF_OK : fail(HBF_EHIP, "precond copy");
  }
  if (!c->use_graphs) {
    e = enqueue_sweeps(c, zout, R, adjoint, s);
    if (e != hipSuccess) return fail(HBF_EHIP, std::string("precond launch: ") + hipGetErrorString(e));
    return HBF_OK;
  }
  const auto key = std::make_pair(R, adjoint ? 1 : 0);
  auto it = c->pc_graphs.find(key);
  if (it == c->pc_graphs.end()) {
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(HBF_EHIP, "graph stream");
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e2 = enqueue_sweeps(c, c->d_pz, R, adjoint, cs);
      e = hipStreamEndCapture(cs, &g);
      if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return fail(HBF_EHIP, std::string("precond graph: ") + hipGetErrorString(e));
    it = c->pc_graphs.emplace(key, ge).first;
  }
  e = hipGraphLaunch(it->second, s);
  if (e == hipSuccess) e = hipMemcpyAsync(zout, c->d_pz, bytes, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return fail(HBF_EHIP, std::string("precond graph launch: ") + hipGetErrorString(e));
  return HBF_OK;
}

}  // namespace hbf

extern "C" {

hbf_status hbf_build(const hbf_curve* curve, double kappa, int32_t leaf, double tol, const hbf_build_opts* opts,
                     hbf_ctx** out) {
  if (!out) return fail(HBF_EINVAL, "hbf_build: out is NULL");
  *out = nullptr;
  auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<hbf_ctx> c(new (std::nothrow) hbf_ctx());
  if (!c) return fail(HBF_ENOMEM, "hbf_build: out of host memory");
  hipStream_t s = nullptr;
  try {
    c->dtype = opts ? opts->dtype : HBF_C64;
    c->prec = opts ? opts->prec : HBF_PREC_BLOCK_LU;
    if (c->dtype != HBF_C64 && c->dtype != HBF_C128) return fail(HBF_EINVAL, "hbf_build: bad dtype");
    if (c->prec != HBF_PREC_BLOCK_LU && c->prec != HBF_PREC_PAPER_TRI && c->prec != HBF_PREC_NONE)
      return fail(HBF_EINVAL, "hbf_build: bad preconditioner");
    if (leaf > 64) return fail(HBF_EINVAL, "hbf_build: the device path supports leaf <= 64");
    c->max_nrhs = (opts && opts->max_nrhs > 0) ? opts->max_nrhs : 1;
    c->restart = (opts && opts->restart > 0) ? std::min(opts->restart, 255) : 30;
    c->device = opts ? opts->device : 0;
    c->elt = c->dtype == HBF_C64 ? 8 : 16;
    const bool verbose = opts && opts->verbose;
    auto progress = [&](const char* what) {
      if (!verbose) return;
      const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      std::fprintf(stderr, "[hbf] %s (%.1f s)\n", what, sec);
      std::fflush(stderr);
    };
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
      (void)hipGetLastError();
      return fail(HBF_EHIP, "hbf_build: no HIP device");
    }
    if (c->device < 0 || c->device >= ndev) return fail(HBF_EINVAL, "hbf_build: bad device ordinal");
    hip_check(hipSetDevice(c->device), "hipSetDevice");
    hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");

    if (!curve || curve->ncurves < 1 || !curve->node_off || !curve->xy)
      return fail(HBF_EINVAL, "hbf_build: empty curve");
    {
      const uint64_t key = plan_key(curve, kappa, leaf, tol, opts);
      PlanCache& pc = plan_cache();
      bool hit = false;
      {
        std::lock_guard<std::mutex> lk(pc.mu);
        if (pc.valid && pc.key == key) {
          c->P = pc.plan;
          hit = true;
        }
      }
      if (!hit) {
        std::unique_ptr<EntryEval> ev;
        if (!(opts && opts->host_entries)) ev = make_device_entry_eval(c->device);
        build_plan(c->P, curve, kappa, leaf, tol, opts, ev.get());
        progress("host plan built");
        if (opts && opts->cache_plan) {
          std::lock_guard<std::mutex> lk(pc.mu);
          pc.plan = c->P;
          pc.key = key;
          pc.valid = true;
        }
      }
    }
    Plan& P = c->P;
    c->n = P.n;
    c->n_ext = P.n_real;
    const int64_t N = P.n;
    c->vmap.n_int = P.n;
    c->vmap.n_ext = P.n_real;
    if (c->padded()) {
      // device copies of the padding map (library row <-> caller's unknown)
      std::vector<int32_t> real_of(static_cast<size_t>(P.n), -1);
      for (int64_t j = 0; j < P.n_real; ++j) real_of[P.lib_of[j]] = static_cast<int32_t>(j);
      dmalloc(&c->d_real_of, real_of.size() * sizeof(int32_t), "padding map");
      dmalloc(&c->d_lib_of, P.lib_of.size() * sizeof(int32_t), "padding map");
      hip_check(hipMemcpy(c->d_real_of, real_of.data(), real_of.size() * sizeof(int32_t), hipMemcpyHostToDevice),
                "padding map");
      hip_check(hipMemcpy(c->d_lib_of, P.lib_of.data(), P.lib_of.size() * sizeof(int32_t), hipMemcpyHostToDevice),
                "padding map");
      c->vmap.real_of = c->d_real_of;
      c->vmap.lib_of = c->d_lib_of;
    }
    const int n0 = P.n0;
    const int64_t nl = N / n0;
    const int64_t bs = static_cast<int64_t>(n0) * n0;
    // keep FP64 leaf blocks without z for refactoring
    c->diag_noz.resize(static_cast<size_t>(nl * bs));
    for (int64_t b = 0; b < nl; ++b) {
      const Unit& u = P.units[P.diag_unit[b]];
      for (int64_t e = 0; e < bs; ++e) {
        cplx v = P.fac[u.mat + e];
        c->diag_noz[b * bs + e] = cd{v.real(), v.imag()};
      }
      if (!P.z.empty())
        for (int i = 0; i < n0; ++i) {
          cd& d = c->diag_noz[b * bs + static_cast<int64_t>(i) * n0 + i];
          d.x -= P.z[b * n0 + i].real();
          d.y -= P.z[b * n0 + i].imag();
        }
    }
    const int64_t fac_entries = P.leaf_fac_begin + P.leaf_fac_len;
    // 16 spare entries: the sweep programs' L2 prefetch touches whole 16-entry granules
    dmalloc(&c->d_fac, static_cast<size_t>(fac_entries + 16) * c->elt, "factors");
    upload_factors(c.get(), 0, P.leaf_fac_begin, s);
    dmalloc(&c->d_perm, P.perm.size() + 16, "perm");
    if (!P.perm.empty())
      hip_check(hipMemcpy(c->d_perm, P.perm.data(), P.perm.size(), hipMemcpyHostToDevice), "upload perm");
    dmalloc(&c->d_units, P.units.size() * sizeof(Unit), "units");
    hip_check(hipMemcpy(c->d_units, P.units.data(), P.units.size() * sizeof(Unit), hipMemcpyHostToDevice), "units");
    dmalloc(&c->d_gofs, P.group_off.size() * sizeof(int32_t), "groups");
    hip_check(hipMemcpy(c->d_gofs, P.group_off.data(), P.group_off.size() * sizeof(int32_t), hipMemcpyHostToDevice),
              "groups");
    dmalloc(&c->d_gunits, P.group_units.size() * sizeof(int32_t), "groups");
    hip_check(hipMemcpy(c->d_gunits, P.group_units.data(), P.group_units.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice),
              "groups");
    {
      // Matvec launches whose groups are single units run direct over copies
      // of their unit descriptors in launch order: a team finds each item's
      // descriptor without reading the group tables first.
      std::vector<Unit> lu;
      c->mv_fwd = P.mv_fwd;
      c->mv_adj = P.mv_adj;
      for (auto* L : {&c->mv_fwd, &c->mv_adj})
        for (Launch& l : *L) {
          if (l.direct || !l.single) continue;
          const int32_t base = static_cast<int32_t>(lu.size());
          for (int32_t g = l.first; g < l.first + l.count; ++g) lu.push_back(P.units[P.group_units[P.group_off[g]]]);
          l.first = base;
          l.direct = 1;
          l.ucopy = 1;
        }
      dmalloc(&c->d_lunits, std::max<size_t>(lu.size(), 1) * sizeof(Unit), "units");
      if (!lu.empty())
        hip_check(hipMemcpy(c->d_lunits, lu.data(), lu.size() * sizeof(Unit), hipMemcpyHostToDevice), "units");
    }
    build_lane_tables(c.get());
    progress("factors uploaded");
    rebuild_sweeps(c.get(), c->S.prog_levels);
    progress("sweep schedules built");
    prepare_launch_shapes();
    const size_t R = static_cast<size_t>(c->max_nrhs);
    const size_t vbytes = static_cast<size_t>(N) * R * 16;
    dmalloc(&c->d_arena, static_cast<size_t>(std::max<int64_t>(P.arena_rows, 1)) * R * 16, "arena");
    dmalloc(&c->d_vin, vbytes, "vectors");
    dmalloc(&c->d_vout, vbytes, "vectors");
    dmalloc(&c->d_u, vbytes, "vectors");
    dmalloc(&c->d_t, vbytes, "vectors");
    dmalloc(&c->d_pz, vbytes, "vectors");
    dmalloc(&c->d_flag, 256, "flag");
    // solver workspace (inner Krylov basis in the context dtype, FP64 outer vectors)
    const int nkry = solver_krylov_vectors(c->restart);
    dmalloc(&c->d_krylov, static_cast<size_t>(nkry) * N * R * c->elt, "krylov");
    dmalloc(&c->d_w, static_cast<size_t>(N) * R * c->elt, "krylov");
    dmalloc(&c->d_x64, 4 * vbytes, "solver vectors");
    c->red_len = static_cast<size_t>(2 * 34) * R * 1024;
    dmalloc(&c->d_red, c->red_len * sizeof(double), "reduction");
    dmalloc(&c->d_small, solver_small_bytes(c->restart, static_cast<int>(R)), "solver state");
    hip_check(hipHostMalloc(reinterpret_cast<void**>(&c->h_flags), 256, hipHostMallocDefault), "hipHostMalloc");
    for (auto& e : c->ev_step) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
    c->workspace_bytes = static_cast<size_t>(std::max<int64_t>(P.arena_rows, 1)) * R * 16 + 5 * vbytes +
                         static_cast<size_t>(nkry + 1) * N * R * c->elt + 4 * vbytes;
    if (c->prec != HBF_PREC_NONE) {
      std::unique_ptr<EntryEval> ev;
      if (!(opts && opts->host_entries)) {
        ev = make_device_entry_eval(c->device);
        ev->prepare(P);
      }
      superleaf_entries(c.get(), ev.get());
      progress("super-leaf blocks evaluated");
    }
    factor_leaves(c.get(), s);
    progress("leaf blocks factored");
    // release the host copies of the factors
    fill_stats(P, &c->stats, c->elt);
    c->stats.bytes_index = static_cast<int64_t>(P.perm.size() + P.units.size() * sizeof(Unit));
    {
      const int64_t vec = 2 * N * static_cast<int64_t>(c->elt);
      c->stats.apply_bytes_matvec = schedule_bytes(P, P.mv_fwd, nullptr, c->elt) + vec;
      c->stats.launches_matvec = static_cast<int64_t>(P.mv_fwd.size());
      int64_t nl = 0, ns = 0;
      if (c->prec != HBF_PREC_NONE)
        for (const auto* L : {&c->S.fwd, &c->S.bwd, &c->S.diag}) {
          if (L == &c->S.diag && c->prec != HBF_PREC_BLOCK_LU) continue;
          for (const Launch& l : *L) {
            nl += 1;
            ns += l.prog ? l.count : 1;
          }
        }
      c->stats.launches_precond = nl;
      c->stats.steps_precond = ns;
      c->stats.apply_bytes_precond =
          c->prec == HBF_PREC_NONE
              ? vec
              : schedule_bytes(P, c->S.fwd, &c->S.steps, c->elt, &c->S.punits) +
                    schedule_bytes(P, c->S.bwd, &c->S.steps, c->elt, &c->S.punits) +
                    (c->prec == HBF_PREC_BLOCK_LU ? schedule_bytes(P, c->S.diag, nullptr, c->elt) : 0) + vec;
    }
    std::vector<cplx>().swap(P.fac);
    hip_check(hipStreamSynchronize(s), "build sync");
    (void)hipStreamDestroy(s);
    s = nullptr;
    c->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    c->stats.build_seconds = c->build_seconds;
    c->stats.bytes_workspace = static_cast<int64_t>(c->workspace_bytes);
    *out = c.release();
    return HBF_OK;
  } catch (const std::invalid_argument& e) {
    if (s) (void)hipStreamDestroy(s);
    free_device(c.get());
    return fail(HBF_EINVAL, e.what());
  } catch (const std::bad_alloc&) {
    if (s) (void)hipStreamDestroy(s);
    free_device(c.get());
    return fail(HBF_ENOMEM, "hbf_build: out of memory");
  } catch (const std::domain_error& e) {
    if (s) (void)hipStreamDestroy(s);
    free_device(c.get());
    return fail(HBF_ESINGULAR, e.what());
  } catch (const std::exception& e) {
    if (s) (void)hipStreamDestroy(s);
    free_device(c.get());
    return fail(HBF_EHIP, e.what());
  }
}

hbf_status hbf_set_impedance(hbf_ctx* c, const double* z) {
  if (!c || !z) return fail(HBF_EINVAL, "hbf_set_impedance: NULL argument");
  for (int64_t i = 0; i < 2 * c->n_ext; ++i)
    if (!std::isfinite(z[i])) return fail(HBF_EINVAL, "hbf_set_impedance: non-finite impedance");
  try {
    hip_check(hipSetDevice(c->device), "hipSetDevice");
    // library order; padding rows keep z = 0 (their diagonal stays 1)
    c->P.z.assign(c->n, cplx(0.0, 0.0));
    for (int64_t i = 0; i < c->n_ext; ++i) c->P.z[c->P.lib(i)] = cplx(z[2 * i], z[2 * i + 1]);
    // refresh the dense diagonal units used by the matvec (their matrices hold A_bb)
    const int n0 = c->P.n0;
    const int64_t nl = c->n / n0;
    const int64_t bs = static_cast<int64_t>(n0) * n0;
    std::vector<cd> D(static_cast<size_t>(nl * bs));
    for (int64_t b = 0; b < nl; ++b) {
      for (int64_t e = 0; e < bs; ++e) D[b * bs + e] = c->diag_noz[b * bs + e];
      for (int i = 0; i < n0; ++i) {
        cd& d = D[b * bs + static_cast<int64_t>(i) * n0 + i];
        d.x += c->P.z[b * n0 + i].real();
        d.y += c->P.z[b * n0 + i].imag();
      }
    }
    // the rescaling follows the largest diagonal entry of the caller's unknowns
    {
      int64_t ib = 0;
      double best = -1.0;
      for (int64_t j = 0; j < c->n_ext; ++j) {
        const int64_t i = c->P.lib(j);
        const cd& d = D[(i / n0) * bs + (i % n0) * n0 + (i % n0)];
        const double m = std::hypot(d.x, d.y);
        if (m > best) { best = m; ib = i; }
      }
      const cd& d = D[(ib / n0) * bs + (ib % n0) * n0 + (ib % n0)];
      c->P.scale = 1.0 / cplx(d.x, d.y);
    }
    hipStream_t s = nullptr;
    for (int64_t b = 0; b < nl; ++b) {
      const Unit& u = c->P.units[c->P.diag_unit[b]];
      if (c->dtype == HBF_C64) {
        std::vector<float> f(2 * bs);
        for (int64_t e = 0; e < bs; ++e) {
          f[2 * e] = static_cast<float>(D[b * bs + e].x);
          f[2 * e + 1] = static_cast<float>(D[b * bs + e].y);
        }
        hip_check(hipMemcpy(static_cast<char*>(c->d_fac) + u.mat * c->elt, f.data(), bs * 8, hipMemcpyHostToDevice),
                  "diag upload");
      } else {
        hip_check(hipMemcpy(static_cast<char*>(c->d_fac) + u.mat * c->elt, &D[b * bs], bs * 16,
                            hipMemcpyHostToDevice),
                  "diag upload");
      }
    }
    factor_leaves(c, s);
    c->stats.scale_re = c->P.scale.real();
    c->stats.scale_im = c->P.scale.imag();
    return HBF_OK;
  } catch (const std::domain_error& e) {
    return fail(HBF_ESINGULAR, e.what());
  } catch (const std::bad_alloc&) {
    return fail(HBF_ENOMEM, "hbf_set_impedance: out of memory");
  } catch (const std::exception& e) {
    return fail(HBF_EHIP, e.what());
  }
}

hbf_status hbf_matvec(hbf_ctx* c, const void* x, void* y, int32_t nrhs, hbf_dtype io, int32_t adjoint, void* stream) {
  if (!c || !x || !y) return fail(HBF_EINVAL, "hbf_matvec: NULL argument");
  if (nrhs < 1 || nrhs > c->max_nrhs) return fail(HBF_EINVAL, "hbf_matvec: nrhs out of range [1, max_nrhs]");
  if (io != HBF_C64 && io != HBF_C128) return fail(HBF_EINVAL, "hbf_matvec: bad io dtype");
  if (c->dtype == HBF_C128 && io == HBF_C64) return fail(HBF_EINVAL, "hbf_matvec: complex64 io on a complex128 context");
  if (hipSetDevice(c->device) != hipSuccess) return fail(HBF_EHIP, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool v128 = io == HBF_C128;
  if (nrhs == 1 && !c->padded()) return matvec_internal(c, const_cast<void*>(x), y, 1, v128, adjoint != 0, s);
  if (launch_to_internal(x, v128, c->d_vin, v128, c->vmap, nrhs, s) != hipSuccess) return fail(HBF_EHIP, "layout");
  hbf_status st = matvec_internal(c, c->d_vin, c->d_vout, nrhs, v128, adjoint != 0, s);
  if (st != HBF_OK) return st;
  if (launch_to_external(c->d_vout, v128, y, v128, c->vmap, nrhs, s) != hipSuccess) return fail(HBF_EHIP, "layout");
  return HBF_OK;
}

hbf_status hbf_precond_apply(hbf_ctx* c, const void* r, void* z, int32_t nrhs, hbf_dtype io, int32_t adjoint,
                             void* stream) {
  if (!c || !r || !z) return fail(HBF_EINVAL, "hbf_precond_apply: NULL argument");
  if (nrhs < 1 || nrhs > c->max_nrhs) return fail(HBF_EINVAL, "hbf_precond_apply: nrhs out of range");
  if (io != c->dtype) return fail(HBF_EINVAL, "hbf_precond_apply: io dtype must equal the context dtype");
  if (hipSetDevice(c->device) != hipSuccess) return fail(HBF_EHIP, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool v128 = io == HBF_C128;
  if (nrhs == 1 && !c->padded()) return precond_internal(c, r, z, 1, adjoint != 0, s);
  if (launch_to_internal(r, v128, c->d_vin, v128, c->vmap, nrhs, s) != hipSuccess) return fail(HBF_EHIP, "layout");
  hbf_status st = precond_internal(c, c->d_vin, c->d_vout, nrhs, adjoint != 0, s);
  if (st != HBF_OK) return st;
  if (launch_to_external(c->d_vout, v128, z, v128, c->vmap, nrhs, s) != hipSuccess) return fail(HBF_EHIP, "layout");
  return HBF_OK;
}

hbf_status hbf_tune(hbf_ctx* c, const char* key, int64_t value) {
  if (!c || !key) return fail(HBF_EINVAL, "hbf_tune: NULL argument");
  const std::string k(key);
  if (hipSetDevice(c->device) != hipSuccess) return fail(HBF_EHIP, "hipSetDevice");
  if (k == "prog_levels") {
    if (value < 0 || value > 12) return fail(HBF_EINVAL, "hbf_tune: prog_levels out of range");
    (void)hipDeviceSynchronize();
    free_graphs(c);
    try {
      rebuild_sweeps(c, static_cast<int>(value));
    } catch (const std::exception& e) {
      return fail(HBF_ENOMEM, std::string("hbf_tune: ") + e.what());
    }
    return HBF_OK;
  }
  if (k == "lane_max_entries") {
    if (value < 0 || value > (1 << 20)) return fail(HBF_EINVAL, "hbf_tune: lane_max_entries out of range");
    (void)hipDeviceSynchronize();
    free_graphs(c);
    c->lane_max_entries = static_cast<int>(value);
    return HBF_OK;
  }
  if (k == "mfma_split_rows") {
    if (value < 0 || value > (int64_t(1) << 30)) return fail(HBF_EINVAL, "hbf_tune: mfma_split_rows out of range");
    (void)hipDeviceSynchronize();
    free_graphs(c);
    c->mfma_split_rows = static_cast<int>(value);
    return HBF_OK;
  }
  if (k == "lane_scatter_split") {
    if (value != 0 && value != 1) return fail(HBF_EINVAL, "hbf_tune: lane_scatter_split must be 0 or 1");
    (void)hipDeviceSynchronize();
    free_graphs(c);
    c->lane_scatter_split = value != 0;
    try {
      build_lane_tables(c);
    } catch (const std::exception& e) {
      return fail(HBF_ENOMEM, std::string("hbf_tune: ") + e.what());
    }
    return HBF_OK;
  }
  if (k == "lane_units" || k == "mv_direct") {
    if (value != 0 && value != 1) return fail(HBF_EINVAL, "hbf_tune: " + k + " must be 0 or 1");
    // the solver's captured steps hold the matvec and sweep launches
    (void)hipDeviceSynchronize();
    free_graphs(c);
    (k == "lane_units" ? c->lane_units : c->mv_direct) = value != 0;
    return HBF_OK;
  }
  if (k == "prog_lds") {
    (void)hipDeviceSynchronize();
    free_graphs(c);
    c->prog_lds = value != 0;
    try {
      rebuild_sweeps(c, c->S.prog_levels);
    } catch (const std::exception& e) {
      return fail(HBF_ENOMEM, std::string("hbf_tune: ") + e.what());
    }
    return HBF_OK;
  }
  if (k == "prog_pipe") {
    (void)hipDeviceSynchronize();
    free_graphs(c);
    c->prog_pipe = value != 0;
    try {
      rebuild_sweeps(c, c->S.prog_levels);
    } catch (const std::exception& e) {
      return fail(HBF_ENOMEM, std::string("hbf_tune: ") + e.what());
    }
    return HBF_OK;
  }
  if (k == "pipe_max_r") {
    if (value < 0 || value > 1024) return fail(HBF_EINVAL, "hbf_tune: pipe_max_r out of range");
    c->pipe_max_r = static_cast<int>(value);
    free_graphs(c);
    return HBF_OK;
  }
  if (k == "mfma") { c->mfma = value != 0; free_graphs(c); return HBF_OK; }
  if (k == "mfma_tiles" || k == "sweep_mfma_tiles") {
    if (value != 1 && value != 2 && value != 4) return fail(HBF_EINVAL, "hbf_tune: " + k + " must be 1, 2 or 4");
    (k == "mfma_tiles" ? c->mfma_tiles : c->sweep_mfma_tiles) = static_cast<int>(value);
    free_graphs(c);
    return HBF_OK;
  }
  if (k == "mfma_min_r") {
    if (value < 1 || value > 1 << 20) return fail(HBF_EINVAL, "hbf_tune: mfma_min_r out of range");
    c->mfma_min_r = static_cast<int>(value);
    free_graphs(c);
    return HBF_OK;
  }
  if (k == "wave_units") { c->wave_units = value != 0; free_graphs(c); return HBF_OK; }
  if (k == "lane_split") { c->lane_split = value != 0; free_graphs(c); return HBF_OK; }
  if (k == "sweep_rc1") { c->sweep_rc1 = value != 0; free_graphs(c); return HBF_OK; }
  if (k == "sweep_pipe_max_r") {
    if (value < 0 || value > 1024) return fail(HBF_EINVAL, "hbf_tune: sweep_pipe_max_r out of range");
    c->sweep_pipe_max_r = static_cast<int>(value);
    free_graphs(c);
    return HBF_OK;
  }
  if (k == "use_graphs") { c->use_graphs = value != 0; free_graphs(c); return HBF_OK; }
  if (k == "r1_max_blocks") {
    if (value < 0 || value > (1 << 20)) return fail(HBF_EINVAL, "hbf_tune: r1_max_blocks out of range");
    c->r1_max_blocks = static_cast<int>(value);
    free_graphs(c);
    return HBF_OK;
  }
  return fail(HBF_EINVAL, "hbf_tune: unknown key " + k);
}

hbf_status hbf_stats(const hbf_ctx* c, hbf_stats_t* out) {
  if (!c || !out) return fail(HBF_EINVAL, "hbf_stats: NULL argument");
  *out = c->stats;
  return HBF_OK;
}

int64_t hbf_size(const hbf_ctx* c) { return c ? c->n_ext : -1; }

void hbf_free(hbf_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  free_device(c);
  delete c;
}

}  // extern "C"
