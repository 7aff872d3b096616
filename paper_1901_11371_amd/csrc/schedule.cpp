// Sweep schedules (block forward / back substitution of Algorithms 3 and 4
// over the H-IDBF), the FP64 host executor of any schedule, the host leaf
// factorisation used by the construction checks, and the host-only C ABI.
#include <algorithm>
#include <cstdint>
#include <cmath>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <atomic>
#include <mutex>
#include <thread>

#include "hbf_internal.h"
#include "kernels.h"
#include "schedule.h"

namespace hbf {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// Sweeps.  The recursion over the diagonal tree follows Algorithm 3 (lower:
// first child, then the off-diagonal update of the second child, then the
// second child) and Algorithm 4 (upper: second child first).  For the
// adjoint preconditioner the systems are conjugate-transposed, so the lower
// sweep uses the upper blocks F12^H and the upper sweep the lower blocks
// F21^H, each traversed in reverse factor order.
// ---------------------------------------------------------------------------
namespace {

struct SweepGen {
  const Plan& P;
  const std::vector<int>& level_base;
  bool lower_dir, adjoint;
  const std::vector<int32_t>& leaf_units;   // first unit of each super-leaf
  std::vector<Launch>& out;
  std::vector<int32_t>& steps;
  int prog_levels;
  std::vector<Unit>* punits = nullptr;
  int lds_rows = 0;

  // Keep the program over rows [r0, r0 + nrows) in LDS if its vectors fit:
  // copy its units with every segment remapped to LDS rows (X rows at
  // [0, nrows), Y rows at [nrows, 2 nrows), each skeleton segment packed
  // after them) and point its steps at the copies.
  void make_lds(Launch& l, int64_t r0, int64_t nrows) const {
    if (!punits || lds_rows <= 0) return;
    std::vector<std::pair<int32_t, int32_t>> segs;  // arena (offset, length)
    for (int st = l.first; st < l.first + l.count; ++st) {
      for (int32_t q = steps[kStepInts * st]; q < steps[kStepInts * st + 1]; ++q) {
        const Unit& u = P.units[q];
        for (int side = 0; side < 2; ++side) {
          const uint8_t buf = side ? u.out_buf : u.in_buf;
          const int32_t* off = side ? u.out_off : u.in_off;
          const int16_t* len = side ? u.out_len : u.in_len;
          for (int sgi = 0; sgi < 2; ++sgi) {
            if (len[sgi] <= 0) continue;
            if (buf == BUF_ARENA) segs.push_back({off[sgi], len[sgi]});
            else if (off[sgi] < r0 || off[sgi] + len[sgi] > r0 + nrows) return;
          }
        }
      }
    }
    std::sort(segs.begin(), segs.end());
    segs.erase(std::unique(segs.begin(), segs.end()), segs.end());
    for (size_t i = 1; i < segs.size(); ++i)
      if (segs[i].first < segs[i - 1].first + segs[i - 1].second) return;  // overlapping segments
    // A skeleton segment's value lives from the step that writes it to the
    // last step that reads it (steps are separated by workgroup barriers), so
    // segments whose lives do not overlap share LDS rows.  refs: every arena
    // reference in step order (segment, instance); an instance starts at a
    // write.  A read of a segment no earlier step of the program wrote keeps
    // the program in HBM.
    struct Ref { size_t seg; int32_t inst; };
    std::vector<Ref> refs;
    std::vector<int32_t> inst_seg, inst_write, inst_last;  // per instance
    auto seg_index = [&](int32_t o, int16_t n) {
      return static_cast<size_t>(
          std::lower_bound(segs.begin(), segs.end(), std::pair<int32_t, int32_t>(o, static_cast<int32_t>(n))) -
          segs.begin());
    };
    {
      std::vector<int32_t> live(segs.size(), -1);
      for (int st = l.first; st < l.first + l.count; ++st) {
        // adjoint steps read the units' output segments and write their inputs
        const int read_side = (adjoint && !(steps[kStepInts * st + 2] & 2)) ? 1 : 0;
        for (int32_t q = steps[kStepInts * st]; q < steps[kStepInts * st + 1]; ++q) {
          const Unit& u = P.units[q];
          for (int side = 0; side < 2; ++side) {
            if ((side ? u.out_buf : u.in_buf) != BUF_ARENA) continue;
            const int32_t* off = side ? u.out_off : u.in_off;
            const int16_t* len = side ? u.out_len : u.in_len;
            for (int sgi = 0; sgi < 2; ++sgi) {
              if (len[sgi] <= 0) continue;
              const size_t i = seg_index(off[sgi], len[sgi]);
              if (side == read_side) {
                if (live[i] < 0 || inst_write[live[i]] >= st) return;
                inst_last[live[i]] = st;
              } else if (live[i] < 0 || inst_write[live[i]] != st) {
                live[i] = static_cast<int32_t>(inst_seg.size());
                inst_seg.push_back(static_cast<int32_t>(i));
                inst_write.push_back(st);
                inst_last.push_back(st);
              }
              refs.push_back({i, live[i]});
            }
          }
        }
      }
    }
    // first-fit placement from row 2 nrows on, in order of the writing step
    std::vector<int32_t> inst_row(inst_seg.size(), -1);
    int64_t total = 2 * nrows;
    {
      std::vector<std::pair<int64_t, int32_t>> used;  // (row, instance), sorted by row
      size_t k = 0;
      for (int st = l.first; st < l.first + l.count && k < inst_seg.size(); ++st) {
        used.erase(std::remove_if(used.begin(), used.end(),
                                  [&](const std::pair<int64_t, int32_t>& e) { return inst_last[e.second] < st; }),
                   used.end());
        for (; k < inst_seg.size() && inst_write[k] == st; ++k) {
          const int64_t need = segs[inst_seg[k]].second;
          int64_t row = 2 * nrows;
          size_t pos = 0;
          for (; pos < used.size(); ++pos) {
            if (used[pos].first - row >= need) break;
            row = std::max(row, used[pos].first + segs[inst_seg[used[pos].second]].second);
          }
          used.insert(used.begin() + static_cast<std::ptrdiff_t>(pos), {row, static_cast<int32_t>(k)});
          inst_row[k] = static_cast<int32_t>(row);
          total = std::max(total, row + need);
        }
      }
    }
    std::vector<int32_t> slots(refs.size());
    for (size_t k = 0; k < refs.size(); ++k) slots[k] = inst_row[refs[k].inst];
    if (total > lds_rows) return;
    size_t next_slot = 0;
    auto remap = [&](uint8_t& buf, int32_t* off, const int16_t* len) {
      for (int sgi = 0; sgi < 2; ++sgi) {
        if (len[sgi] <= 0) continue;
        if (buf == BUF_ARENA) {
          off[sgi] = slots[next_slot++];
        } else {
          off[sgi] = static_cast<int32_t>(off[sgi] - r0 + (buf == BUF_Y ? nrows : 0));
        }
      }
      buf = BUF_LDS;
    };
    for (int st = l.first; st < l.first + l.count; ++st) {
      const int32_t u0 = steps[kStepInts * st], u1 = steps[kStepInts * st + 1];
      const int32_t c0 = static_cast<int32_t>(punits->size());
      for (int32_t q = u0; q < u1; ++q) {
        Unit u = P.units[q];
        remap(u.in_buf, u.in_off, u.in_len);
        remap(u.out_buf, u.out_off, u.out_len);
        punits->push_back(u);
      }
      steps[kStepInts * st] = c0;
      steps[kStepInts * st + 1] = c0 + (u1 - u0);
    }
    l.lv_rows = static_cast<int32_t>(total);
    l.prow0 = static_cast<int32_t>(r0);
    l.prows = static_cast<int32_t>(nrows);
  }

  void bound(Launch& l, int32_t u0, int32_t u1) const {
    for (int32_t u = u0; u < u1; ++u) {
      const Unit& q = P.units[u];
      const int a = q.in_len[0] + q.in_len[1], b = q.out_len[0] + q.out_len[1];
      l.max_src = std::max({l.max_src, a, b});
      l.max_dst = std::max({l.max_dst, a, b});
      l.max_in = std::max(l.max_in, a);
      l.max_out = std::max(l.max_out, b);
      l.max_mat = std::max<int32_t>(l.max_mat, q.mat_len);
    }
  }
  // emit one ordered step (into a program when `prog` is non-null)
  void emit(int32_t u0, int32_t u1, int acc, int kind, Launch* prog, int force_fwd = 0) {
    if (prog) {
      int64_t m0 = INT64_MAX, m1 = 0;
      for (int32_t u = u0; u < u1; ++u) {
        m0 = std::min<int64_t>(m0, P.units[u].mat);
        m1 = std::max<int64_t>(m1, P.units[u].mat + P.units[u].mat_len);
      }
      if (m1 <= m0) m0 = m1 = 0;
      // flag 4: every unit is a dense 8-row slab read from one input segment
      // and written (not accumulated) to one output segment
      bool slab = acc == 0 && u1 > u0;
      for (int32_t u = u0; u < u1 && slab; ++u) {
        const Unit& q = P.units[u];
        slab = q.type == UNIT_DENSE && q.out_len[0] == 8 && q.out_len[1] == 0 && q.in_len[1] == 0 &&
               q.in_len[0] % 64 == 0 && q.in_len[0] > 0;
      }
      steps.push_back(u0);
      steps.push_back(u1);
      // flag 8: the slab widths grow with the unit index (claim them from the end)
      const bool rev = slab && P.units[u1 - 1].in_len[0] > P.units[u0].in_len[0];
      steps.push_back(acc | (force_fwd << 1) | (slab ? 4 : 0) | (rev ? 8 : 0));
      steps.push_back(static_cast<int32_t>(m0 / 16));
      steps.push_back(static_cast<int32_t>((m1 + 15) / 16 - m0 / 16));
      prog->count += 1;
      bound(*prog, u0, u1);
      return;
    }
    Launch l;
    l.direct = 1;
    l.first = u0;
    l.count = u1 - u0;
    l.max_src = l.max_dst = l.max_mat = 0;
    l.out_leaf = acc;
    l.kind = kind;
    l.prog = 0;
    l.force_fwd = force_fwd;
    bound(l, u0, u1);
    out.push_back(l);
  }
  void rec(int dd, int64_t idx, Launch* prog) {
    if (!prog && P.V - dd <= prog_levels) {
      Launch l;
      l.direct = 1;
      l.first = static_cast<int32_t>(steps.size() / kStepInts);
      l.count = 0;
      l.max_src = l.max_dst = l.max_mat = 0;
      l.out_leaf = 1;
      l.kind = 2;
      l.prog = 1;
      rec(dd, idx, &l);
      const int64_t rows = static_cast<int64_t>(P.n0) << (P.V - dd);
      make_lds(l, idx * rows, rows);
      out.push_back(l);
      return;
    }
    if (dd == P.V - P.sl) {
      // super-leaf solve: one unit per row slab, all independent; the
      // adjoint sweeps use the stored conjugate-transposed sets in forward mode
      emit(leaf_units[idx], leaf_units[idx] + P.sl_units, 0, 1, prog, adjoint ? 1 : 0);
      return;
    }
    const int64_t first = lower_dir ? 2 * idx : 2 * idx + 1;
    const int64_t second = lower_dir ? 2 * idx + 1 : 2 * idx;
    rec(dd + 1, first, prog);
    const bool use_lower = (lower_dir != adjoint);
    if (dd + 1 == P.V) {
      const int32_t u = use_lower ? P.l0_lower_unit[idx] : P.l0_upper_unit[idx];
      emit(u, u + 1, 1, 0, prog);
    } else {
      const BlockInfo& bi = P.blocks[level_base[dd + 1] + 2 * idx + (use_lower ? 1 : 0)];
      const int nl = 2 * bi.D + 1;
      for (int s = 0; s < nl; ++s) {
        const int l = adjoint ? nl - 1 - s : s;
        emit(bi.lvl_begin[l], bi.lvl_end[l], s == nl - 1 ? 1 : 0, 0, prog);
      }
    }
    rec(dd + 1, second, prog);
  }
};

}  // namespace

void build_sweeps(const Plan& P, Sweeps& S, int prog_levels, int lds_rows) {
  std::vector<int> level_base(P.V + 1, 0);
  {
    int cur = 0;
    for (int v = 1; v < P.V; ++v) {
      level_base[v] = cur;
      cur += 2 * (1 << (v - 1));
    }
  }
  S.fwd.clear();
  S.bwd.clear();
  S.adj_fwd.clear();
  S.adj_bwd.clear();
  S.steps.clear();
  S.punits.clear();
  S.prog_levels = prog_levels;
  if (P.sl_fwd.empty()) return;
  // P^{-1}: lower sweep with the L~ super-leaf inverses, upper with the U~ ones.
  // P^{-H}: lower sweep with (U~ inverse)^H, upper with (L~ inverse)^H.
  SweepGen g1{P, level_base, true, false, P.sl_fwd, S.fwd, S.steps, prog_levels};
  g1.punits = &S.punits;
  g1.lds_rows = lds_rows;
  g1.rec(0, 0, nullptr);
  SweepGen g2{P, level_base, false, false, P.sl_bwd, S.bwd, S.steps, prog_levels};
  g2.punits = &S.punits;
  g2.lds_rows = lds_rows;
  g2.rec(0, 0, nullptr);
  SweepGen g3{P, level_base, true, true, P.sl_adj_fwd, S.adj_fwd, S.steps, prog_levels};
  g3.punits = &S.punits;
  g3.lds_rows = lds_rows;
  g3.rec(0, 0, nullptr);
  SweepGen g4{P, level_base, false, true, P.sl_adj_bwd, S.adj_bwd, S.steps, prog_levels};
  g4.punits = &S.punits;
  g4.lds_rows = lds_rows;
  g4.rec(0, 0, nullptr);
  // the block reading's middle vector s = D t uses the diagonal leaf units
  const int64_t nl = P.n / P.n0;
  Launch d;
  d.direct = 1;
  d.first = P.diag_unit.empty() ? 0 : P.diag_unit[0];
  d.count = static_cast<int32_t>(nl);
  d.max_src = d.max_dst = d.max_in = d.max_out = P.n0;
  d.max_mat = P.n0 * P.n0;
  d.out_leaf = 0;
  d.kind = 0;
  d.prog = 0;
  d.force_fwd = 0;
  S.diag = {d};
}

// ---------------------------------------------------------------------------
// FP64 host executor of a schedule (the same unit semantics as the device
// stage kernel).
// ---------------------------------------------------------------------------
namespace {

struct Seg {
  cplx* base;
  int64_t off;
  int len;
};

void unit_eval(const Plan& P, const Unit& u, bool adj, const std::vector<cplx>& src, std::vector<cplx>& dst) {
  const cplx* M = P.fac.data() + u.mat;
  const uint8_t* pm = P.perm.data() + u.perm;
  const int nin = u.in_len[0] + u.in_len[1];
  const int nout = u.out_len[0] + u.out_len[1];
  if (u.type == UNIT_DENSE) {
    if (!adj) {
      for (int i = 0; i < nout; ++i) {
        cplx a = 0;
        for (int t = 0; t < nin; ++t) a += M[static_cast<size_t>(t) * nout + i] * src[t];
        dst[i] += a;
      }
    } else {
      for (int t = 0; t < nin; ++t) {
        cplx a = 0;
        for (int i = 0; i < nout; ++i) a += std::conj(M[static_cast<size_t>(t) * nout + i]) * src[i];
        dst[t] += a;
      }
    }
    return;
  }
  if (u.type == UNIT_GATHER) {
    // forward: src = in_cat (nin), dst = [out_a; out_b]
    int mo = 0, po = 0, base = 0;
    for (int o = 0; o < 2; ++o) {
      const int k = u.k[o];
      const int r = nin - k;
      const cplx* T = M + mo;
      const uint8_t* perm = pm + po;
      if (!adj) {
        for (int i = 0; i < k; ++i) {
          cplx a = src[perm[i]];
          for (int t = 0; t < r; ++t) a += T[static_cast<size_t>(t) * k + i] * src[perm[k + t]];
          dst[base + i] += a;
        }
      } else {
        // src = [out_a; out_b], dst = in_cat
        for (int i = 0; i < k; ++i) dst[perm[i]] += src[base + i];
        for (int t = 0; t < r; ++t) {
          cplx a = 0;
          for (int i = 0; i < k; ++i) a += std::conj(T[static_cast<size_t>(t) * k + i]) * src[base + i];
          dst[perm[k + t]] += a;
        }
      }
      mo += k * r;
      po += nin;
      base += k;
    }
    return;
  }
  // SCATTER: forward src = [in_a; in_b], dst = out_cat (nout)
  int mo = 0, po = 0, base = 0;
  for (int o = 0; o < 2; ++o) {
    const int k = u.k[o];
    const int r = nout - k;
    const cplx* T = M + mo;          // row-major k x r
    const uint8_t* inv = pm + po;    // invperm over nout
    if (!adj) {
      for (int p = 0; p < nout; ++p) {
        const int q = inv[p];
        cplx a;
        if (q < k) {
          a = src[base + q];
        } else {
          a = 0;
          for (int j = 0; j < k; ++j) a += T[static_cast<size_t>(j) * r + (q - k)] * src[base + j];
        }
        dst[p] += a;
      }
    } else {
      // src = out_cat, dst = [in_a; in_b]
      for (int p = 0; p < nout; ++p) {
        const int q = inv[p];
        if (q < k) {
          dst[base + q] += src[p];
        } else {
          for (int j = 0; j < k; ++j) dst[base + j] += std::conj(T[static_cast<size_t>(j) * r + (q - k)]) * src[p];
        }
      }
    }
    mo += k * r;
    po += nout;
    base += k;
  }
}

}  // namespace

int64_t schedule_bytes(const Plan& P, const std::vector<Launch>& launches, const std::vector<int32_t>* steps,
                       int elt, const std::vector<Unit>* punits) {
  int64_t total = 0;
  const std::vector<Unit>* table = &P.units;
  auto add = [&](int32_t uid) {
    const Unit& u = (*table)[uid];
    total += static_cast<int64_t>(u.mat_len) * elt + static_cast<int64_t>(sizeof(Unit));
    if (u.type == UNIT_GATHER) total += 2 * (u.in_len[0] + u.in_len[1]);
    if (u.type == UNIT_SCATTER) total += 2 * (u.out_len[0] + u.out_len[1]);
  };
  for (const Launch& L : launches) {
    table = (L.prog && L.lv_rows > 0 && punits) ? punits : &P.units;
    if (L.prog) {
      for (int st = L.first; st < L.first + L.count; ++st)
        for (int32_t q = (*steps)[kStepInts * st]; q < (*steps)[kStepInts * st + 1]; ++q) add(q);
    } else if (L.direct) {
      for (int32_t q = L.first; q < L.first + L.count; ++q) add(q);
    } else {
      for (int g = L.first; g < L.first + L.count; ++g)
        for (int32_t q = P.group_off[g]; q < P.group_off[g + 1]; ++q) add(P.group_units[q]);
    }
  }
  return total;
}

void exec_host(const Plan& P, const std::vector<Launch>& launches, bool adj_all, cplx* X, cplx* Y,
               cplx* arena, int R, cplx alpha, const std::vector<int32_t>* steps, const std::vector<Unit>* punits) {
  std::vector<cplx> src, dst, lds;
  // one ordered launch over `units`; BUF_LDS names the emulated LDS rows
  auto run = [&](const Launch& L, const Unit* units) {
    auto bufp = [&](uint8_t id) -> cplx* {
      return id == BUF_X ? X : id == BUF_Y ? Y : id == BUF_LDS ? lds.data() : arena;
    };
    const bool adj = adj_all && !L.force_fwd;
    for (int g = L.first; g < L.first + L.count; ++g) {
      std::vector<int32_t> us;
      if (L.direct) {
        us.push_back(g);
      } else {
        for (int32_t q = P.group_off[g]; q < P.group_off[g + 1]; ++q) us.push_back(P.group_units[q]);
      }
      // destination segments are those of the first unit (shared by the group)
      const Unit& u0 = units[us[0]];
      const uint8_t dbuf = adj ? u0.in_buf : u0.out_buf;
      const int32_t* doff = adj ? u0.in_off : u0.out_off;
      const int16_t* dlen = adj ? u0.in_len : u0.out_len;
      const int nd = dlen[0] + dlen[1];
      for (int r = 0; r < R; ++r) {
        dst.assign(nd, cplx(0.0));
        for (int32_t uid : us) {
          const Unit& u = units[uid];
          const uint8_t sbuf = adj ? u.out_buf : u.in_buf;
          const int32_t* soff = adj ? u.out_off : u.in_off;
          const int16_t* slen = adj ? u.out_len : u.in_len;
          const int ns = slen[0] + slen[1];
          src.resize(ns);
          cplx* sb = bufp(sbuf);
          for (int t = 0; t < slen[0]; ++t) src[t] = sb[(static_cast<int64_t>(soff[0]) + t) * R + r];
          for (int t = 0; t < slen[1]; ++t) src[slen[0] + t] = sb[(static_cast<int64_t>(soff[1]) + t) * R + r];
          unit_eval(P, u, adj, src, dst);
        }
        cplx* db = bufp(dbuf);
        int pos = 0;
        for (int s = 0; s < 2; ++s) {
          for (int t = 0; t < dlen[s]; ++t, ++pos) {
            cplx& o = db[(static_cast<int64_t>(doff[s]) + t) * R + r];
            o = L.out_leaf ? o + alpha * dst[pos] : dst[pos];
          }
        }
      }
    }
  };
  for (const Launch& L0 : launches) {
    if (!L0.prog) {
      run(L0, P.units.data());
      continue;
    }
    // a program is its steps, in order; with LDS-resident vectors its rows
    // of X and Y are copied in before the first step and out after the last
    const bool lv = L0.lv_rows > 0;
    if (lv && !punits) throw std::logic_error("exec_host: LDS-resident program without its unit copies");
    const int64_t r0 = L0.prow0, nr = L0.prows;
    if (lv) {
      lds.assign(static_cast<size_t>(L0.lv_rows) * R, cplx(std::nan(""), 0.0));
      std::copy(X + r0 * R, X + (r0 + nr) * R, lds.begin());
      std::copy(Y + r0 * R, Y + (r0 + nr) * R, lds.begin() + nr * R);
    }
    for (int st = L0.first; st < L0.first + L0.count; ++st) {
      Launch l = L0;
      l.prog = 0;
      l.direct = 1;
      l.first = (*steps)[kStepInts * st];
      l.count = (*steps)[kStepInts * st + 1] - (*steps)[kStepInts * st];
      l.out_leaf = (*steps)[kStepInts * st + 2] & 1;
      l.force_fwd = ((*steps)[kStepInts * st + 2] >> 1) & 1;
      run(l, lv ? punits->data() : P.units.data());
    }
    if (lv) {
      std::copy(lds.begin(), lds.begin() + nr * R, X + r0 * R);
      std::copy(lds.begin() + nr * R, lds.begin() + 2 * nr * R, Y + r0 * R);
    }
  }
}

// Leaf factorisation on the host in FP64 (construction checks only): writes
// the leaf-solve matrices into the leaf region of P.fac.
static void invert_dense(std::vector<cplx>& A, int n) {
  // Gauss-Jordan with partial pivoting on a row-major n x n matrix
  std::vector<cplx> I(static_cast<size_t>(n) * n, cplx(0.0));
  for (int i = 0; i < n; ++i) I[static_cast<size_t>(i) * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    double best = std::abs(A[static_cast<size_t>(c) * n + c]);
    for (int r = c + 1; r < n; ++r) {
      const double v = std::abs(A[static_cast<size_t>(r) * n + c]);
      if (v > best) { best = v; p = r; }
    }
    if (best == 0.0) throw std::runtime_error("singular leaf block");
    if (p != c) {
      for (int j = 0; j < n; ++j) {
        std::swap(A[static_cast<size_t>(p) * n + j], A[static_cast<size_t>(c) * n + j]);
        std::swap(I[static_cast<size_t>(p) * n + j], I[static_cast<size_t>(c) * n + j]);
      }
    }
    const cplx inv = 1.0 / A[static_cast<size_t>(c) * n + c];
    for (int j = 0; j < n; ++j) {
      A[static_cast<size_t>(c) * n + j] *= inv;
      I[static_cast<size_t>(c) * n + j] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const cplx f = A[static_cast<size_t>(r) * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        A[static_cast<size_t>(r) * n + j] -= f * A[static_cast<size_t>(c) * n + j];
        I[static_cast<size_t>(r) * n + j] -= f * I[static_cast<size_t>(c) * n + j];
      }
    }
  }
  A.swap(I);
}

// Fill the four super-leaf sets from the inverses Linv (of the lower block)
// and Uinv (of the upper block) of super-leaf S (both row-major ns x ns).
void store_superleaf(Plan& P, int64_t S, const std::vector<cplx>& Linv, const std::vector<cplx>& Uinv) {
  const int64_t ns = static_cast<int64_t>(P.n0) << P.sl;
  for (int set = 0; set < 4; ++set) {
    const std::vector<int32_t>& first = set == 0 ? P.sl_fwd : set == 1 ? P.sl_bwd : set == 2 ? P.sl_adj_fwd : P.sl_adj_bwd;
    for (int q = 0; q < P.sl_units; ++q) {
      const Unit& u = P.units[first[S] + q];
      const int r0 = u.out_off[0] - static_cast<int32_t>(S * ns);
      const int rows = u.out_len[0];
      const int c0 = u.in_off[0] - static_cast<int32_t>(S * ns);
      const int w = u.in_len[0];
      for (int c = 0; c < w; ++c)
        for (int r = 0; r < rows; ++r) {
          const int64_t gr = r0 + r, gc = c0 + c;
          cplx v;
          if (set == 0) v = Linv[gr * ns + gc];
          else if (set == 1) v = Uinv[gr * ns + gc];
          else if (set == 2) v = std::conj(Uinv[gc * ns + gr]);
          else v = std::conj(Linv[gc * ns + gr]);
          P.fac[u.mat + static_cast<int64_t>(c) * rows + r] = v;
        }
    }
  }
}

// The lower and upper super-leaf blocks of L~ / U~ (row-major ns x ns) from
// the exact entries A_SS (row-major): block reading D + A_low, D + A_up;
// point-wise reading I + a * strict_lower(A), upper(A).
void superleaf_blocks(const Plan& P, const std::vector<cplx>& A, hbf_prec prec, std::vector<cplx>& Lm,
                      std::vector<cplx>& Um) {
  const int64_t ns = static_cast<int64_t>(P.n0) << P.sl;
  Lm.assign(ns * ns, cplx(0.0));
  Um.assign(ns * ns, cplx(0.0));
  for (int64_t i = 0; i < ns; ++i)
    for (int64_t j = 0; j < ns; ++j) {
      const cplx a = A[i * ns + j];
      if (prec == HBF_PREC_BLOCK_LU) {
        const int64_t bi = i / P.n0, bj = j / P.n0;
        if (bi >= bj) Lm[i * ns + j] = a;
        if (bi <= bj) Um[i * ns + j] = a;
      } else {
        if (i > j) Lm[i * ns + j] = P.scale * a;
        if (i == j) Lm[i * ns + j] = 1.0;
        if (i <= j) Um[i * ns + j] = a;
      }
    }
}

void host_leaf_factor(Plan& P, hbf_prec prec) {
  if (P.sl_fwd.empty()) return;
  P.fac.resize(P.leaf_fac_begin + P.leaf_fac_len, cplx(0.0));
  const int64_t ns = static_cast<int64_t>(P.n0) << P.sl;
  const int64_t nsl = P.n / ns;
  std::vector<std::thread> th;
  std::atomic<int64_t> next(0);
  std::exception_ptr err = nullptr;
  std::mutex mu;
  const int T = std::max(1, std::min<int>(8, static_cast<int>(std::thread::hardware_concurrency())));
  for (int t = 0; t < T; ++t)
    th.emplace_back([&]() {
      try {
        for (;;) {
          const int64_t S = next.fetch_add(1);
          if (S >= nsl) return;
          std::vector<cplx> A(ns * ns), Lm, Um;
          for (int64_t i = 0; i < ns; ++i)
            for (int64_t j = 0; j < ns; ++j) A[i * ns + j] = P.entry(S * ns + i, S * ns + j);
          superleaf_blocks(P, A, prec, Lm, Um);
          invert_dense(Lm, static_cast<int>(ns));
          invert_dense(Um, static_cast<int>(ns));
          store_superleaf(P, S, Lm, Um);
        }
      } catch (...) {
        std::lock_guard<std::mutex> lk(mu);
        if (!err) err = std::current_exception();
      }
    });
  for (auto& x : th) x.join();
  if (err) std::rethrow_exception(err);
}

}  // namespace hbf

// ---------------------------------------------------------------------------
// host-only C ABI
// ---------------------------------------------------------------------------
using namespace hbf;

struct hbf_plan {
  Plan P;
  Sweeps S;
  hbf_prec prec = HBF_PREC_BLOCK_LU;
};

extern "C" {

const char* hbf_last_error(void) { return hbf::last_error(); }

void hbf_hankel2_0(const double* x, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    const cplx h = hankel2_0(x[i]);
    out[2 * i] = h.real();
    out[2 * i + 1] = h.imag();
  }
}

namespace {
// The batched entry interface served on the host (P.entry per element,
// threads over the jobs): lets the host check build take the same batched
// path as a device build, so the batching itself is checked without a GPU.
class HostBatchedEntries final : public hbf::EntryEval {
 public:
  explicit HostBatchedEntries(int threads) : threads_(threads) {}
  void prepare(const hbf::Plan& P) override { P_ = &P; }
  void eval(const std::vector<hbf::EntryJob>& jobs, const std::vector<hbf::IdJob>& ids) override {
    // jobs whose matrices feed an ID (with or without an output pointer)
    std::vector<int> id_of(jobs.size(), -1);
    for (size_t q = 0; q < ids.size(); ++q) id_of[static_cast<size_t>(ids[q].job)] = static_cast<int>(q);
    std::atomic<size_t> next(0);
    std::vector<std::thread> th;
    for (int t = 0; t < threads_; ++t)
      th.emplace_back([&]() {
        for (;;) {
          const size_t q = next.fetch_add(1);
          if (q >= jobs.size()) return;
          const hbf::EntryJob& J = jobs[q];
          std::vector<hbf::cplx> tmp;
          hbf::cplx* out = J.out;
          if (!out || id_of[q] >= 0) {
            tmp.resize(static_cast<size_t>(J.nrows) * J.ncols);
            out = tmp.data();
          }
          for (int c = 0; c < J.ncols; ++c)
            for (int a = 0; a < J.nrows; ++a)
              out[static_cast<size_t>(c) * J.nrows + a] =
                  J.swap ? P_->entry(J.cols[c], J.rows[a]) : P_->entry(J.rows[a], J.cols[c]);
          if (id_of[q] >= 0) {
            if (J.out) std::copy(tmp.begin(), tmp.end(), J.out);
            const hbf::IdJob& I = ids[static_cast<size_t>(id_of[q])];
            hbf::column_id_into(tmp, J.nrows, J.ncols, I.eps, I.kmax, I.k, I.perm, I.T);
          }
        }
      });
    for (auto& x : th) x.join();
  }

 private:
  int threads_;
  const hbf::Plan* P_ = nullptr;
};
}  // namespace

hbf_status hbf_plan_build(const hbf_curve* curve, double kappa, int32_t leaf, double tol,
                          const hbf_build_opts* opts, hbf_plan** out) {
  if (!out) { set_error("hbf_plan_build: out is NULL"); return HBF_EINVAL; }
  *out = nullptr;
  try {
    auto p = std::make_unique<hbf_plan>();
    if (opts && opts->host_entries == 2) {
      HostBatchedEntries ev(std::max(1, build_threads(opts)));
      build_plan(p->P, curve, kappa, leaf, tol, opts, &ev);
    } else {
      build_plan(p->P, curve, kappa, leaf, tol, opts);
    }
    p->prec = opts ? opts->prec : HBF_PREC_BLOCK_LU;
    host_leaf_factor(p->P, p->prec);
    // the device's default sweep schedule: programs over subtrees of 2^5
    // leaves, vectors LDS-resident where they fit the storage dtype's budget
    const int elt = (opts && opts->dtype == HBF_C128) ? 16 : 8;
    build_sweeps(p->P, p->S, 5, prog_lds_rows_budget(elt, elt));
    *out = p.release();
    return HBF_OK;
  } catch (const std::invalid_argument& e) {
    set_error(e.what());
    return HBF_EINVAL;
  } catch (const std::bad_alloc&) {
    set_error("hbf_plan_build: out of host memory");
    return HBF_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return HBF_ESINGULAR;
  }
}

hbf_status hbf_plan_apply(const hbf_plan* plan, const double* x, double* y, int32_t nrhs, int32_t adjoint) {
  if (!plan || !x || !y || nrhs < 1) { set_error("hbf_plan_apply: bad arguments"); return HBF_EINVAL; }
  const Plan& P = plan->P;
  const int64_t N = P.n, NE = P.n_real;
  // internal layout (N, R) in library order (ghost rows zero)
  std::vector<cplx> xi(N * nrhs), yi(N * nrhs), arena(P.arena_rows * nrhs);
  for (int r = 0; r < nrhs; ++r)
    for (int64_t i = 0; i < NE; ++i) xi[P.lib(i) * nrhs + r] = cplx(x[2 * (r * NE + i)], x[2 * (r * NE + i) + 1]);
  if (!adjoint) exec_host(P, P.mv_fwd, false, xi.data(), yi.data(), arena.data(), nrhs, 0.0);
  else exec_host(P, P.mv_adj, true, yi.data(), xi.data(), arena.data(), nrhs, 0.0);
  for (int r = 0; r < nrhs; ++r)
    for (int64_t i = 0; i < NE; ++i) {
      y[2 * (r * NE + i)] = yi[P.lib(i) * nrhs + r].real();
      y[2 * (r * NE + i) + 1] = yi[P.lib(i) * nrhs + r].imag();
    }
  return HBF_OK;
}

hbf_status hbf_plan_precond(const hbf_plan* plan, const double* rin, double* zout, int32_t nrhs, int32_t adjoint) {
  if (!plan || !rin || !zout || nrhs < 1) { set_error("hbf_plan_precond: bad arguments"); return HBF_EINVAL; }
  const Plan& P = plan->P;
  const Sweeps& S = plan->S;
  const int64_t N = P.n, NE = P.n_real;
  std::vector<cplx> u(N * nrhs), t(N * nrhs), z(N * nrhs), arena(P.arena_rows * nrhs);
  for (int r = 0; r < nrhs; ++r)
    for (int64_t i = 0; i < NE; ++i)
      u[P.lib(i) * nrhs + r] = cplx(rin[2 * (r * NE + i)], rin[2 * (r * NE + i) + 1]);
  if (plan->prec == HBF_PREC_NONE) {
    z = u;
  } else {
    const bool paper = plan->prec == HBF_PREC_PAPER_TRI;
    const cplx a = paper ? P.scale : cplx(1.0);
    if (!adjoint) {
      exec_host(P, S.fwd, false, t.data(), u.data(), arena.data(), nrhs, -a, &S.steps, &S.punits);
      if (!paper) exec_host(P, S.diag, false, t.data(), u.data(), arena.data(), nrhs, 0.0);  // u = D t
      cplx* mid = paper ? t.data() : u.data();
      exec_host(P, S.bwd, false, z.data(), mid, arena.data(), nrhs, -1.0, &S.steps, &S.punits);
    } else {
      exec_host(P, S.adj_fwd, true, u.data(), t.data(), arena.data(), nrhs, -1.0, &S.steps, &S.punits);
      if (!paper) exec_host(P, S.diag, true, u.data(), t.data(), arena.data(), nrhs, 0.0);  // u = D^H t
      cplx* mid = paper ? t.data() : u.data();
      exec_host(P, S.adj_bwd, true, mid, z.data(), arena.data(), nrhs, -std::conj(a), &S.steps, &S.punits);
    }
  }
  for (int r = 0; r < nrhs; ++r)
    for (int64_t i = 0; i < NE; ++i) {
      zout[2 * (r * NE + i)] = z[P.lib(i) * nrhs + r].real();
      zout[2 * (r * NE + i) + 1] = z[P.lib(i) * nrhs + r].imag();
    }
  return HBF_OK;
}

hbf_status hbf_plan_entries(const hbf_plan* plan, const int64_t* rows, int64_t nr, const int64_t* cols,
                            int64_t nc, double* out) {
  if (!plan || !rows || !cols || !out) { set_error("hbf_plan_entries: bad arguments"); return HBF_EINVAL; }
  for (int64_t a = 0; a < nr; ++a)
    for (int64_t b = 0; b < nc; ++b) {
      if (rows[a] < 0 || rows[a] >= plan->P.n_real || cols[b] < 0 || cols[b] >= plan->P.n_real) {
        set_error("hbf_plan_entries: index out of range");
        return HBF_EINVAL;
      }
      const cplx e = plan->P.entry(plan->P.lib(rows[a]), plan->P.lib(cols[b]));
      out[2 * (a * nc + b)] = e.real();
      out[2 * (a * nc + b) + 1] = e.imag();
    }
  return HBF_OK;
}

void fill_stats(const Plan& P, hbf_stats_t* s, int elt) {
  std::memset(s, 0, sizeof(*s));
  s->n = P.n_real;
  s->n_internal = P.n;
  s->leaf = P.n0;
  s->levels = P.V;
  s->n_blocks = static_cast<int64_t>(P.blocks.size());
  s->n_units = static_cast<int64_t>(P.units.size());
  s->max_rank = P.max_rank;
  s->mean_rank = P.n_ids ? P.sum_rank / P.n_ids : 0.0;
  s->bytes_butterfly = P.bytes_butterfly_c128 / 16 * elt;
  s->bytes_dense = P.bytes_dense_c128 / 16 * elt;
  s->bytes_precond = P.leaf_fac_len * elt;
  s->build_seconds = P.build_seconds;
  s->scale_re = P.scale.real();
  s->scale_im = P.scale.imag();
  s->arena_rows = P.arena_rows;
}

hbf_status hbf_plan_stats(const hbf_plan* plan, hbf_stats_t* out) {
  if (!plan || !out) { set_error("hbf_plan_stats: bad arguments"); return HBF_EINVAL; }
  fill_stats(plan->P, out, 16);
  out->bytes_index = static_cast<int64_t>(plan->P.perm.size());
  return HBF_OK;
}

void hbf_plan_free(hbf_plan* plan) { delete plan; }

}  // extern "C"
