// Sweep schedules and the host executor (shared by the host checks and the
// device context, which uploads the same launch lists).
#pragma once

#include <vector>

#include "hbf_internal.h"

namespace hbf {

struct Sweeps {
  std::vector<Launch> fwd, bwd;          // P^{-1}: lower then upper substitution
  std::vector<Launch> adj_fwd, adj_bwd;  // P^{-H}
  std::vector<Launch> diag;              // s = D t (block reading, between the sweeps)
  std::vector<int32_t> steps;            // program steps, kStepInts entries each
  std::vector<Unit> punits;              // unit copies of the LDS-resident programs (Launch::lv_rows)
  int prog_levels = 5;                   // subtrees of <= 2^prog_levels leaves run as one program
};

// lds_rows: largest LDS vector footprint (rows) a program may keep in LDS
// (0: every program works on the vectors in global memory).
void build_sweeps(const Plan& P, Sweeps& S, int prog_levels = 5, int lds_rows = 0);

// Run a schedule on host buffers in the internal (rows, R) layout.  In
// adjoint mode every unit reads its forward output segments and writes its
// forward input segments.  Launches with out_leaf set add alpha * result to
// the destination; the others overwrite it.
void exec_host(const Plan& P, const std::vector<Launch>& launches, bool adj, cplx* X, cplx* Y,
               cplx* arena, int R, cplx alpha, const std::vector<int32_t>* steps = nullptr,
               const std::vector<Unit>* punits = nullptr);

// Bytes a schedule streams once per application: matrices (elt bytes per
// entry), permutations and descriptors of every unit it runs.
int64_t schedule_bytes(const Plan& P, const std::vector<Launch>& launches, const std::vector<int32_t>* steps, int elt,
                       const std::vector<Unit>* punits = nullptr);

void host_leaf_factor(Plan& P, hbf_prec prec);
void superleaf_blocks(const Plan& P, const std::vector<cplx>& A, hbf_prec prec, std::vector<cplx>& Lm,
                      std::vector<cplx>& Um);

const char* last_error();

}  // namespace hbf

extern "C" void fill_stats(const hbf::Plan& P, hbf_stats_t* s, int elt);
