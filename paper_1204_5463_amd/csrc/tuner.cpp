// Autotuner: coordinate search over SAP block shape, MR steps, SAP cycles
// and (m, k), scored by the wall-clock time of the whole solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <vector>

#include "dw_internal.hpp"

using namespace dw;

namespace {

struct Tuner {
  dw_ctx ctx;
  int L[4];
  const double* U;
  double m0;
  double csw;
  const double* b;
  double* x;
  int nrhs;
  hipStream_t st;
  const dw_tune_space* sp;
  dw_tune_trial* trials;
  int max_trials;
  int n = 0;
  bool have_best = false;
  dw_tune_trial best{};
  // field cached for the current block shape
  dw_field f = nullptr;
  int fblock[4] = {0, 0, 0, 0};

  ~Tuner() {
    if (f) dw_field_destroy(f);
  }

  dw_status field_for(const int B[4]) {
    if (f && std::equal(B, B + 4, fblock)) return DW_OK;
    if (f) {
      (void)hipStreamSynchronize(st);
      dw_field_destroy(f);
      f = nullptr;
    }
    DW_TRY(dw_field_create(ctx, L, B, U, st, &f));
    if (csw != 0.0) DW_TRY(dw_field_set_clover(f, csw, st));
    std::copy(B, B + 4, fblock);
    return DW_OK;
  }

  // Runs one candidate (unless already tried); updates best.
  dw_status run(fgmresdr_params p) {
    for (int i = 0; i < n; ++i) {
      const fgmresdr_params& q = trials[i].params;
      if (q.m == p.m && q.k == p.k && q.sap.ncycles == p.sap.ncycles && q.sap.nmr == p.sap.nmr &&
          std::equal(q.sap.block, q.sap.block + 4, p.sap.block))
        return DW_OK;
    }
    if (n >= max_trials) return DW_OK;
    if (have_best && sp->iter_cap > 0) {
      const double cap = std::ceil(sp->iter_cap * best.iterations);
      p.max_iter = (int)std::min<double>(p.max_iter, std::max(cap, (double)p.m));
    }
    DW_TRY(field_for(p.sap.block));
    std::vector<dw_solve_stats> stats(nrhs);
    dw_tune_trial t{};
    t.params = p;
    t.seconds = INFINITY;
    t.converged = 1;
    for (int rep = 0; rep < std::max(1, sp->repeats); ++rep) {
      DW_CHECK_HIP(hipStreamSynchronize(st));
      const auto t0 = std::chrono::steady_clock::now();
      const dw_status s = fgmresdr_solve(f, m0, &p, b, x, nrhs, stats.data(), st);
      DW_CHECK_HIP(hipStreamSynchronize(st));
      const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (s != DW_OK && s != DW_ENOTCONV) return s;
      int it = 0;
      bool conv = true;
      for (const auto& q : stats) {
        it = std::max(it, (int)q.iterations);
        conv = conv && q.converged;
      }
      t.iterations = it;
      if (!conv) {
        t.converged = 0;
        break;  // no point timing a candidate that misses the tolerance again
      }
      t.seconds = std::min(t.seconds, sec);
    }
    trials[n++] = t;
    if (t.converged && (!have_best || t.seconds < best.seconds)) {
      best = t;
      have_best = true;
    }
    return DW_OK;
  }

  // best parameters with the caller's iteration limit
  fgmresdr_params current(const fgmresdr_params& base) const {
    fgmresdr_params p = have_best ? best.params : base;
    p.max_iter = base.max_iter;
    return p;
  }
};

bool valid_block(const int L[4], const int B[4]) {
  Geom g;
  return make_geom(L, B, &g) == nullptr;
}

std::vector<std::array<int, 4>> default_blocks(const int L[4]) {
  std::vector<std::array<int, 4>> out;
  const int ext[3] = {2, 4, 8};
  for (int a : ext)
    for (int b : ext)
      for (int c : ext)
        for (int d : ext) {
          const int B[4] = {a, b, c, d};
          const int vol = a * b * c * d;
          const int lo = std::min({a, b, c, d}), hi = std::max({a, b, c, d});
          if (vol < 128 || vol > 512 || hi > 2 * lo || !valid_block(L, B)) continue;
          out.push_back({a, b, c, d});
        }
  return out;
}

}  // namespace

extern "C" dw_status dw_autotune(dw_ctx ctx, const int32_t L[4], const double* U, double m0, double csw,
                                 const fgmresdr_params* base, const dw_tune_space* space, const double* b, double* x,
                                 int32_t nrhs, dw_tune_trial* trials, int32_t max_trials, int32_t* ntrials,
                                 fgmresdr_params* best, hipStream_t stream) {
  clear_error();
  if (!ctx || !L || !U || !base || !space || !b || !x || nrhs < 1 || !trials || max_trials < 1 || !ntrials ||
      !best || b == x || space->nblocks < 0 || space->nblocks > 16 || space->nmk < 0 || space->nmk > 8) {
    set_error("dw_autotune: invalid argument");
    return DW_EINVAL;
  }
  for (int i = 0; i < space->nmk; ++i) {
    const int m = space->mk[i][0], k = space->mk[i][1];
    if (m < 1 || m > 48 || k < 0 || k >= m || k > 23) {
      set_error("dw_autotune: candidate (m, k) = (%d, %d) is invalid", m, k);
      return DW_EINVAL;
    }
  }
  *ntrials = 0;
  const int Li[4] = {L[0], L[1], L[2], L[3]};
  if (!valid_block(Li, base->sap.block)) {
    set_error("dw_autotune: the base block shape is not valid for the lattice");
    return DW_EINVAL;
  }
  if (!std::isfinite(csw)) {
    set_error("dw_autotune: non-finite csw");
    return DW_EINVAL;
  }
  Tuner T{ctx, {Li[0], Li[1], Li[2], Li[3]}, U, m0, csw, b, x, nrhs, stream, space, trials, max_trials};
  dw_status s = DW_OK;
  auto step = [&](fgmresdr_params p) {
    if (s == DW_OK) s = T.run(p);
  };
  step(*base);
  // block shape
  std::vector<std::array<int, 4>> blocks;
  if (space->nblocks > 0) {
    for (int i = 0; i < space->nblocks; ++i) {
      const int* B = space->blocks[i];
      if (!valid_block(Li, B)) {
        set_error("dw_autotune: candidate block %d %d %d %d is not valid for the lattice", B[0], B[1], B[2], B[3]);
        return DW_EINVAL;
      }
      blocks.push_back({B[0], B[1], B[2], B[3]});
    }
  } else {
    blocks = default_blocks(Li);
  }
  for (const auto& B : blocks) {
    fgmresdr_params p = T.current(*base);
    std::copy(B.begin(), B.end(), p.sap.block);
    step(p);
  }
  // MR steps, SAP cycles, (m, k); they interact, so the sweep is repeated
  for (int pass = 0; pass < std::max(1, space->passes); ++pass) {
    for (int nmr = space->nmr_min; nmr <= space->nmr_max && nmr >= 0; ++nmr) {
      fgmresdr_params p = T.current(*base);
      p.sap.nmr = nmr;
      step(p);
    }
    for (int c = space->s_min; c <= space->s_max && c >= 1; ++c) {
      fgmresdr_params p = T.current(*base);
      p.sap.ncycles = c;
      step(p);
    }
    for (int i = 0; i < space->nmk; ++i) {
      fgmresdr_params p = T.current(*base);
      p.m = space->mk[i][0];
      p.k = space->mk[i][1];
      step(p);
    }
  }
  *ntrials = T.n;
  if (s != DW_OK) return s;
  if (!T.have_best) {
    set_error("dw_autotune: no candidate reached the tolerance");
    return DW_ENOTCONV;
  }
  *best = T.current(*base);
  return DW_OK;
}
