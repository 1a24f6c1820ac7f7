// Krylov solvers for the fermion-matrix inversion (the operation the paper's
// introduction identifies with the bulk of the floating-point work).
//
//  * CG (Hestenes-Stiefel) on A = Mhat^dag Mhat for the HMC force, x0 = 0,
//    stop at the first k with |r_k| <= tol |b|.
//  * CGLS on Mhat x_e = bhat_e for Wilson solves M x = b, through the
//    Schur complement bhat_e = b_e + kappa D_eo b_o, x_o = b_o + kappa D_oe x_e.
//  * Mixed precision: the same iteration on FP32 / FP16 / BF16 storage with
//    FP32 arithmetic and FP64 global sums; whenever the inner residual has
//    fallen by reliable_delta since the last update, the inner solution is
//    folded into the FP64 solution and the residual replaced by the FP64
//    true residual (reliable updates, Clark et al., Comput. Phys. Commun.
//    181 (2010) 1517); the search direction is kept.
//
// An iteration is six launches on one stream (four Dslash, two vector
// kernels) with alpha, beta and the stop test computed on the device.  The
// host enqueues chunks of iterations and reads the 32-byte solver state once
// per chunk; iterations enqueued after the stop exit at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>

#include "fields.h"
#include "solver.h"

namespace hmc {

namespace {
constexpr int kChunk = 16;
constexpr int kMaxReliable = 2000;  // a solve that needs more has stagnated
}  // namespace

void build_iteration(const SolveVecs& v, int iter0, double thr, int mixed, double delta2, IterArgs* o) {
  const double k2 = v.kappa * v.kappa;
  DslashArgs b{};
  b.U = v.Ulow;
  b.su3 = v.su3;
  b.shape = v.shape;
  b.stop_at = &v.state->stop_at;
  b.iter0 = iter0;
  b.a = 1.0;
  b.b = 1.0;
  for (int i = 0; i < 4; ++i) o->d[i] = b;
  if (!v.cgls) {
    // t = D_oe p;  s = p - k^2 D_eo t (|s|^2 = <p, A p>);
    // t = D^dag_oe s (block 0: alpha = |r|^2 / |s|^2);
    // r -= alpha (s - k^2 D^dag_eo t) (|r|^2);  then x += alpha p, p = r + beta p
    o->d[0].in = v.p, o->d[0].out = v.t;
    o->d[1].in = v.t, o->d[1].out = v.s, o->d[1].y = v.p, o->d[1].b = -k2, o->d[1].partial = v.pq;
    o->d[2].in = v.s, o->d[2].out = v.t;
    o->d[2].alpha_pp[0] = v.pp[0], o->d[2].alpha_pp[1] = v.pp[1], o->d[2].alpha_den = v.pq;
    o->d[2].alpha_n_pp = v.nbD, o->d[2].alpha_n_den = v.nbD;
    o->d[2].alpha_out = &v.state->alpha;
    o->d[3].in = v.t, o->d[3].out = v.r, o->d[3].y = v.s, o->d[3].b = -k2;
    o->d[3].r = v.r, o->d[3].alpha_in = &v.state->alpha;
    o->d[3].partial_pp[0] = v.pp[0], o->d[3].partial_pp[1] = v.pp[1];
  } else {
    // t = D_oe p;  q = p - k^2 D_eo t (|q|^2);  [update];  t = D^dag_oe r;  s = r - k^2 D^dag_eo t (|s|^2)
    o->d[0].in = v.p, o->d[0].out = v.t;
    o->d[1].in = v.t, o->d[1].out = v.q, o->d[1].y = v.p, o->d[1].b = -k2, o->d[1].partial = v.pq;
    o->d[2].in = v.r, o->d[2].out = v.t;
    o->d[3].in = v.t, o->d[3].out = v.s, o->d[3].y = v.r, o->d[3].b = -k2;
    o->d[3].partial_pp[0] = v.pp[0];
    o->d[3].partial_pp[1] = v.pp[1];
  }
  CgArgs c{};
  c.x = v.xl;
  c.p = v.p;
  c.r = v.r;
  c.q = v.q;
  c.s = v.s;
  c.pp[0] = v.pp[0];
  c.pp[1] = v.pp[1];
  c.pq = v.pq;
  c.pr = v.pr;
  c.n_pp = v.nbD;  // |r|^2 (CG) or |s|^2 (CGLS), both from a Dslash epilogue
  c.n_pq = v.nbD;
  c.n_pr = v.nbR;
  c.state = v.state;
  c.iter0 = iter0;
  c.cgls = v.cgls;
  c.thr = thr;
  c.delta2 = delta2;
  c.mixed = mixed;
  c.fused = v.cgls ? 0 : 1;
  o->c[0] = c;
  o->c[1] = c;
}

hipError_t launch_iteration(const LatArg& g, hmc_prec prec, int cgls, const IterTables* tab, const IterArgs& one,
                            int nbatch, int nbD, int nbR, int j, hipStream_t st) {
  (void)nbD;
  hipError_t e;
  auto D = [&](int i, int out_par, int dag, int epi) {
    return launch_dslash(prec, dag, epi, g, out_par, tab ? tab->d[i] : nullptr, nbatch, one.d[i], st, j);
  };
  auto UPD = [&](int i) { return launch_cg_update(g, prec, one.c[i], nbR, tab ? tab->c[i] : nullptr, nbatch, j, st); };
  auto PUP = [&](int i) { return launch_cg_pupdate(g, prec, one.c[i], nbR, tab ? tab->c[i] : nullptr, nbatch, j, st); };
  if (!cgls) {
    // the four hops are consecutive: one timing sample brackets them all
    timing_group_begin(TK_DSLASH, 4);
    if (!(e = D(0, 1, 0, EPI_PLAIN)) && !(e = D(1, 0, 0, EPI_AXPY_NORM)) && !(e = D(2, 1, 1, EPI_PLAIN)))
      e = D(3, 0, 1, EPI_CG);
    timing_group_end();
    if (e) return e;
    return PUP(1);
  }
  if ((e = D(0, 1, 0, EPI_PLAIN))) return e;
  if ((e = D(1, 0, 0, EPI_AXPY_NORM))) return e;
  if ((e = UPD(0))) return e;
  if ((e = D(2, 1, 1, EPI_PLAIN))) return e;
  if ((e = D(3, 0, 1, EPI_AXPY_NORM))) return e;
  return PUP(1);
}

static hipError_t ds64(const SolveVecs& v, void* out, const void* in, int out_par, int dag, int epi, const void* y,
                       double a, double b, double* partial, hipStream_t st) {
  DslashArgs d{};
  d.U = v.U64;
  d.su3 = v.su3;
  d.shape = v.shape64;
  d.in = in;
  d.out = out;
  d.y = y;
  d.a = a;
  d.b = b;
  d.partial = partial;
  return launch_dslash(HMC_F64, dag, epi, v.g, out_par, nullptr, 1, d, st, 0);
}

hipError_t mhat64(const SolveVecs& v, void* out, const void* in, int dag, double* partial, hipStream_t st) {
  hipError_t e = ds64(v, v.t64, in, 1, dag, EPI_PLAIN, nullptr, 0.0, 1.0, nullptr, st);
  if (e != hipSuccess) return e;
  return ds64(v, out, v.t64, 0, dag, partial ? EPI_AXPY_NORM : EPI_AXPY, in, 1.0, -v.kappa * v.kappa, partial, st);
}

hipError_t true_residual(const SolveVecs& v, hipStream_t st) {
  hipError_t e;
  if (v.cgls) {
    if ((e = mhat64(v, v.q64, v.x, 0, nullptr, st))) return e;
  } else {
    if ((e = mhat64(v, v.s64, v.x, 0, nullptr, st))) return e;
    if ((e = mhat64(v, v.q64, v.s64, 1, nullptr, st))) return e;
  }
  if ((e = launch_xmy_norm(v.g, v.rhs, v.q64, v.r64, v.red, v.nbR, st))) return e;
  return launch_finalize(v.red, v.nbR, 1, v.slot, 1.0, 0, st);
}

hipError_t reliable_update(const SolveVecs& v, hipStream_t st) {
  hipError_t e = launch_add_low_to_f64(v.g, v.x, v.xl, st);
  if (e != hipSuccess) return e;
  return true_residual(v, st);
}

hipError_t inner_restart(const SolveVecs& v, int k, bool first, hipStream_t st) {
  hipError_t e;
  const size_t lowbytes = (size_t)v.g.Vh * (v.prec == HMC_F32 ? 96 : v.prec == HMC_F16 ? 52 : 48);
  if ((e = launch_convert_spinor(v.g, v.r64, HMC_F64, v.r, v.prec, 1, nullptr, nullptr, st))) return e;
  double* part = v.pp[k & 1];
  if (v.cgls) {
    DslashArgs d{};
    d.U = v.Ulow;
    d.su3 = v.su3;
    d.shape = v.shape;
    d.in = v.r;
    d.out = v.t;
    d.a = 1.0;
    d.b = 1.0;
    if ((e = launch_dslash(v.prec, 1, EPI_PLAIN, v.g, 1, nullptr, 1, d, st, 0))) return e;
    d.in = v.t;
    d.out = v.s;
    d.y = v.r;
    d.b = -v.kappa * v.kappa;
    d.partial = part;
    if ((e = launch_dslash(v.prec, 1, EPI_AXPY_NORM, v.g, 0, nullptr, 1, d, st, 0))) return e;
    if (first && (e = launch_copy(v.p, v.s, lowbytes, st))) return e;
  } else {
    if ((e = launch_norm2_partials(v.g, v.prec, v.r, part, v.nbD, st))) return e;
    if (first && (e = launch_copy(v.p, v.r, lowbytes, st))) return e;
  }
  if (first && (e = launch_zero(v.xl, (size_t)v.g.Vh * 96, st))) return e;
  return launch_state_reset(v.state, v.slot, 1, first ? 1 : 0, st);
}

namespace {

hipError_t read_state(Fields* F, SolverState* out, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(F->pinned + SL_COUNT, F->state, sizeof(SolverState), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  std::memcpy(out, F->pinned + SL_COUNT, sizeof(SolverState));
  return hipSuccess;
}

// A chunk of enqueued iterations whose solver state is being copied back
// into pinned slot `slot` (completion marked by F->state_ev[slot]).
struct Chunk {
  int k, n, slot;
};

hipError_t enqueue_chunk(Fields* F, const SolveVecs& v, const IterArgs& args, const Chunk& c, hipStream_t st) {
  for (int j = 0; j < c.n; ++j) {
    hipError_t e = launch_iteration(v.g, v.prec, v.cgls, nullptr, args, 1, v.nbD, v.nbR, c.k + j, st);
    if (e != hipSuccess) return e;
  }
  static_assert(sizeof(SolverState) <= 8 * sizeof(double), "state slot");
  hipError_t e = hipMemcpyAsync(F->pinned + SL_COUNT + 8 * c.slot, F->state, sizeof(SolverState),
                                hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipEventRecord(F->state_ev[c.slot], st);
}

hipError_t wait_chunk(Fields* F, const Chunk& c, SolverState* out) {
  hipError_t e = hipEventSynchronize(F->state_ev[c.slot]);
  if (e != hipSuccess) return e;
  std::memcpy(out, F->pinned + SL_COUNT + 8 * c.slot, sizeof(SolverState));
  return hipSuccess;
}

// Runs iterations with labels *k.. until the device stops or `limit` is
// reached; leaves the next label in *k.  The chunk length follows the
// observed convergence rate toward `target` (|r|^2 at which the device will
// stop), so few iterations are enqueued past the stop; while the host waits
// for one chunk's state, the next chunk is already queued whenever the
// prediction says the stop lies beyond the first, so the GPU does not idle
// during the read-back.  *rate carries log(|r|^2) per iteration between
// calls (0 = unknown).  Iterations enqueued past the stop exit at once.
hipError_t run_until_stop(Fields* F, const SolveVecs& v, const IterArgs& args, int* k, int limit, SolverState* stt,
                          hipStream_t st, double rr_start, double target, double* rate) {
  const bool fixed = !(target > 0);
  // iterations still needed from residual rr (kChunk when unknown)
  auto predict = [&](double rr) -> double {
    if (fixed) return limit;
    if (*rate < 0 && rr > 0) return std::log(target / rr) / *rate;
    return kChunk;
  };
  double rr_now = rr_start;
  int next = *k;
  if (next >= limit) return hipSuccess;
  Chunk cur{next, std::min({kChunk, limit - next, std::max(1, (int)std::ceil(predict(rr_now)))}), 0};
  hipError_t e = enqueue_chunk(F, v, args, cur, st);
  if (e != hipSuccess) return e;
  next += cur.n;
  while (true) {
    // queue the following chunk before waiting when the stop is predicted past this one
    Chunk nxt{next, 0, cur.slot ^ 1};
    const double after = predict(rr_now) - cur.n;
    if (next < limit && (fixed ? after >= 1.0 : after >= 2.0)) {
      // CG often speeds up near the end: queue 80% of the predicted rest
      nxt.n = std::min({kChunk, limit - next, fixed ? (int)after : std::max(1, (int)(0.8 * after))});
      if ((e = enqueue_chunk(F, v, args, nxt, st))) return e;
      next += nxt.n;
    }
    if ((e = wait_chunk(F, cur, stt))) return e;
    if (stt->stop_at != INT_MAX) {
      *k = stt->last + 1;
      return hipSuccess;  // a queued chunk after the stop exits at once
    }
    if (stt->rr > 0 && rr_now > 0 && stt->rr < rr_now) *rate = std::log(stt->rr / rr_now) / cur.n;
    rr_now = stt->rr;
    if (nxt.n > 0) {
      cur = nxt;
      continue;
    }
    if (next >= limit) {
      *k = next;
      return hipSuccess;
    }
    cur = Chunk{next, std::min({kChunk, limit - next, std::max(1, (int)std::ceil(predict(rr_now)))}), cur.slot ^ 1};
    if ((e = enqueue_chunk(F, v, args, cur, st))) return e;
    next += cur.n;
  }
}

}  // namespace

#define CHK(expr) HMC_CHECK_HIP(expr)

hmc_status cg_solve_impl(Fields* F, void* x, const void* b, const hmc_cg_params* prm, hmc_cg_stats* stats,
                         hipStream_t st) {
  HMC_REQUIRE(prm->mode == HMC_CG_NORMAL_MHAT || prm->mode == HMC_CG_WILSON_SOLVE, "bad solver mode %d", prm->mode);
  HMC_REQUIRE(prm->prec >= HMC_F64 && prm->prec <= HMC_BF16, "bad solver precision %d", prm->prec);
  HMC_REQUIRE(prm->maxiter >= 1 || prm->fixed_iters > 0, "maxiter must be >= 1");
  HMC_REQUIRE(prm->fixed_iters == 0 || prm->prec == HMC_F64, "fixed_iters needs prec = HMC_F64");
  const hmc_prec prec = (hmc_prec)prm->prec;
  HMC_REQUIRE(prec == HMC_F64 || (F->flags & HMC_FIELDS_LOWPREC), "mixed precision needs HMC_FIELDS_LOWPREC");
  HMC_REQUIRE(x != b, "x and b must not alias");
  auto t0 = std::chrono::steady_clock::now();
  const int cgls = prm->mode == HMC_CG_WILSON_SOLVE;
  const int fixed = prm->fixed_iters;
  const int limit = fixed > 0 ? fixed : prm->maxiter;
  const double delta = prm->reliable_delta > 0 ? prm->reliable_delta : 0.1;
  if (prec != HMC_F64) CHK(ensure_lowprec(F, prec, st));

  SolveVecs v{};
  v.g = F->g;
  v.kappa = F->kappa;
  v.cgls = cgls;
  v.prec = prec;
  v.U64 = F->U;
  v.Ulow = low_links(F, prec);
  v.su3 = F->su3;
  v.x = x;
  v.r64 = F->r;
  v.rhs = cgls ? F->bhat : const_cast<void*>(b);
  v.q64 = F->q;
  v.s64 = F->s;
  v.t64 = F->t;
  if (prec == HMC_F64) {
    v.r = F->r, v.p = F->p, v.q = F->q, v.s = F->s, v.t = F->t, v.xl = x;
  } else {
    v.r = F->lr, v.p = F->lp, v.q = F->lq, v.s = F->ls, v.t = F->lt, v.xl = F->lx;
  }
  v.pp[0] = F->part[0];
  v.pp[1] = F->part[1];
  v.pq = F->part[2];
  v.pr = F->part[3];
  v.red = F->part[4];
  v.slot = F->slots + SL_SOLVER;
  v.state = F->state;
  // shapes fixed for the whole solve (the partial counts follow from them)
  v.shape = dslash_shape(F->g, prec);
  v.shape64 = dslash_shape(F->g, HMC_F64);
  v.nbD = dslash_shape_blocks(F->g.Vh, v.shape);
  v.nbR = F->nbR;
  hmc_cg_stats S{};

  // ---- set-up in FP64: |b|^2, the even right-hand side, x = x0 (0 unless
  // initial_guess), r = rhs - A x0
  const char* bb = (const char*)b;
  const bool guess = !cgls && prm->initial_guess;
  double bnorm2 = 0, rr0 = 0;
  if (cgls) {
    CHK(launch_norm2_partials(F->g, HMC_F64, bb, v.red, F->nbR, st));
    CHK(launch_norm2_partials(F->g, HMC_F64, bb + F->half64, v.red + F->nbR, F->nbR, st));
    CHK(launch_finalize(v.red, 2 * F->nbR, 1, v.slot, 1.0, 0, st));
    CHK(read_slots(F, SL_SOLVER, 1, &bnorm2, st));
    // bhat_e = b_e + kappa D_eo b_o
    CHK(dslash_f64(F, F->bhat, bb + F->half64, 0, 0, EPI_AXPY, bb, 1.0, F->kappa, nullptr, nullptr, 0, st));
  }
  if (guess) {
    CHK(launch_norm2_partials(F->g, HMC_F64, bb, v.red, F->nbR, st));
    CHK(launch_finalize(v.red, F->nbR, 1, v.slot, 1.0, 0, st));
    CHK(read_slots(F, SL_SOLVER, 1, &bnorm2, st));
    // r = b - Mhat^dag Mhat x0, |r|^2 partials in pp[0]; p = r (F64)
    CHK(mhat64(v, v.s64, x, 0, nullptr, st));
    CHK(mhat64(v, v.q64, v.s64, 1, nullptr, st));
    CHK(launch_xmy_norm(F->g, v.rhs, v.q64, v.r64, v.pp[0], v.nbD, st));
    if (prec == HMC_F64) CHK(launch_copy(v.p, v.r64, F->half64, st));
  } else {
    // |r|^2 partials in pp[0] with the Dslash-epilogue count, as the iteration reads them
    CHK(launch_cg_init(F->g, HMC_F64, v.rhs, x, v.r64, prec == HMC_F64 ? v.p : v.q64, v.pp[0], v.nbD, st));
  }
  CHK(launch_finalize(v.pp[0], v.nbD, 1, v.slot, 1.0, 0, st));
  CHK(read_slots(F, SL_SOLVER, 1, &rr0, st));
  if (!cgls && !guess) bnorm2 = rr0;
  const double thr = fixed > 0 ? -1.0 : prm->tol * prm->tol * bnorm2;

  int k = 0;
  SolverState stt{};
  stt.rr = rr0;
  hmc_status status = HMC_OK;
  if (!std::isfinite(bnorm2) || !std::isfinite(rr0)) {
    status = HMC_E_NAN;  // a non-finite right-hand side or operator: no iteration can help
  } else if (bnorm2 == 0.0 || (fixed == 0 && rr0 <= thr)) {
    // x = 0 already meets the tolerance
  } else if (prec == HMC_F64) {
    if (cgls) {
      CHK(mhat64(v, v.s, v.r, 1, v.pp[0], st));  // s = Mhat^dag r, |s|^2 into pp[0]
      CHK(launch_copy(v.p, v.s, F->half64, st));
    }
    CHK(launch_state_reset(v.state, nullptr, 1, 1, st));
    IterArgs args;
    build_iteration(v, 0, thr, 0, 0.0, &args);
    double rate = 0;
    CHK(run_until_stop(F, v, args, &k, limit, &stt, st, rr0, thr, &rate));
    S.iters = stt.iters;
    S.rel_res = std::sqrt(stt.rr / bnorm2);
    if (!std::isfinite(stt.rr)) status = HMC_E_NAN;  // the device stops at a non-finite |r|^2
    else if (fixed == 0 && !(stt.rr <= thr)) status = HMC_E_NOCONV;
  } else {
    IterArgs args;
    build_iteration(v, 0, thr, 1, delta * delta, &args);
    CHK(inner_restart(v, 0, true, st));  // the slot holds |r64|^2 = rr0
    double rr64 = rr0, rate = 0;
    while (true) {
      // the inner iteration pauses once |r|^2 < delta^2 max|r|^2 (or <= thr)
      CHK(run_until_stop(F, v, args, &k, limit, &stt, st, rr64, std::max(thr, delta * delta * rr64), &rate));
      CHK(reliable_update(v, st));
      CHK(read_slots(F, SL_SOLVER, 1, &rr64, st));
      S.reliable_updates++;
      if (rr64 <= thr) break;
      if (!std::isfinite(rr64) || !std::isfinite(stt.rr)) {
        status = HMC_E_NAN;
        break;
      }
      if (k >= limit || S.reliable_updates >= kMaxReliable) {
        status = HMC_E_NOCONV;
        break;
      }
      CHK(inner_restart(v, k, false, st));
    }
    CHK(read_state(F, &stt, st));
    S.iters = stt.iters;
    S.rel_res = std::sqrt(rr64 / bnorm2);
  }

  // ---- odd half and FP64 true residual
  char* xx = (char*)x;
  double res2 = 0;
  if (cgls) {
    // x_o = b_o + kappa D_oe x_e;  r = b - M x on both halves (into tmp)
    CHK(dslash_f64(F, xx + F->half64, xx, 1, 0, EPI_AXPY, bb + F->half64, 1.0, F->kappa, nullptr, nullptr, 0, st));
    char* tmp = (char*)F->tmp;
    CHK(dslash_f64(F, tmp, xx + F->half64, 0, 0, EPI_AXPY, xx, 1.0, -F->kappa, nullptr, nullptr, 0, st));
    CHK(dslash_f64(F, tmp + F->half64, xx, 1, 0, EPI_AXPY, xx + F->half64, 1.0, -F->kappa, nullptr, nullptr, 0, st));
    CHK(launch_xmy_norm(F->g, bb, tmp, tmp, v.red, F->nbR, st));
    CHK(launch_xmy_norm(F->g, bb + F->half64, tmp + F->half64, tmp + F->half64, v.red + F->nbR, F->nbR, st));
    CHK(launch_finalize(v.red, 2 * F->nbR, 1, v.slot, 1.0, 0, st));
  } else {
    CHK(true_residual(v, st));
  }
  CHK(read_slots(F, SL_SOLVER, 1, &res2, st));
  S.true_rel_res = bnorm2 > 0 ? std::sqrt(res2 / bnorm2) : 0.0;
  S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = S;
  if (status == HMC_E_NOCONV) set_error("solver stopped after %d iterations at |r|/|b| = %.3e", S.iters, S.rel_res);
  if (status == HMC_E_NAN) set_error("non-finite residual after %d iterations", S.iters);
  return status;
}

}  // namespace hmc
