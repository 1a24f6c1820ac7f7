// Krylov solvers for the fermion-matrix inversion (the operation the paper's
// introduction identifies with the bulk of the floating-point work).
//
//  * CG (Hestenes-Stiefel) on A = Mhat^dag Mhat for the HMC force, x0 = 0,
//    stop at the first k with |r_k| <= tol |b|.
//  * CGLS on Mhat x_e = bhat_e for Wilson solves M x = b, through the
//    Schur complement bhat_e = b_e + kappa D_eo b_o, x_o = b_o + kappa D_oe x_e.
//  * Mixed precision: the same iteration on FP32 / FP16 / BF16 storage with
//    FP32 arithmetic and FP64 global sums; whenever the inner residual has
//    fallen by reliable_delta since the last update, x is folded into the
//    FP64 solution and the residual replaced by the FP64 true residual
//    (reliable updates, Clark et al., Comput. Phys. Commun. 181 (2010) 1517).
//
// Each iteration is a fixed sequence of kernels on one stream with every
// scalar (alpha, beta, the stop test) computed on the device.  The host
// enqueues chunks of iterations and reads the 32-byte solver state once per
// chunk; iterations enqueued after the stop are no-ops (stop_at).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>

#include "fields.h"

namespace hmc {

namespace {

constexpr int kChunk = 16;
constexpr int kMaxReliable = 2000;  // a solve that needs more has stagnated

struct Ctx {
  Fields* F;
  hipStream_t st;
  int nbD, nbR;
};

// Vectors of one iteration family (FP64 or low precision).
struct Vecs {
  hmc_prec prec;
  const void* U;
  void *x, *r, *p, *q, *s, *t;
};

hipError_t ds(const Ctx& c, const Vecs& v, void* out, const void* in, int out_par, int dag, int epi, const void* y,
              double a, double b, double* partial, int iter) {
  DslashArgs d;
  d.U = v.U;
  d.in = in;
  d.out = out;
  d.y = y;
  d.a = a;
  d.b = b;
  d.partial = partial;
  d.stop_at = &c.F->state->stop_at;
  d.iter = iter;
  return launch_dslash(v.prec, dag, epi, c.F->g, out_par, nullptr, 1, d, c.st);
}

// out = Mhat(dag) in with |out|^2 partials when `partial` is set.
hipError_t mhat(const Ctx& c, const Vecs& v, void* out, const void* in, int dag, double* partial, int iter) {
  hipError_t e = ds(c, v, v.t, in, 1, dag, EPI_PLAIN, nullptr, 0.0, 1.0, nullptr, iter);
  if (e != hipSuccess) return e;
  const double k2 = c.F->kappa * c.F->kappa;
  return ds(c, v, out, v.t, 0, dag, partial ? EPI_AXPY_NORM : EPI_AXPY, in, 1.0, -k2, partial, iter);
}

struct Parts {
  double* a[2];  // ping-pong: CG |r|^2 (nbR) / CGLS |s|^2 (nbD)
  double* q;     // CG <p,Ap> = |Mhat p|^2 (nbD) / CGLS |q|^2 (nbD)
  double* r;     // CGLS |r|^2 (nbR)
};

// One iteration (index k) of CG (cgls=0) or CGLS (cgls=1).
hipError_t iterate(const Ctx& c, const Vecs& v, const Parts& P, int cgls, int k, double thr, int mixed,
                   double delta2) {
  hipError_t e;
  const int cur = k & 1, nxt = cur ^ 1;
  CgArgs u{};
  u.state = c.F->state;
  u.iter = k;
  u.thr = thr;
  u.mixed = mixed;
  u.delta2 = delta2;
  if (!cgls) {
    // s = Mhat p (|s|^2 = <p, A p>), q = Mhat^dag s
    if ((e = mhat(c, v, v.s, v.p, 0, P.q, k))) return e;
    if ((e = mhat(c, v, v.q, v.s, 1, nullptr, k))) return e;
    u.x = v.x;
    u.p = v.p;
    u.r = v.r;
    u.q = v.q;
    u.part_a = P.a[cur];
    u.n_a = c.nbR;
    u.part_b = P.q;
    u.n_b = c.nbD;
    u.part_out = P.a[nxt];
    if ((e = launch_cg_update(c.F->g, v.prec, u, c.nbR, nullptr, 1, c.st))) return e;
    u.part_a = P.a[nxt];
    u.n_a = c.nbR;
    u.part_b = P.a[cur];
    u.n_b = c.nbR;
    return launch_cg_pupdate(c.F->g, v.prec, 0, u, c.nbR, nullptr, 1, c.st);
  }
  // q = Mhat p, |q|^2 ; x += alpha p ; r -= alpha q ; s = Mhat^dag r ; p = s + beta p
  if ((e = mhat(c, v, v.q, v.p, 0, P.q, k))) return e;
  u.x = v.x;
  u.p = v.p;
  u.r = v.r;
  u.q = v.q;
  u.s = v.s;
  u.part_a = P.a[cur];
  u.n_a = c.nbD;
  u.part_b = P.q;
  u.n_b = c.nbD;
  u.part_out = P.r;
  if ((e = launch_cg_update(c.F->g, v.prec, u, c.nbR, nullptr, 1, c.st))) return e;
  if ((e = mhat(c, v, v.s, v.r, 1, P.a[nxt], k))) return e;
  u.part_a = P.a[nxt];
  u.n_a = c.nbD;
  u.part_b = P.a[cur];
  u.n_b = c.nbD;
  u.part_c = P.r;
  u.n_c = c.nbR;
  return launch_cg_pupdate(c.F->g, v.prec, 1, u, c.nbR, nullptr, 1, c.st);
}

hipError_t read_state(const Ctx& c, SolverState* out) {
  hipError_t e = hipMemcpyAsync(c.F->pinned + SL_COUNT, c.F->state, sizeof(SolverState), hipMemcpyDeviceToHost, c.st);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(c.st)) != hipSuccess) return e;
  std::memcpy(out, c.F->pinned + SL_COUNT, sizeof(SolverState));
  return hipSuccess;
}

hipError_t reduce_to_host(const Ctx& c, const double* part, int n, double* out) {
  hipError_t e = launch_finalize(part, n, 1, c.F->slots + SL_SOLVER, 1.0, 0, c.st);
  if (e != hipSuccess) return e;
  return read_slots(c.F, SL_SOLVER, 1, out, c.st);
}

// Runs iterations k0.. until the device stops (converged / reliable update
// requested) or `limit` iterations in total.  Returns the state.
hipError_t run_until_stop(const Ctx& c, const Vecs& v, const Parts& P, int cgls, int* k, int limit, double thr,
                          int mixed, double delta2, SolverState* stt) {
  while (*k < limit) {
    int n = std::min(kChunk, limit - *k);
    for (int j = 0; j < n; ++j) {
      hipError_t e = iterate(c, v, P, cgls, *k + j, thr, mixed, delta2);
      if (e != hipSuccess) return e;
    }
    hipError_t e = read_state(c, stt);
    if (e != hipSuccess) return e;
    *k = stt->iter;
    if (stt->stop_at != INT_MAX) return hipSuccess;
  }
  return hipSuccess;
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
  Ctx c{F, st, F->nbD, F->nbR};
  const double tol = prm->tol;
  const int fixed = prm->fixed_iters;
  const int limit = fixed > 0 ? fixed : prm->maxiter;
  const double delta = prm->reliable_delta > 0 ? prm->reliable_delta : 0.1;
  Parts P{{F->part[0], F->part[1]}, F->part[2], F->part[3]};
  Vecs v64{HMC_F64, F->U, x, F->r, F->p, F->q, F->s, F->t};
  hmc_cg_stats S{};

  // ---- set-up in FP64: b_norm2, the right-hand side rhs (b or bhat), x = 0, r = rhs
  const char* bb = (const char*)b;
  double bnorm2 = 0;
  const void* rhs = b;
  if (cgls) {
    CHK(launch_norm2_partials(F->g, HMC_F64, bb, F->part[4], F->nbR, st));
    CHK(launch_norm2_partials(F->g, HMC_F64, bb + F->half64, F->part[4] + F->nbR, F->nbR, st));
    CHK(reduce_to_host(c, F->part[4], 2 * F->nbR, &bnorm2));
    // bhat_e = b_e + kappa D_eo b_o
    CHK(dslash_f64(F, F->bhat, bb + F->half64, 0, 0, EPI_AXPY, bb, 1.0, F->kappa, nullptr, nullptr, 0, st));
    rhs = F->bhat;
  }
  double rr0 = 0;
  CHK(launch_cg_init(F->g, HMC_F64, rhs, x, F->r, F->p, P.a[0], F->nbR, st));
  CHK(reduce_to_host(c, P.a[0], F->nbR, &rr0));
  if (!cgls) bnorm2 = rr0;
  const double thr = fixed > 0 ? -1.0 : tol * tol * bnorm2;

  int k = 0;
  SolverState stt{};
  hmc_status status = HMC_OK;
  if (bnorm2 == 0.0) {
    // x = 0 solves it exactly
  } else if (prec == HMC_F64) {
    CHK(launch_state_reset(F->state, 0, nullptr, 1, st));
    if (cgls) {
      // s = Mhat^dag r, p = s, |s|^2 -> P.a[0]
      CHK(mhat(c, v64, F->s, F->r, 1, P.a[0], 0));
      CHK(launch_copy(F->p, F->s, F->half64, st));
    }
    if (rr0 > thr) CHK(run_until_stop(c, v64, P, cgls, &k, limit, thr, 0, 0.0, &stt));
    const double rr_last = k ? stt.rr : rr0;
    S.rel_res = std::sqrt(rr_last / bnorm2);
    if (fixed == 0 && !(rr_last <= thr)) status = HMC_E_NOCONV;
  } else {
    // ---- mixed precision with reliable updates
    CHK(ensure_lowprec(F, prec, st));
    Vecs vl{prec, low_links(F, prec), F->lx, F->lr, F->lp, F->lq, F->ls, F->lt};
    // FP64 residual of the current x (x = 0): r64 = rhs, |r64|^2 = rr0
    double rr64 = rr0;
    CHK(launch_zero(F->lx, (size_t)F->g.Vh * 96, st));
    bool first = true;
    while (true) {
      if (rr64 <= thr) break;
      if (k >= limit || S.reliable_updates >= kMaxReliable) {
        status = HMC_E_NOCONV;
        break;
      }
      // r_low = low(r64); CG: p = r (first time); CGLS: s = Mhat^dag r, p = s (first time)
      CHK(launch_convert_spinor(F->g, F->r, HMC_F64, F->lr, prec, 1, nullptr, nullptr, st));
      const int cur = k & 1;
      if (cgls) {
        CHK(mhat(c, vl, F->ls, F->lr, 1, P.a[cur], k));
        if (first) CHK(launch_copy(F->lp, F->ls, F->halflow, st));
      } else {
        CHK(launch_norm2_partials(F->g, prec, F->lr, P.a[cur], F->nbR, st));
        if (first) CHK(launch_copy(F->lp, F->lr, F->halflow, st));
      }
      first = false;
      // the last reduction left |r64|^2 in the solver slot: it seeds maxrr
      CHK(launch_state_reset(F->state, k, F->slots + SL_SOLVER, 1, st));
      CHK(run_until_stop(c, vl, P, cgls, &k, limit, thr, 1, delta * delta, &stt));
      // reliable update: x += x_low; r64 = rhs - A x
      CHK(launch_add_low_to_f64(F->g, x, F->lx, st));
      if (cgls) {
        CHK(mhat_f64(F, F->q, x, 0, nullptr, st));
      } else {
        CHK(mhat_f64(F, F->s, x, 0, nullptr, st));
        CHK(mhat_f64(F, F->q, F->s, 1, nullptr, st));
      }
      CHK(launch_xmy_norm(F->g, rhs, F->q, F->r, F->part[5], F->nbR, st));
      CHK(reduce_to_host(c, F->part[5], F->nbR, &rr64));
      S.reliable_updates++;
      if (!(rr64 == rr64)) {
        status = HMC_E_NOCONV;
        break;
      }
    }
    S.rel_res = std::sqrt(rr64 / bnorm2);
  }

  // ---- odd half and FP64 true residual
  char* xx = (char*)x;
  double res2 = 0;
  if (cgls) {
    // x_o = b_o + kappa D_oe x_e
    CHK(dslash_f64(F, xx + F->half64, xx, 1, 0, EPI_AXPY, bb + F->half64, 1.0, F->kappa, nullptr, nullptr, 0, st));
    // r = b - M x on both halves (into tmp)
    char* tmp = (char*)F->tmp;
    CHK(dslash_f64(F, tmp, xx + F->half64, 0, 0, EPI_AXPY, xx, 1.0, -F->kappa, nullptr, nullptr, 0, st));
    CHK(dslash_f64(F, tmp + F->half64, xx, 1, 0, EPI_AXPY, xx + F->half64, 1.0, -F->kappa, nullptr, nullptr, 0, st));
    CHK(launch_xmy_norm(F->g, bb, tmp, tmp, F->part[5], F->nbR, st));
    CHK(launch_xmy_norm(F->g, bb + F->half64, tmp + F->half64, tmp + F->half64, F->part[5] + F->nbR, F->nbR, st));
    CHK(reduce_to_host(c, F->part[5], 2 * F->nbR, &res2));
  } else {
    CHK(mhat_f64(F, F->s, x, 0, nullptr, st));
    CHK(mhat_f64(F, F->q, F->s, 1, nullptr, st));
    CHK(launch_xmy_norm(F->g, b, F->q, F->tmp, F->part[5], F->nbR, st));
    CHK(reduce_to_host(c, F->part[5], F->nbR, &res2));
  }
  S.iters = k;
  S.true_rel_res = bnorm2 > 0 ? std::sqrt(res2 / bnorm2) : 0.0;
  S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = S;
  if (status == HMC_E_NOCONV) set_error("solver stopped after %d iterations at |r|/|b| = %.3e", k, S.rel_res);
  return status;
}

}  // namespace hmc
