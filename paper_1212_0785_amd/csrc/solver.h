// Krylov solver building blocks shared by the single-solve entry point and
// the batched solve service: the device vectors of one solve, the kernel
// arguments of one iteration, and launchers for one solve or a batch of
// same-volume solves (one launch per step, blockIdx.y = batch entry).
#pragma once

#include "internal.h"

namespace hmc {

// Device buffers of one solve.  For an FP64 solve the inner vectors alias
// the FP64 ones and xl is the FP64 solution.
struct SolveVecs {
  LatArg g;
  double kappa;
  int cgls;          // 1: Wilson solve (CGLS on Mhat), 0: CG on Mhat^dag Mhat
  hmc_prec prec;     // storage of the inner iteration
  const void* U64;   // FP64 links
  const void* Ulow;  // links in `prec` (== U64 for F64)
  int su3;           // links are SU(3): compact link forms allowed
  int shape, shape64;  // Dslash shapes of the solve (inner storage, FP64), fixed at its start
  void* x;           // FP64 solution, even half
  void* r64;         // FP64 residual (mixed) / residual (F64)
  void* rhs;         // right-hand side of the even system (b or bhat)
  void* q64;         // FP64 temporaries (even, even, odd)
  void* s64;
  void* t64;
  void *r, *p, *q, *s, *t, *xl;  // inner vectors (t odd)
  double* pp[2];     // ping-pong partials
  double* pq;        // Dslash-epilogue partials
  double* pr;        // update-kernel partials
  double* red;       // scratch partials for FP64 reductions (>= 2 * nbR)
  double* slot;      // device scalar (FP64 reductions land here)
  SolverState* state;
  double thr;        // stop threshold on |r|^2 of the solve
  int nbD, nbR;
};

// Arguments of the six launches of one iteration.
struct IterArgs {
  DslashArgs d[4];
  CgArgs c[2];
};

// device_updates: mixed precision with the reliable updates decided and
// performed on the device (the iteration that asks for one folds the inner
// solution into the FP64 one).
void build_iteration(const SolveVecs& v, int iter0, int mixed, double delta2, IterArgs* out,
                     bool device_updates = false);

// Device copies of the per-entry arguments of a batch (each an array of
// nbatch entries), or nullptrs for a single solve taken from `one`.
struct IterTables {
  const DslashArgs* d[4];
  const CgArgs* c[2];
};

// Launch one iteration (label iter0 + j per entry).
hipError_t launch_iteration(const LatArg& g, hmc_prec prec, int cgls, const IterTables* tab, const IterArgs& one,
                            int nbatch, int nbD, int nbR, int j, hipStream_t st);

// FP64 helpers on one solve (single-entry launches).
hipError_t mhat64(const SolveVecs& v, void* out, const void* in, int dag, double* partial, hipStream_t st);
// r64 = rhs - A x (A = Mhat or Mhat^dag Mhat), |r64|^2 -> v.slot.
hipError_t true_residual(const SolveVecs& v, hipStream_t st);
// Mixed precision: fold xl into x, FP64 residual into v.slot.
hipError_t reliable_update(const SolveVecs& v, hipStream_t st);
// Restart the inner iteration from the FP64 residual at label k: r = low(r64),
// CGLS s = Mhat^dag r (partials into pp[k&1]) / CG |r|^2 into pp[k&1]; on the
// first start, or with restart_p, also p = s (CGLS) or r (CG); state reset
// with maxrr = |r64|^2.
hipError_t inner_restart(const SolveVecs& v, int k, bool first, hipStream_t st, bool restart_p = false);

}  // namespace hmc
