// Host-side fields object: device pointers carved from the caller's arena,
// plus the small pinned host buffer used to read back device scalars.
#pragma once

#include <climits>
#include <cstdint>
#include <string>
#include <vector>

#include "internal.h"

namespace hmc {

// Device scalar slots (doubles) used by the trajectory and the reductions.
enum Slot {
  SL_KE_OLD = 0,
  SL_PLAQ_OLD = 1,
  SL_ETA2 = 2,
  SL_KE_NEW = 3,
  SL_PLAQ_NEW = 4,
  SL_PHIX = 5,  // 5 re, 6 im (overwritten by the Metropolis outputs 6..12)
  SL_H_OLD = 6,
  SL_H_NEW = 7,
  SL_DH = 8,
  SL_U = 9,
  SL_ACC = 10,
  SL_SG_OLD = 11,
  SL_SG_NEW = 12,
  SL_RED = 16,  // 16..31 general reductions
  SL_SOLVER = 32,  // 32..47 solver scalars
  SL_CHRONO = 64,  // 64..103 Gram matrix and right-hand side of the chronological guess
  SL_COUNT = 128
};

constexpr int kNumPart = 8;

struct Fields {
  LatArg g;
  long long V;
  double beta, kappa;
  uint32_t flags;
  char* arena;
  size_t arena_bytes;
  size_t half64;  // bytes of an F64 half spinor
  size_t halflow; // bytes reserved for a low-precision half spinor

  void* U;
  void* U_old;
  double* P;
  void* eta;
  void* phi;
  void* Xe;
  void* Xo;
  void* Ye;
  void* Yo;
  // mass-preconditioned action: second pseudofermion, its noise, chi and X_2
  void *eta2, *phi2, *chi, *X2;
  // chronological guess: previous solutions of the trajectory, oldest first
  static constexpr int kChronoMax = 4;
  void* hist[kChronoMax];
  int n_hist;
  // FP64 solver vectors (even half spinors, t odd)
  void *r, *p, *q, *s, *t, *bhat, *tmp;
  // partial-sum buffers, each of npart doubles
  double* part[kNumPart];
  int npart;
  int nbD, nbR;
  double* multi;  // sumMulti partial rows
  size_t multi_doubles;
  SolverState* state;
  double* slots;
  // low precision copies (index by hmc_prec; [0] unused)
  void* Ulow[4];
  void *lr, *lp, *lq, *ls, *lt, *lx;
  uint64_t u_version;
  uint64_t low_version[4];
  // U is SU(3) to rounding in the sense the two-row link loads need: every
  // stored third row equals conj(row0 x row1) (checked on import and sync,
  // kept by the reunitarised updates).  su3_old: the same for U_old.
  bool su3, su3_old;
  double* pinned;  // host, hipHostMalloc'ed, SL_COUNT + 64 doubles
  hipEvent_t state_ev[2];  // solver-state read-backs in flight (pinned + SL_COUNT + 16 * i)
  // Recorded chunks of solver iterations (HIP graphs replayed on the
  // caller's stream), keyed by everything their launches depend on, and the
  // stream they are recorded on (no work ever runs there).
  struct Recorded {
    std::string key;
    hipGraphExec_t exec;
    uint64_t last_use;
  };
  std::vector<Recorded> recorded;
  hipStream_t record_stream = nullptr;
  uint64_t record_clock = 0;
  bool record_failed = false;
};

inline Fields* as_fields(hmc_fields* f) { return reinterpret_cast<Fields*>(f); }

// Solver entry (solver.cpp).
hmc_status cg_solve_impl(Fields* F, void* x, const void* b, const hmc_cg_params* prm, hmc_cg_stats* stats,
                         hipStream_t st);
// Half-lattice helpers (hmc.cpp) used by the solver and the integrator.
hipError_t dslash_f64(Fields* F, void* out, const void* in, int out_par, int dag, int epi, const void* y, double a,
                      double b, double* partial, const int* stop_at, int iter, hipStream_t st);
// out = Mhat(dag) in on F64 half spinors (uses the odd temporary t).
hipError_t mhat_f64(Fields* F, void* out, const void* in, int dag, double* partial, hipStream_t st);
hipError_t ensure_lowprec(Fields* F, hmc_prec prec, hipStream_t st);
// Re-derives F->su3 from the stored links (one reduction; syncs).
hipError_t check_su3(Fields* F, hipStream_t st);
void* low_links(Fields* F, hmc_prec prec);
// Read `n` device doubles from slots[first..] into the pinned buffer (syncs).
hipError_t read_slots(Fields* F, int first, int n, double* out, hipStream_t st);

}  // namespace hmc
