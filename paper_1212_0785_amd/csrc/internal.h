// Host-side internals of libhmc: device-argument structs shared by the
// kernel files and the host runtime, kernel launchers, error plumbing and
// the timing registry.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "hmc.h"

namespace hmc {

constexpr int kThreads = 256;

// Lattice description passed by value to every kernel (mirrors the device
// struct in device.h; kept layout-identical).
struct LatArg {
  int L[4];
  int Vh;
  int stride;
};

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Number of blocks of the grid-stride BLAS kernels (and of their partial
// sums): enough to fill 256 CUs several times over, never more than needed.
inline int blas_blocks(int Vh) {
  int nb = ceil_div(Vh, kThreads);
  return nb < 2048 ? nb : 2048;
}
inline int site_blocks(int Vh) { return ceil_div(Vh, kThreads); }

// Launch shapes and link forms (tune.cpp).  Dslash shape: 1 = one site per
// work-item (256 sites per block), 2 / 4 = direction split with that many
// wavefronts per 64-site group.  Staple-force shape: 0 = one link per
// work-item, 1 = plane split.  Link form: the reals read per link (LinkForm).
// Each is decided by the environment override, else the tuning table, else
// the built-in rule.
enum TuneKind {
  TUNE_DSLASH = 0,
  TUNE_GFORCE = 1,
  TUNE_DSLASH_LINKS = 2,
  TUNE_GFORCE_LINKS = 3,
  TUNE_DSLASH_STREAM = 4,
  TUNE_DSLASH_ORDER = 5,
  TUNE_DSLASH_OCC = 6
};
// All nine entries; rows 0 and 1 (LkRows2); row 0 and column 2 (LkRowCol).
// The compact forms need SU(3) links.
enum LinkForm { LINK_FULL = 18, LINK_ROWS2 = 12, LINK_ROWCOL = 10 };
int dslash_shape(const LatArg& g, hmc_prec prec);
int gauge_force_shape(const LatArg& g);
// Compact form of the hop kernels (Dslash at storage prec; the fermion
// force follows FP64) and of the staple kernels (gauge force, plaquette).
int dslash_link_form(const LatArg& g, hmc_prec prec);
int staple_link_form(const LatArg& g);
// Whether the Dslash at storage prec streams: non-temporal loads of its
// (compact) links and stores of its output, which keep that once-used data
// from displacing the neighbour spinors in L2 (pays at large volumes) but
// also from the last-level cache (costs where the fields fit in it).
bool dslash_link_stream(const LatArg& g, hmc_prec prec);
// Site order of the one-site-per-work-item Dslash (dslash_site in
// device.h): 0 linear, 1 tiled with whole z-planes, n >= 2 tiled with
// y-blocks of n 64-site chunks.  The lattice admits the tiled order with
// whole 256-site blocks, a multiple of 8 of them, a multiple of 8 t-slices
// and 64-site chunks per z-plane, or else per t-slice (then order 1 walks
// the chunks of the t-slices, t fastest); y-blocks of n chunks need whole
// chunks per z-plane and n to divide their number.
int dslash_tiled_order(const LatArg& g, hmc_prec prec);
constexpr int kMaxYBlock = 64;  // largest y-block, in chunks
// Workgroups per CU of the tiled-order Dslash: 2 (an LDS reservation keeps
// the wavefronts in flight on an XCD within a few rows of the walk) or 0 (as
// many as registers allow).
int dslash_tiled_occupancy(const LatArg& g, hmc_prec prec);
inline bool tiled_order_valid(const LatArg& g, int order = 1) {
  const int plane = g.L[0] * g.L[1] / 2, slice = plane * g.L[2];
  if (!(g.Vh % kThreads == 0 && (g.Vh / kThreads) % 8 == 0 && slice % 64 == 0 && g.L[3] % 8 == 0)) return false;
  return order == 1 || (order >= 2 && order <= kMaxYBlock && plane % 64 == 0 && (plane / 64) % order == 0);
}
// The form a kernel reads: the compact one on SU(3) links, else all entries.
inline int link_form_for(bool su3, int compact) { return su3 ? compact : (int)LINK_FULL; }
inline int dslash_shape_blocks(int Vh, int shape) { return shape == 1 ? site_blocks(Vh) : ceil_div(Vh, kThreads / 4); }
inline int dslash_blocks(const LatArg& g, hmc_prec prec) { return dslash_shape_blocks(g.Vh, dslash_shape(g, prec)); }
// Largest block count (and Dslash-epilogue partial count) of any shape.
inline int dslash_blocks_max(int Vh) { return ceil_div(Vh, kThreads / 4); }
// Tuning table: -1 when absent; load/save return entries read/written or -1.
int tune_lookup(const int* L, int kind, int prec);
void tune_store(const int* L, int kind, int prec, int choice, double us);
int tune_load(const char* path);
int tune_save(const char* path);
// Changes whenever a table entry may have changed.
uint64_t tune_generation();
// True when HMC_DSLASH_SPLIT, HMC_GFORCE_PLANES, HMC_LINK_FORM,
// HMC_LINK_STREAM or HMC_DSLASH_ORDER forces a decision.
bool tune_env_forced();

// Iteration control of the Krylov solvers, resident in device memory.
// Kernels of iteration k do nothing once k >= stop_at.  Only block 0 of the
// p-update kernel writes it, and only with a value > k, so blocks of the
// same launch never observe a change that concerns them.
struct SolverState {
  int stop_at;   // iteration label at which kernels stop (INT_MAX while running)
  int reason;    // 1 converged, 2 reliable update requested, 3 non-finite
  int iters;     // iterations completed
  int last;      // label of the last completed iteration
  int base;      // label base: added to every iteration label (advanced on the device)
  int ru_gate;   // mixed precision: INT_MAX while a reliable update is pending, else 0
  int done;      // device-driven mixed solve ended: 1 converged, 3 non-finite, 4 limit
  int nru;       // device-driven reliable updates performed
  int ru_iter;   // iterations completed at the last device-driven update
  int ru_label;  // label of the first iteration after the last device-driven update
  int restart;   // the last device-driven update restarts the search direction (p = r, or s for CGLS)
  double rr;     // last residual norm^2 seen by the p-update
  double maxrr;  // mixed precision: max inner |r|^2 since the last update
  double alpha;  // CG step length of the current iteration (fused form)
  double thr;    // stop threshold on |r|^2 (< 0: never)
  double rr64;   // FP64 |r|^2 of the last device-driven reliable update
};

// Iteration labels: a solver iteration carries the label iter0 + base + j,
// where iter0 is fixed per solve (per batch entry), base is read from the
// solver state when the kernel runs (so a recorded chunk of iterations,
// followed by a kernel that advances base, can be replayed) and j is passed
// with each launch.  Ping-pong partial buffers are chosen by the parity of
// the label.

// One Dslash application (one batch entry).
struct DslashArgs {
  const void* U;        // links in the storage format of the launch
  const void* in;       // input half-field (parity 1 - out_parity)
  void* out;            // output half-field
  const void* y;        // epilogue addend on the output parity (may be null)
  double a, b;          // out = a*y + b*(D in) for the AXPY epilogues
  double* partial;      // per-block |out|^2 for the NORM epilogue
  double* partial_pp[2];  // if set: partial_pp[(label + 1) & 1] instead
  const int* stop_at;   // solver control (may be null)
  const int* label_base;  // added to the label when set (the solver state's base)
  int iter0;            // label offset compared with *stop_at
  int su3;              // host dispatch: links are SU(3) (compact link forms allowed)
  int shape;            // host dispatch: 0 = dslash_shape(), else a fixed Dslash shape (1, 2, 4)
  // Step-length prologue (block 0 only, when alpha_out is set):
  //   *alpha_out = sum(alpha_pp[label & 1][0..n_pp)) / sum(alpha_den[0..n_den))
  const double* alpha_pp[2];
  const double* alpha_den;
  int alpha_n_pp, alpha_n_den;
  double* alpha_out;
  // EPI_CG: r <- r - (*alpha_in) (a y + b D in) with out == r, |r|^2 per block
  const void* r;
  const double* alpha_in;
};


enum Epilogue { EPI_PLAIN = 0, EPI_AXPY = 1, EPI_AXPY_NORM = 2, EPI_CG = 3 };

// Launchers (defined in the .hip files).  All return hipGetLastError().
hipError_t launch_dslash(hmc_prec prec, int dagger, int epi, const LatArg& g, int out_par, const DslashArgs* table,
                         int nbatch, const DslashArgs& one, hipStream_t st, int j = 0);

// Layout conversion between canonical AoS complex128 (device) and SoA.
hipError_t launch_pack_gauge(const LatArg& g, const void* canon, void* U, hipStream_t st);
hipError_t launch_unpack_gauge(const LatArg& g, const void* U, void* canon, hipStream_t st);
hipError_t launch_pack_spinor(const LatArg& g, const void* canon, void* half, int par, hipStream_t st);
hipError_t launch_unpack_spinor(const LatArg& g, const void* half, void* canon, int par, hipStream_t st);
hipError_t launch_pack_momenta(const LatArg& g, const void* canon, double* P, hipStream_t st);
hipError_t launch_unpack_momenta(const LatArg& g, const double* P, void* canon, hipStream_t st);
// Per-block counts of links whose third row is not conj(row0 x row1) to `tol`.
hipError_t launch_su3_check(const LatArg& g, const void* U, double tol, double* part, int nb, hipStream_t st);
hipError_t launch_convert_gauge(const LatArg& g, const void* U64, void* Ulow, hmc_prec prec, hipStream_t st);
// Launchers taking `gate`: when it is set the kernel does nothing while
// *gate == 0 (the device-driven reliable update of the mixed-precision
// solver runs them only when the inner iteration asked for one).
hipError_t launch_convert_spinor(const LatArg& g, const void* in, hmc_prec pin, void* out, hmc_prec pout,
                                 int nbatch, const void* const* tab_in, void* const* tab_out, hipStream_t st,
                                 const int* gate = nullptr);

// Reductions: per-block partials of one half-field (or several), then a
// fixed-order finalisation into a device slot.
hipError_t launch_norm2_partials(const LatArg& g, hmc_prec prec, const void* x, double* part, int nb,
                                 hipStream_t st, const int* gate = nullptr);
hipError_t launch_inner_partials(const LatArg& g, const void* a, const void* b, double* part, int nb,
                                 hipStream_t st);  // FP64 only; part holds [re..., im...]
hipError_t launch_finalize(const double* part, int n, int nvals, double* out, double scale, int accumulate,
                           hipStream_t st, const int* gate = nullptr);
hipError_t launch_sum_multi(const LatArg& g, const void* x, int nhalves, const int* subset, int nsub, double* part,
                            int nb, double* out, hipStream_t st);

// Element-wise FP64 helpers.
// out = sum_k (c[2k] + i c[2k+1]) y[k], n in 1..4 F64 half spinors.
hipError_t launch_lincomb(const LatArg& g, const void* const* y, const double* c, int n, void* out, hipStream_t st);
hipError_t launch_xmy_norm(const LatArg& g, const void* b, const void* q, void* r, double* part, int nb,
                           hipStream_t st, const int* gate = nullptr);  // r = b - q, partials of |r|^2
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
// dst = src (bytes a multiple of 8) while *gate != 0.
hipError_t launch_copy_gated(void* dst, const void* src, size_t bytes, const int* gate, hipStream_t st);

// Krylov solver kernels.  `prec` is the storage of p/r/q/s; x is FP64 for
// HMC_F64 and FP32 (inner accumulator) otherwise.
struct CgArgs {
  void* x;
  void* p;
  void* r;
  const void* q;   // operator applied to p
  const void* s;   // CGLS: Mhat^dag r
  double* pp[2];   // ping-pong partials: CG |r|^2 (n_pp = blas blocks), CGLS |s|^2 (site blocks)
  double* pq;      // CG <p, A p> = |Mhat p|^2, CGLS |q|^2 (site blocks, from the Dslash epilogue)
  double* pr;      // CGLS |r|^2 written by the update (blas blocks)
  int n_pp, n_pq, n_pr;
  SolverState* state;
  int iter0;       // label offset (the state's base is added)
  int cgls;
  double delta2;   // mixed precision: reliable-update trigger (delta^2)
  void* x64;       // mixed precision with device-driven updates: the FP64 solution, into which the
                   // iteration that asks for an update folds the inner solution (null: the host does)
  int mixed;       // 1: never declare convergence, pause instead
  int fused;       // CG with the residual update in the Dslash epilogue: the p-update also does x += alpha p
  int max_iters;   // device-driven updates: the iteration that completes this many asks for the last one (0: none)
};
hipError_t launch_cg_init(const LatArg& g, hmc_prec prec, const void* b, void* x, void* r, void* p, double* part,
                          int nb, hipStream_t st);
hipError_t launch_cg_update(const LatArg& g, hmc_prec prec, const CgArgs& a, int nb, const CgArgs* table,
                            int nbatch, int j, hipStream_t st);
hipError_t launch_cg_pupdate(const LatArg& g, hmc_prec prec, const CgArgs& a, int nb, const CgArgs* table,
                             int nbatch, int j, hipStream_t st);
// Start (reset_iters: counts, base and the device-driven fields cleared) or
// resume a solve: stop_at = INT_MAX, reason = 0, maxrr from a device slot
// (null -> 0), stop threshold thr; label >= 0 sets ru_label, the label of the
// first iteration of a host-driven restart.
hipError_t launch_state_reset(SolverState* st_dev, const double* maxrr, int nbatch, int reset_iters, double thr,
                              hipStream_t st, int label = -1);
// base += n (one solve): closes a chunk of n iterations launched with j = 0..n-1.
hipError_t launch_advance_base(SolverState* st_dev, int n, hipStream_t st);
// STREAM triad a = b + sc * c over n2 double2 elements (nt: non-temporal).
hipError_t launch_triad(void* a, const void* b, const void* c, double sc, size_t n2, bool nt, hipStream_t st);
hipError_t launch_add_low_to_f64(const LatArg& g, void* x64, void* xlow, hipStream_t st,
                                 const int* gate = nullptr);  // x += xl; xl = 0
// Ends a device-driven reliable update (when st->ru_gate is set): sums the n
// |r64|^2 partials into *rr64_slot, counts the update and either ends the
// solve (converged, non-finite, max_ru updates or max_iters iterations
// reached) or resumes the inner iteration (stop_at = INT_MAX, maxrr =
// |r64|^2); sets st->restart when the search direction must restart (the
// FP64 residual exceeds twice the inner one that asked for the update, or
// did not fall below the previous update's), else clears it (also when no
// update was pending); clears the gate.
hipError_t launch_ru_finish(SolverState* st_dev, const double* part64, int n, double* rr64_slot, int max_ru,
                            int max_iters, hipStream_t st);
// Device-driven reliable update after q = A x (gated): r64 = rhs - q with
// |r64|^2 partials (nb blocks), r = r64 in storage prec; with pp0 set also
// the |r|^2 partials of the stored r into pp0 and pp1 (nb = the iteration's
// partial count).
hipError_t launch_ru_residual(const LatArg& g, hmc_prec prec, const void* rhs, const void* q, void* r64, void* rlow,
                              double* part64, double* pp0, double* pp1, int nb, const int* gate, hipStream_t st);
// dst = src over n doubles while *gate != 0.
hipError_t launch_copy_doubles_gated(double* dst, const double* src, int n, const int* gate, hipStream_t st);
// Asks for a reliable update from the host: opens the gate and stops the
// iterations still queued.
hipError_t launch_ru_request(SolverState* st_dev, hipStream_t st);

// Gauge-field kernels.
// su3: U is SU(3) to rounding (compact link forms allowed).
// Plaquette sum on SU(3) links: 1 = three wavefronts per 64 sites, two
// planes each; 0 = four 64-site units per block, all planes per work-item
// (the only form on links that are not SU(3)).
int plaquette_shape(const LatArg& g);
// Non-temporal loads and stores of the once-used data in the link update
// and in the fermion force (large lattices).
bool exp_update_stream(const LatArg& g);
bool fermion_force_stream(const LatArg& g);
// The same for the momenta of the site-blocked staple force.
bool gauge_force_stream(const LatArg& g);
// Compact link form of the plaquette sum on SU(3) links.
int plaquette_link_form(const LatArg& g);
// One partial per block, plaquette_blocks(g, su3) of them (at most
// 2 ceil(Vh / 64)).
int plaquette_blocks(const LatArg& g, bool su3);
hipError_t launch_plaquette_partials(const LatArg& g, const void* U, double* part, hipStream_t st, bool su3);
hipError_t launch_kinetic_partials(const LatArg& g, const double* P, double* part, int nb, hipStream_t st);
// shape: -1 = gauge_force_shape(), 0 / 1 / 2 = fixed; form: 0 =
// staple_link_form(), else a fixed compact form (used on SU(3) links only).
hipError_t launch_gauge_force(const LatArg& g, const void* U, double* P, double coef_beta, hipStream_t st,
                              bool su3, int shape = -1, int form = 0);
// su3: U is SU(3) to rounding (rows 0 and 1 read, row 2 rebuilt).
hipError_t launch_exp_update(const LatArg& g, void* U, const double* P, double eps, hipStream_t st, bool su3);
hipError_t launch_fermion_force(const LatArg& g, const void* U, const void* Xe, const void* Xo, const void* Ye,
                                const void* Yo, double* P, double coef, hipStream_t st,
                                bool su3);

// Random fields (Philox4x64-10, counter = (block, lex site, stream, epoch),
// key = (seed, 0)).
hipError_t launch_refresh_momenta(const LatArg& g, uint64_t seed, uint64_t epoch, double* P, hipStream_t st);
hipError_t launch_weak_field(const LatArg& g, uint64_t seed, double eps, void* U, hipStream_t st);
// Pseudofermion noise from Philox stream 2 (second = 0) or stream 5 (the
// second pseudofermion of the mass-preconditioned action).
hipError_t launch_eta(const LatArg& g, uint64_t seed, uint64_t epoch, int par, void* half, hipStream_t st,
                      int second = 0);
hipError_t launch_source(const LatArg& g, int kind, uint64_t seed, uint64_t epoch, void* even, void* odd,
                         hipStream_t st);
hipError_t launch_site_words(uint64_t seed, uint64_t stream, uint64_t epoch, const long long* sites, int nsites,
                             int nblocks, uint64_t* out, hipStream_t st);
hipError_t launch_site_gaussians(uint64_t seed, uint64_t stream, uint64_t epoch, const long long* sites,
                                 int nsites, int n, double* out, hipStream_t st);
// Metropolis on device: slots[0..] hold the action pieces (see hmc.cpp).
hipError_t launch_metropolis(uint64_t seed, uint64_t traj, double beta, double V, double* slots, hipStream_t st);

// ----------------------------------------------------------- errors

void set_error(const char* fmt, ...);
const char* last_error();

#define HMC_CHECK_HIP(expr)                                                                     \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) {                                                                      \
      ::hmc::set_error("%s:%d: %s: %s", __FILE__, __LINE__, #expr, hipGetErrorString(e_));       \
      return HMC_E_HIP;                                                                          \
    }                                                                                            \
  } while (0)

#define HMC_REQUIRE(cond, ...)        \
  do {                                \
    if (!(cond)) {                    \
      ::hmc::set_error(__VA_ARGS__);  \
      return HMC_E_ARG;               \
    }                                 \
  } while (0)

// ----------------------------------------------------------- timing

// Kernel families timed with HIP events when sampling is on.
enum TimedKernel {
  TK_DSLASH = 0,
  TK_CG_BLAS,
  TK_REDUCE,
  TK_GAUGE_FORCE,
  TK_FERMION_FORCE,
  TK_EXP_UPDATE,
  TK_REFRESH,
  TK_PLAQUETTE,
  TK_OTHER,
  TK_COUNT
};
const char* timed_kernel_name(int k);
// Byte counts of a timed launch: `bytes` are the method's algorithmic bytes
// (every datum of the operation read once and every output written once,
// SU(3) links as their nine complex entries), `moved` the bytes of the data
// the kernel as implemented must move (compact links: the stored reals it
// reads); moved < 0 means the same as bytes.
// Returns true and records a start event when this launch is sampled.
bool timing_begin(int kernel, hipStream_t st, double bytes, double moved = -1.0);
void timing_end(int kernel, hipStream_t st);

// Event pair for a sampled launch of `kernel` (both null when this launch is
// not sampled).  Passed to hipExtLaunchKernelGGL, the events take the
// kernel's own start and end stamps, so their elapsed time is the kernel's
// duration as a kernel trace reports it.
struct KernelEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
KernelEvents timing_kernel_events(int kernel, double bytes, double moved = -1.0);
// The next n launches of `kernel` (consecutive on one stream, nothing of
// another family between them) form one sample: one event pair from the
// start of the first to the end of the last, so the pair's own cost is
// paid once for the group; their bytes and launch count add up.
void timing_group_begin(int kernel, int n);
// Closes the group (drops its sample if fewer than n launches happened).
void timing_group_end();
// While on, launches of this thread are being recorded into a graph: they
// take no events and are not counted (timing_count counts them per replay).
void timing_set_recording(bool on);
void timing_count(int kernel, long long n);
bool timing_enabled();
int timing_sample_every();
// While on, every launch of this thread is sampled.
void timing_sample_all(bool on);
// An empty one-wavefront kernel launched with the event pair of the "other"
// family (sampled like any launch).
hipError_t launch_empty_timed(hipStream_t st);

// Brackets a launch with events recorded on the stream (includes the
// dispatch of the kernel).
struct TimedScope {
  int k;
  hipStream_t st;
  bool on;
  TimedScope(int kernel, hipStream_t s, double bytes, double moved = -1.0)
      : k(kernel), st(s), on(timing_begin(kernel, s, bytes, moved)) {}
  ~TimedScope() {
    if (on) timing_end(k, st);
  }
};

}  // namespace hmc
