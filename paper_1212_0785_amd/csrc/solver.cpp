// Krylov solvers for the fermion-matrix inversion (the operation the paper's
// introduction identifies with the bulk of the floating-point work).
//
//  * CG (Hestenes-Stiefel) on A = Mhat^dag Mhat for the HMC force, x0 = 0,
//    stop at the first k with |r_k| <= tol |b|.
//  * CGLS on Mhat x_e = bhat_e for Wilson solves M x = b, through the
//    Schur complement bhat_e = b_e + kappa D_eo b_o, x_o = b_o + kappa D_oe x_e.
//  * Mixed precision: the same iteration on FP32 / FP16 / BF16 storage with
//    FP32 arithmetic and FP64 global sums; whenever the inner residual has
//    fallen by reliable_delta since the last update (or 48 inner iterations
//    have passed), the inner solution is folded into the FP64 solution and
//    the residual replaced by the FP64 true residual (reliable updates,
//    Clark et al., Comput. Phys. Commun. 181 (2010) 1517).  The search
//    direction is kept unless the update finds the recursion off track
//    (FP64 |r|^2 above twice the inner one, or no decrease over a cycle),
//    when it restarts from the new residual.
//
// An iteration is six launches on one stream (four Dslash, two vector
// kernels) with alpha, beta and the stop test computed on the device.  The
// host enqueues chunks of iterations and reads the solver state once per
// chunk; iterations enqueued after the stop exit at once.  A chunk of n
// iterations is launched with j = 0..n-1 and closed by a kernel that
// advances the state's label base by n, so the same launches serve every
// chunk of that length (and can be recorded once into a HIP graph and
// replayed; see graphs_mode).  In mixed precision the reliable update is
// part of the chunk too, decided and gated on the device (it runs only
// when the inner iteration asked for it), so a solve needs no host round
// trip until it ends.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "fields.h"
#include "solver.h"

namespace hmc {

namespace {
constexpr int kChunk = 16;
constexpr int kMaxReliable = 2000;  // a solve that needs more has stagnated
constexpr int kMaxRecorded = 64;    // recorded chunks kept per fields object
constexpr int kStateSlot = 16;      // doubles per solver-state read-back slot
}  // namespace

void build_iteration(const SolveVecs& v, int iter0, int mixed, double delta2, IterArgs* o, bool device_updates) {
  std::memset(o, 0, sizeof *o);  // the recorded-launch key compares these bytes
  const double k2 = v.kappa * v.kappa;
  DslashArgs b{};
  b.U = v.Ulow;
  b.su3 = v.su3;
  b.shape = v.shape;
  b.stop_at = &v.state->stop_at;
  b.label_base = &v.state->base;
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
  c.delta2 = delta2;
  c.x64 = mixed && device_updates ? v.x : nullptr;
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

// One FP64 hop of a solve; with `gate` set it runs only while *gate != 0
// (label 0 against the gate as stop_at).
static hipError_t ds64(const SolveVecs& v, void* out, const void* in, int out_par, int dag, int epi, const void* y,
                       double a, double b, double* partial, hipStream_t st, const int* gate = nullptr) {
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
  d.stop_at = gate;
  return launch_dslash(HMC_F64, dag, epi, v.g, out_par, nullptr, 1, d, st, 0);
}

static hipError_t mhat64_gated(const SolveVecs& v, void* out, const void* in, int dag, double* partial,
                               hipStream_t st, const int* gate) {
  hipError_t e = ds64(v, v.t64, in, 1, dag, EPI_PLAIN, nullptr, 0.0, 1.0, nullptr, st, gate);
  if (e != hipSuccess) return e;
  return ds64(v, out, v.t64, 0, dag, partial ? EPI_AXPY_NORM : EPI_AXPY, in, 1.0, -v.kappa * v.kappa, partial, st,
              gate);
}

hipError_t mhat64(const SolveVecs& v, void* out, const void* in, int dag, double* partial, hipStream_t st) {
  return mhat64_gated(v, out, in, dag, partial, st, nullptr);
}

static hipError_t true_residual_gated(const SolveVecs& v, hipStream_t st, const int* gate) {
  hipError_t e;
  if (v.cgls) {
    if ((e = mhat64_gated(v, v.q64, v.x, 0, nullptr, st, gate))) return e;
  } else {
    if ((e = mhat64_gated(v, v.s64, v.x, 0, nullptr, st, gate))) return e;
    if ((e = mhat64_gated(v, v.q64, v.s64, 1, nullptr, st, gate))) return e;
  }
  if ((e = launch_xmy_norm(v.g, v.rhs, v.q64, v.r64, v.red, v.nbR, st, gate))) return e;
  return launch_finalize(v.red, v.nbR, 1, v.slot, 1.0, 0, st, gate);
}

hipError_t true_residual(const SolveVecs& v, hipStream_t st) { return true_residual_gated(v, st, nullptr); }

hipError_t reliable_update(const SolveVecs& v, hipStream_t st) {
  hipError_t e = launch_add_low_to_f64(v.g, v.x, v.xl, st);
  if (e != hipSuccess) return e;
  return true_residual(v, st);
}

// r = low(r64) (unless already converted) and the inner |r|^2 (CG) or
// s = Mhat^dag r with |s|^2 (CGLS) into `part`, optionally gated.
static hipError_t restart_vectors(const SolveVecs& v, double* part, hipStream_t st, const int* gate,
                                  bool convert = true) {
  hipError_t e;
  if (convert && (e = launch_convert_spinor(v.g, v.r64, HMC_F64, v.r, v.prec, 1, nullptr, nullptr, st, gate)))
    return e;
  if (!v.cgls) return launch_norm2_partials(v.g, v.prec, v.r, part, v.nbD, st, gate);
  DslashArgs d{};
  d.U = v.Ulow;
  d.su3 = v.su3;
  d.shape = v.shape;
  d.in = v.r;
  d.out = v.t;
  d.a = 1.0;
  d.b = 1.0;
  d.stop_at = gate;
  if ((e = launch_dslash(v.prec, 1, EPI_PLAIN, v.g, 1, nullptr, 1, d, st, 0))) return e;
  d.in = v.t;
  d.out = v.s;
  d.y = v.r;
  d.b = -v.kappa * v.kappa;
  d.partial = part;
  return launch_dslash(v.prec, 1, EPI_AXPY_NORM, v.g, 0, nullptr, 1, d, st, 0);
}

static size_t low_half_bytes(const SolveVecs& v) {
  return (size_t)v.g.Vh * (v.prec == HMC_F32 ? 96 : v.prec == HMC_F16 ? 52 : 48);
}

hipError_t inner_restart(const SolveVecs& v, int k, bool first, hipStream_t st, bool restart_p) {
  hipError_t e;
  if ((e = restart_vectors(v, v.pp[k & 1], st, nullptr))) return e;
  if ((first || restart_p) && (e = launch_copy(v.p, v.cgls ? v.s : v.r, low_half_bytes(v), st))) return e;
  if (first && (e = launch_zero(v.xl, (size_t)v.g.Vh * 96, st))) return e;
  return launch_state_reset(v.state, v.slot, 1, first ? 1 : 0, v.thr, st, k);
}

// The device-driven reliable update closing a mixed-precision chunk: every
// launch is gated on the state's ru_gate, set by the p-update that asked
// for it (which has also folded the inner solution into x).  q = A x in
// FP64, r64 = rhs - q and r = low(r64) in one pass, the restarted |r|^2
// (CG) or s = Mhat^dag r with |s|^2 (CGLS) into both ping-pong buffers (so
// the next iteration finds it whatever the parity of its label; the other
// buffer is rewritten before it is read), then the decision, and p = r
// (CG) or s (CGLS) where the decision restarts the search direction.
static hipError_t reliable_update_block(const SolveVecs& v, int max_ru, int max_iters, hipStream_t st) {
  const int* gate = &v.state->ru_gate;
  hipError_t e;
  if (v.cgls) {
    if ((e = mhat64_gated(v, v.q64, v.x, 0, nullptr, st, gate))) return e;
    if ((e = launch_ru_residual(v.g, v.prec, v.rhs, v.q64, v.r64, v.r, v.red, nullptr, nullptr, v.nbD, gate, st)))
      return e;
    if ((e = restart_vectors(v, v.pp[0], st, gate, false))) return e;
    if ((e = launch_copy_doubles_gated(v.pp[1], v.pp[0], v.nbD, gate, st))) return e;
  } else {
    if ((e = mhat64_gated(v, v.s64, v.x, 0, nullptr, st, gate))) return e;
    if ((e = mhat64_gated(v, v.q64, v.s64, 1, nullptr, st, gate))) return e;
    if ((e = launch_ru_residual(v.g, v.prec, v.rhs, v.q64, v.r64, v.r, v.red, v.pp[0], v.pp[1], v.nbD, gate, st)))
      return e;
  }
  if ((e = launch_ru_finish(v.state, v.red, v.nbD, v.slot, max_ru, max_iters, st))) return e;
  return launch_copy_gated(v.p, v.cgls ? v.s : v.r, low_half_bytes(v), &v.state->restart, st);
}

namespace {

hipError_t read_state(Fields* F, SolverState* out, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(F->pinned + SL_COUNT, F->state, sizeof(SolverState), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  std::memcpy(out, F->pinned + SL_COUNT, sizeof(SolverState));
  return hipSuccess;
}

// What a chunk of a solve launches besides its iterations.
struct ChunkExtra {
  bool ru = false;  // the gated reliable update (mixed precision)
  int max_ru = 0, max_iters = 0;
};

// The launches of one chunk: iterations j = 0..n-1, the label advance and
// (mixed precision) the gated reliable update.
hipError_t chunk_launches(const SolveVecs& v, const IterArgs& args, int n, const ChunkExtra& x, hipStream_t st) {
  for (int j = 0; j < n; ++j) {
    hipError_t e = launch_iteration(v.g, v.prec, v.cgls, nullptr, args, 1, v.nbD, v.nbR, j, st);
    if (e != hipSuccess) return e;
  }
  hipError_t e = launch_advance_base(v.state, n, st);
  if (e != hipSuccess || !x.ru) return e;
  return reliable_update_block(v, x.max_ru, x.max_iters, st);
}

// Which chunks are replayed from recordings.  Measured on MI355X (ROCm
// 7.2), direct launches win everywhere: a replayed launch that exits at
// once (an iteration queued past a stop, an update gate with no request)
// occupies the GPU for several microseconds, more than issued directly, and
// the host issues these launches fast enough once no reliable update waits
// for it (16^3x32 trajectories: FP64 0.1187 direct / 0.1211 replayed; with
// FP32 / FP16 / BF16 force solves 0.1027 / 0.0950 / 0.0867 direct against
// 0.1065 / 0.0990 / 0.0916 replayed).  So chunks launch directly unless
// HMC_SOLVER_GRAPHS asks otherwise: =mixed replays the mixed-precision
// chunks, =all every chunk, =strict every chunk with a failed recording an
// error instead of a fall-back to direct launches (for tests).
enum GraphMode { GRAPHS_NONE = 0, GRAPHS_MIXED = 1, GRAPHS_ALL = 2, GRAPHS_STRICT = 3 };
int graphs_mode() {
  const char* e = std::getenv("HMC_SOLVER_GRAPHS");
  if (!e || e[0] == '0') return GRAPHS_NONE;
  if (std::strcmp(e, "mixed") == 0) return GRAPHS_MIXED;
  if (std::strcmp(e, "all") == 0) return GRAPHS_ALL;
  return std::strcmp(e, "strict") == 0 ? GRAPHS_STRICT : GRAPHS_NONE;
}

// The recorded form of a chunk: everything its launches depend on goes
// into the key (the launch arguments, the buffers of the gated update, the
// launch decisions in force), so a replay issues exactly the launches a
// direct chunk would.
hipError_t recorded_chunk(Fields* F, const SolveVecs& v, const IterArgs& args, int n, const ChunkExtra& x,
                          hipGraphExec_t* out) {
  struct KeyData {
    IterArgs args;
    SolveVecs v;
    int ru, max_ru, max_iters, n;
    uint64_t tune;
  } kd;
  std::memset(&kd, 0, sizeof kd);
  std::memcpy(&kd.args, &args, sizeof args);
  std::memcpy(&kd.v, &v, sizeof v);
  kd.v.thr = 0.0;  // read from the solver state, not recorded
  kd.ru = x.ru ? 1 : 0;
  kd.max_ru = x.max_ru;
  kd.max_iters = x.max_iters;
  kd.n = n;
  kd.tune = tune_generation();
  std::string key(reinterpret_cast<const char*>(&kd), sizeof kd);
  ++F->record_clock;
  for (Fields::Recorded& r : F->recorded)
    if (r.key == key) {
      r.last_use = F->record_clock;
      *out = r.exec;
      return hipSuccess;
    }
  hipError_t e;
  if (!F->record_stream && (e = hipStreamCreateWithFlags(&F->record_stream, hipStreamNonBlocking))) return e;
  if ((e = hipStreamBeginCapture(F->record_stream, hipStreamCaptureModeThreadLocal))) return e;
  timing_set_recording(true);
  hipError_t le = chunk_launches(v, args, n, x, F->record_stream);
  timing_set_recording(false);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(F->record_stream, &graph);
  if (le != hipSuccess || e != hipSuccess) {
    if (graph) hipGraphDestroy(graph);
    return le != hipSuccess ? le : e;
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  if ((int)F->recorded.size() >= kMaxRecorded) {  // drop the least recently used
    auto old = std::min_element(F->recorded.begin(), F->recorded.end(),
                                [](const Fields::Recorded& a, const Fields::Recorded& b) {
                                  return a.last_use < b.last_use;
                                });
    hipGraphExecDestroy(old->exec);
    F->recorded.erase(old);
  }
  F->recorded.push_back(Fields::Recorded{key, exec, F->record_clock});
  *out = exec;
  return hipSuccess;
}

// Launches a chunk of n iterations: replayed from its recording, or
// directly (see graphs_mode).  While the kernel timing samples every m-th
// launch, every m-th chunk that would be replayed runs directly with all
// its launches timed, so the sampled durations are those of the launches a
// replay issues.
// Whether the chunks of this kind are replayed from recordings.
bool chunk_records(const ChunkExtra& x) {
  const int mode = graphs_mode();
  return mode == GRAPHS_ALL || mode == GRAPHS_STRICT || (mode == GRAPHS_MIXED && x.ru);
}

hipError_t launch_chunk(Fields* F, const SolveVecs& v, const IterArgs& args, int n, const ChunkExtra& x,
                        hipStream_t st) {
  static thread_local unsigned counter = 0;
  const int mode = graphs_mode();
  const bool record = chunk_records(x);
  if (!record || (F->record_failed && mode != GRAPHS_STRICT)) return chunk_launches(v, args, n, x, st);
  const int every = timing_sample_every();
  if (every > 0 && counter++ % every == 0) {
    timing_sample_all(true);
    hipError_t e = chunk_launches(v, args, n, x, st);
    timing_sample_all(false);
    return e;
  }
  hipGraphExec_t exec;
  hipError_t e = recorded_chunk(F, v, args, n, x, &exec);
  if (e != hipSuccess) {
    if (mode == GRAPHS_STRICT) return e;
    (void)hipGetLastError();  // a runtime that cannot record these launches: launch them directly from now on
    F->record_failed = true;
    return chunk_launches(v, args, n, x, st);
  }
  timing_count(TK_DSLASH, 4LL * n);
  timing_count(TK_CG_BLAS, (v.cgls ? 2LL : 1LL) * n);
  return hipGraphLaunch(exec, st);
}

// A chunk of enqueued iterations whose solver state is being copied back
// into pinned slot `slot` (completion marked by F->state_ev[slot]).
struct Chunk {
  int k, n, slot;
};

// F64 chunks: lengths taken as sums of powers of two, so at most five
// recordings per solve configuration serve every length.
// A chunk with no reliable update that is not replayed takes its labels
// from the launch arguments instead (c.k + j on a base that stays at its
// reset value 0), which spares the label advance after every chunk.
hipError_t enqueue_chunk(Fields* F, const SolveVecs& v, const IterArgs& args, const Chunk& c, hipStream_t st,
                         const ChunkExtra& x = ChunkExtra{}) {
  if (!x.ru && !chunk_records(x)) {
    for (int j = 0; j < c.n; ++j) {
      hipError_t e = launch_iteration(v.g, v.prec, v.cgls, nullptr, args, 1, v.nbD, v.nbR, c.k + j, st);
      if (e != hipSuccess) return e;
    }
  } else {
    int left = c.n;
    for (int p = kChunk; p >= 1; p >>= 1)
      while (left >= p) {
        hipError_t e = launch_chunk(F, v, args, p, x, st);
        if (e != hipSuccess) return e;
        left -= p;
      }
  }
  static_assert(sizeof(SolverState) <= kStateSlot * sizeof(double), "state slot");
  hipError_t e = hipMemcpyAsync(F->pinned + SL_COUNT + kStateSlot * c.slot, F->state, sizeof(SolverState),
                                hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipEventRecord(F->state_ev[c.slot], st);
}

hipError_t wait_chunk(Fields* F, const Chunk& c, SolverState* out) {
  hipError_t e = hipEventSynchronize(F->state_ev[c.slot]);
  if (e != hipSuccess) return e;
  std::memcpy(out, F->pinned + SL_COUNT + kStateSlot * c.slot, sizeof(SolverState));
  return hipSuccess;
}

// Runs F64 iterations with labels *k.. until the device stops or `limit` is
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

// Mixed precision with the reliable updates on the device: chunks of inner
// iterations, each closed by the gated update, until the device marks the
// solve done (FP64 true residual <= thr, non-finite, or a limit).  The host
// reads the state of one chunk while the next is queued and sizes the chunk
// after it so that it ends at the iteration predicted to ask for the next
// update: the spacing of the last two updates (inner iterations), or before
// two updates the decrease of the inner |r|^2 toward max(thr, delta^2
// maxrr) at the observed rate.  An iteration queued past the request exits
// at once, an update gate that finds no request does nothing; both cost a
// few microseconds of dispatch.  The host stops queueing when the last
// update read implies that the next one ends the solve.  Returns the final
// state in *stt.
hipError_t run_mixed(Fields* F, const SolveVecs& v, const IterArgs& args, int limit, double rr0, double thr,
                     double delta2, SolverState* stt, hipStream_t st) {
  ChunkExtra x;
  x.ru = true;
  x.max_ru = kMaxReliable;
  x.max_iters = limit;
  double rate = std::log(delta2) / 8;  // log |r|^2 per inner iteration (a first guess)
  auto iterations_to = [&](double ratio) {  // inner iterations until |r|^2 falls by `ratio`
    if (!(rate < 0)) return kChunk;
    const double m = std::log(ratio) / rate;
    if (!(m > 1)) return 1;
    return m >= kChunk ? kChunk : (int)std::ceil(m - 1e-9);
  };
  int spacing = 0;  // inner iterations between the last two updates (0: not seen yet)
  int labels = 0;
  Chunk cur{labels, iterations_to(std::max(thr / rr0, delta2)), 0};
  hipError_t e;
  if ((e = enqueue_chunk(F, v, args, cur, st, x))) return e;
  labels += cur.n;
  int queued = iterations_to(delta2);  // length of the next chunk to queue
  bool last_expected = false;
  SolverState prev{};
  prev.maxrr = prev.rr = rr0;
  while (true) {
    Chunk nxt{labels, 0, cur.slot ^ 1};
    if (!last_expected && labels < limit + kChunk) {
      nxt.n = queued;
      if ((e = enqueue_chunk(F, v, args, nxt, st, x))) return e;
      labels += nxt.n;
    }
    if ((e = wait_chunk(F, cur, stt))) return e;
    if (stt->done) return hipSuccess;
    const bool updated = stt->nru > prev.nru;
    if (updated && prev.nru > 0) spacing = stt->ru_iter - prev.ru_iter;
    if (!updated && stt->iters > prev.iters && stt->rr > 0 && prev.rr > 0 && stt->rr < prev.rr)
      rate = std::log(stt->rr / prev.rr) / (stt->iters - prev.iters);
    // inner iterations from the end of `cur` to the next request, and what
    // the chunk already queued (nxt) takes of them
    int per_update = spacing > 0 ? std::min(spacing, kChunk) : iterations_to(delta2);
    int m;
    if (spacing > 0)
      m = std::max(1, stt->ru_iter + spacing - stt->iters);
    else
      m = updated ? iterations_to(std::max(thr / stt->rr64, delta2))
                  : iterations_to(std::max(thr, delta2 * stt->maxrr) / stt->rr);
    if (nxt.n > 0)
      queued = m > nxt.n ? m - nxt.n : per_update;
    else
      queued = m;
    queued = std::max(1, std::min(kChunk, queued));
    if (updated) last_expected = stt->rr64 * delta2 <= thr;
    prev = *stt;
    if (nxt.n > 0) {
      cur = nxt;
      continue;
    }
    if (labels >= limit + kChunk) {
      // no update was asked for within the iteration limit: force one,
      // which ends the solve (max_iters 0: converged or at the limit)
      if ((e = launch_ru_request(v.state, st))) return e;
      if ((e = launch_add_low_to_f64(v.g, v.x, v.xl, st))) return e;
      if ((e = reliable_update_block(v, x.max_ru, 0, st))) return e;
      return read_state(F, stt, st);
    }
    cur = Chunk{labels, queued, cur.slot ^ 1};
    last_expected = false;  // nothing is queued: queue one and look again
    if ((e = enqueue_chunk(F, v, args, cur, st, x))) return e;
    labels += cur.n;
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
  // default delta: FP32 storage tracks the FP64 residual over a hundredfold
  // decrease (fewer updates, measured faster); FP16 / BF16 over tenfold
  const double delta = prm->reliable_delta > 0 ? prm->reliable_delta : prec == HMC_F32 ? 0.01 : 0.1;
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
  v.thr = thr;

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
    CHK(launch_state_reset(v.state, nullptr, 1, 1, thr, st));
    IterArgs args;
    build_iteration(v, 0, 0, 0.0, &args);
    double rate = 0;
    CHK(run_until_stop(F, v, args, &k, limit, &stt, st, rr0, thr, &rate));
    S.iters = stt.iters;
    S.rel_res = std::sqrt(stt.rr / bnorm2);
    if (!std::isfinite(stt.rr)) status = HMC_E_NAN;  // the device stops at a non-finite |r|^2
    else if (fixed == 0 && !(stt.rr <= thr)) status = HMC_E_NOCONV;
  } else {
    IterArgs args;
    build_iteration(v, 0, 1, delta * delta, &args, true);
    args.c[0].max_iters = args.c[1].max_iters = limit;  // the update at the limit ends the solve
    CHK(inner_restart(v, 0, true, st));  // the slot holds |r64|^2 = rr0
    CHK(run_mixed(F, v, args, limit, rr0, thr, delta * delta, &stt, st));
    S.iters = stt.iters;
    S.reliable_updates = stt.nru;
    S.rel_res = std::sqrt(stt.rr64 / bnorm2);
    if (stt.done == 3) status = HMC_E_NAN;
    else if (stt.done != 1) status = HMC_E_NOCONV;
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
