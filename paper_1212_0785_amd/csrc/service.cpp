// Solve service: continuous batching of Wilson solves on one GPU.
//
// Requests enter an inbox (never blocked by GPU work).  Each scheduling
// round (a) admits waiting requests in FIFO order while their footprint fits
// a first-fit allocator over the caller's arena, generates their gauge
// field and source and sets up the solve; (b) advances every volume group
// by a chunk of solver iterations, one launch per solver step covering all
// requests of the group (blockIdx.y = request, per-request kappa, links and
// vectors from a device table); (c) reads the per-request solver states in
// one copy, performs reliable updates / convergence checks, and retires
// finished requests, freeing their memory for the next admissions.  Volume
// groups run on the caller's streams (group slot k on stream k mod n), so
// that different volumes overlap on the device when the caller gives
// several.
//
// A request's arithmetic never reads another request's data and its
// reductions use a grid that depends only on its volume, so the result is
// identical alone and in any mix (the iteration labels differ, but they
// only select ping-pong buffers).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"
#include "solver.h"

namespace hmc {
namespace {

constexpr int kMaxActive = 256;
constexpr int kMaxGroups = 8;
constexpr int kMaxBatch = 256;
constexpr int kMaxReliable = 2000;

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }
size_t half_bytes(int Vh, int prec) {
  return (size_t)Vh * (prec == HMC_F64 ? 192 : prec == HMC_F32 ? 96 : prec == HMC_F16 ? 52 : 48);
}
size_t link_bytes(int prec) { return prec == HMC_F64 ? 144 : prec == HMC_F32 ? 72 : 36; }

struct Carve {
  size_t off = 0;
  char* base;
  explicit Carve(char* b) : base(b) {}
  void* take(size_t bytes) {
    void* p = base ? base + off : nullptr;
    off += a256(bytes);
    return p;
  }
};

// Lays out one request's buffers (base == nullptr: size only).
size_t carve_request(char* base, const LatArg& g, int prec, SolveVecs* v, void** U64, void** b, void** x) {
  Carve c(base);
  const int Vh = g.Vh;
  const size_t h64 = half_bytes(Vh, HMC_F64);
  const int shape = dslash_shape(g, (hmc_prec)prec);
  const int nbD = dslash_shape_blocks(Vh, shape), nbR = blas_blocks(Vh);
  SolveVecs t{};
  SolveVecs& s = v ? *v : t;
  *U64 = c.take((size_t)Vh * 8 * 144);
  s.Ulow = prec == HMC_F64 ? *U64 : c.take((size_t)Vh * 8 * link_bytes(prec));
  *b = c.take(2 * h64);
  *x = c.take(2 * h64);
  s.r64 = c.take(h64);
  s.rhs = c.take(h64);
  s.q64 = c.take(h64);
  s.s64 = c.take(h64);
  s.t64 = c.take(h64);
  if (prec == HMC_F64) {
    s.p = c.take(h64);
    s.r = s.r64, s.q = s.q64, s.s = s.s64, s.t = s.t64;
  } else {
    const size_t hl = half_bytes(Vh, prec);
    s.r = c.take(hl), s.p = c.take(hl), s.q = c.take(hl), s.s = c.take(hl), s.t = c.take(hl);
    s.xl = c.take(half_bytes(Vh, HMC_F32));
  }
  // sized for the largest shape, so the footprint does not depend on tuning
  const size_t np = (size_t)dslash_blocks_max(Vh);
  s.pp[0] = (double*)c.take(np * 8);
  s.pp[1] = (double*)c.take(np * 8);
  s.pq = (double*)c.take(np * 8);
  s.pr = (double*)c.take((size_t)nbR * 8);
  s.red = (double*)c.take((size_t)2 * nbR * 8);
  s.nbD = nbD;
  s.nbR = nbR;
  s.shape = shape;
  s.shape64 = dslash_shape(g, HMC_F64);
  return c.off;
}

enum class Phase { Waiting, Setup, Running, Done };

struct Req {
  uint64_t ticket;
  hmc_solve_request q;
  LatArg g;
  size_t bytes = 0, off = 0;
  int idx = -1;  // state / slot index
  Phase phase = Phase::Waiting;
  SolveVecs v{};
  void* U64 = nullptr;
  void* b = nullptr;
  void* x = nullptr;
  double bnorm2 = 0, thr = 0;
  int iter0 = 0;
  int reliable = 0;
  double last_rr64 = 0;  // FP64 |r|^2 of the previous reliable update
  int max_group = 0;
  bool fresh = true;  // first inner start pending
  hmc_solve_result res{};
};

struct Group {
  LatArg g{};
  std::vector<Req*> members;
  int J = 0;  // label counter
  bool dirty = true;
  int slot = -1;  // table region
  hipStream_t stream = nullptr;
};

bool same_volume(const LatArg& a, const LatArg& b) {
  return a.L[0] == b.L[0] && a.L[1] == b.L[1] && a.L[2] == b.L[2] && a.L[3] == b.L[3];
}

}  // namespace

struct Service {
  hmc_service_params prm{};
  double delta2 = 0.01;  // reliable-update threshold delta^2 of the inner iteration
  int chunk = 16;
  std::chrono::steady_clock::time_point t0;
  // device header
  SolverState* states = nullptr;
  double* slots = nullptr;  // 2 per request index
  char* tables = nullptr;   // kMaxGroups regions
  size_t table_region = 0;
  char* heap = nullptr;
  size_t heap_bytes = 0;
  // host
  SolverState* h_states = nullptr;  // pinned
  double* h_slots = nullptr;        // pinned
  char* h_tables = nullptr;         // pinned staging
  std::map<size_t, size_t> free_list;  // offset -> size
  std::deque<Req*> queue;
  std::vector<std::unique_ptr<Group>> groups;
  bool group_slot_used[kMaxGroups] = {};
  int idx_used[kMaxActive] = {};
  hipStream_t streams[kMaxGroups] = {};  // the caller's, by group slot
  // shared with submitters
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> inbox;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  uint64_t next_ticket = 1;
  int pending = 0;
  bool stop = false;
  std::thread worker;
  std::mutex step_mu;  // one round at a time
  hmc_status fatal = HMC_OK;

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_list.begin(); it != free_list.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        size_t rest = it->second - bytes;
        size_t noff = it->first + bytes;
        free_list.erase(it);
        if (rest) free_list[noff] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_list.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_list.erase(nx);
    }
    if (it != free_list.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_list.erase(it);
      }
    }
  }

  Group* group_for(const LatArg& g) {
    for (auto& gr : groups)
      if (same_volume(gr->g, g)) return gr.get();
    int slot = -1;
    for (int k = 0; k < kMaxGroups; ++k)
      if (!group_slot_used[k]) {
        slot = k;
        break;
      }
    if (slot < 0) return nullptr;
    group_slot_used[slot] = true;
    auto gr = std::make_unique<Group>();
    gr->g = g;
    gr->slot = slot;
    gr->stream = streams[slot];
    groups.push_back(std::move(gr));
    return groups.back().get();
  }

  hipError_t setup(Req* r, Group* gr) {
    hipStream_t st = gr->stream;
    SolveVecs& v = r->v;
    char* base = heap + r->off;
    carve_request(base, r->g, prm.inner_prec, &v, &r->U64, &r->b, &r->x);
    v.g = r->g;
    v.kappa = r->q.kappa;
    v.cgls = 1;
    v.prec = (hmc_prec)prm.inner_prec;
    v.U64 = r->U64;
    v.su3 = 1;  // weak-field links are reunitarised: SU(3) rows
    v.x = r->x;
    if (v.prec == HMC_F64) v.xl = r->x;
    v.state = states + r->idx;
    v.slot = slots + 2 * r->idx + 1;
    const size_t h64 = half_bytes(r->g.Vh, HMC_F64);
    hipError_t e;
    if ((e = launch_weak_field(r->g, r->q.gauge_seed, r->q.gauge_eps, r->U64, st))) return e;
    if (v.prec != HMC_F64 && (e = launch_convert_gauge(r->g, r->U64, (void*)v.Ulow, v.prec, st))) return e;
    char* b = (char*)r->b;
    if ((e = launch_source(r->g, r->q.source_kind, r->q.source_seed, r->q.source_epoch, b, b + h64, st))) return e;
    // |b|^2 into slot 0 of the request
    if ((e = launch_norm2_partials(r->g, HMC_F64, b, v.red, v.nbR, st))) return e;
    if ((e = launch_norm2_partials(r->g, HMC_F64, b + h64, v.red + v.nbR, v.nbR, st))) return e;
    if ((e = launch_finalize(v.red, 2 * v.nbR, 1, slots + 2 * r->idx, 1.0, 0, st))) return e;
    // bhat_e = b_e + kappa D_eo b_o ; x_e = 0 ; r64 = bhat ; |r64|^2 into the solver slot
    DslashArgs d{};
    d.U = r->U64;
    d.su3 = 1;
    d.in = b + h64;
    d.out = v.rhs;
    d.y = b;
    d.a = 1.0;
    d.b = r->q.kappa;
    if ((e = launch_dslash(HMC_F64, 0, EPI_AXPY, r->g, 0, nullptr, 1, d, st, 0))) return e;
    if ((e = launch_cg_init(r->g, HMC_F64, v.rhs, r->x, v.r64, v.prec == HMC_F64 ? v.p : v.q64, v.pp[0], v.nbR, st)))
      return e;
    return launch_finalize(v.pp[0], v.nbR, 1, v.slot, 1.0, 0, st);
  }

  // Start (first) or resume the inner iteration at label k.
  hipError_t start_inner(Req* r, int k, hipStream_t st, bool restart_p = false) {
    SolveVecs& v = r->v;
    hipError_t e;
    if (v.prec == HMC_F64) {
      // s = Mhat^dag r (|s|^2 -> pp[k&1]), p = s
      if ((e = mhat64(v, v.s, v.r, 1, v.pp[k & 1], st))) return e;
      if ((e = launch_copy(v.p, v.s, half_bytes(v.g.Vh, HMC_F64), st))) return e;
      return launch_state_reset(v.state, nullptr, 1, 1, r->thr, st);
    }
    e = inner_restart(v, k, r->fresh, st, restart_p);
    r->fresh = false;
    return e;
  }

  // x_o = b_o + kappa D_oe x_e, FP64 |b - M x|^2 into the solver slot.
  hipError_t finalize_enqueue(Req* r, hipStream_t st) {
    SolveVecs& v = r->v;
    const size_t h64 = half_bytes(v.g.Vh, HMC_F64);
    char* x = (char*)r->x;
    char* b = (char*)r->b;
    hipError_t e;
    DslashArgs d{};
    d.U = r->U64;
    d.su3 = 1;
    d.in = x;
    d.out = x + h64;
    d.y = b + h64;
    d.a = 1.0;
    d.b = v.kappa;
    if ((e = launch_dslash(HMC_F64, 0, EPI_AXPY, v.g, 1, nullptr, 1, d, st, 0))) return e;
    // M x: even into s64, odd into t64
    d.in = x + h64;
    d.out = v.s64;
    d.y = x;
    d.b = -v.kappa;
    if ((e = launch_dslash(HMC_F64, 0, EPI_AXPY, v.g, 0, nullptr, 1, d, st, 0))) return e;
    d.in = x;
    d.out = v.t64;
    d.y = x + h64;
    if ((e = launch_dslash(HMC_F64, 0, EPI_AXPY, v.g, 1, nullptr, 1, d, st, 0))) return e;
    if ((e = launch_xmy_norm(v.g, b, v.s64, v.s64, v.red, v.nbR, st))) return e;
    if ((e = launch_xmy_norm(v.g, b + h64, v.t64, v.t64, v.red + v.nbR, v.nbR, st))) return e;
    if ((e = launch_finalize(v.red, 2 * v.nbR, 1, v.slot, 1.0, 0, st))) return e;
    if (r->q.out) return hipMemcpyAsync(r->q.out, r->x, 2 * h64, hipMemcpyDeviceToDevice, st);
    return hipSuccess;
  }

  void retire(Req* r, Group* gr, int status, double res2) {
    SolverState s = h_states[r->idx];
    r->res.status = status;
    r->res.iters = s.iters;
    r->res.reliable_updates = r->reliable;
    r->res.max_group = r->max_group;
    r->res.true_rel_res = r->bnorm2 > 0 ? std::sqrt(res2 / r->bnorm2) : 0.0;
    r->res.t_done = now();
    release(r->off, r->bytes);
    idx_used[r->idx] = 0;
    auto& m = gr->members;
    m.erase(std::remove(m.begin(), m.end(), r), m.end());
    gr->dirty = true;
    {
      std::lock_guard<std::mutex> lk(mu);
      r->phase = Phase::Done;
      pending--;
    }
    cv_done.notify_all();
  }

  hipError_t upload_tables(Group* gr) {
    const int n = (int)gr->members.size();
    char* hb = h_tables + gr->slot * table_region;
    DslashArgs* hd = (DslashArgs*)hb;
    CgArgs* hc = (CgArgs*)(hb + 4 * kMaxBatch * sizeof(DslashArgs));
    for (int i = 0; i < n; ++i) {
      Req* r = gr->members[i];
      IterArgs a;
      build_iteration(r->v, r->iter0, r->v.prec == HMC_F64 ? 0 : 1, r->v.prec == HMC_F64 ? 0.0 : delta2, &a);
      for (int k = 0; k < 4; ++k) hd[k * kMaxBatch + i] = a.d[k];
      for (int k = 0; k < 2; ++k) hc[k * kMaxBatch + i] = a.c[k];
      r->max_group = std::max(r->max_group, n);
    }
    gr->dirty = false;
    return hipMemcpyAsync(tables + gr->slot * table_region, hb, table_region, hipMemcpyHostToDevice, gr->stream);
  }

  IterTables device_tables(Group* gr) {
    char* db = tables + gr->slot * table_region;
    IterTables t;
    for (int k = 0; k < 4; ++k) t.d[k] = (const DslashArgs*)db + k * kMaxBatch;
    for (int k = 0; k < 2; ++k) t.c[k] = (const CgArgs*)(db + 4 * kMaxBatch * sizeof(DslashArgs)) + k * kMaxBatch;
    return t;
  }

  hipError_t sync_all() {
    for (auto& gr : groups) {
      hipError_t e = hipStreamSynchronize(gr->stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  hipError_t read_states() {
    if (groups.empty()) return hipSuccess;
    hipStream_t st = groups[0]->stream;
    hipError_t e = hipMemcpyAsync(h_states, states, sizeof(SolverState) * kMaxActive, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h_slots, slots, sizeof(double) * 2 * kMaxActive, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
  }

  // One scheduling round.
  hmc_status round() {
    {
      std::lock_guard<std::mutex> lk(mu);
      while (!inbox.empty()) {
        queue.push_back(inbox.front());
        inbox.pop_front();
      }
    }
    // (a) admission, FIFO
    std::vector<std::pair<Req*, Group*>> admitted;
    while (!queue.empty()) {
      Req* r = queue.front();
      int idx = -1;
      for (int k = 0; k < kMaxActive; ++k)
        if (!idx_used[k]) {
          idx = k;
          break;
        }
      if (idx < 0) break;
      Group* gr = group_for(r->g);
      if (!gr || (int)gr->members.size() >= prm.max_batch) break;
      size_t off;
      if (!alloc(r->bytes, &off)) break;
      queue.pop_front();
      idx_used[idx] = 1;
      r->idx = idx;
      r->off = off;
      r->phase = Phase::Setup;
      r->res.t_start = now();
      HMC_CHECK_HIP(setup(r, gr));
      admitted.push_back({r, gr});
    }
    if (!admitted.empty()) {
      HMC_CHECK_HIP(sync_all());
      HMC_CHECK_HIP(read_states());
      for (auto& [r, gr] : admitted) {
        r->bnorm2 = h_slots[2 * r->idx];
        r->thr = prm.tol * prm.tol * r->bnorm2;
        r->v.thr = r->thr;
        double rr0 = h_slots[2 * r->idx + 1];
        gr->members.push_back(r);
        gr->dirty = true;
        r->iter0 = -gr->J;
        r->phase = Phase::Running;
        if (r->bnorm2 == 0.0 || rr0 <= r->thr) {
          r->fresh = false;
          HMC_CHECK_HIP(launch_state_reset(r->v.state, nullptr, 1, 1, r->thr, gr->stream));
          HMC_CHECK_HIP(finalize_enqueue(r, gr->stream));
          r->phase = Phase::Setup;  // finished below without iterating
        } else {
          HMC_CHECK_HIP(start_inner(r, 0, gr->stream));
        }
      }
      // requests that needed no iteration
      bool any = false;
      for (auto& [r, gr] : admitted) any |= r->phase == Phase::Setup;
      if (any) {
        HMC_CHECK_HIP(sync_all());
        HMC_CHECK_HIP(read_states());
        for (auto& [r, gr] : admitted)
          if (r->phase == Phase::Setup) retire(r, gr, HMC_OK, h_slots[2 * r->idx + 1]);
      }
    }
    // (b) advance every group by one chunk
    for (auto& gr : groups) {
      if (gr->members.empty()) continue;
      if (gr->dirty) HMC_CHECK_HIP(upload_tables(gr.get()));
      IterTables t = device_tables(gr.get());
      Req* r0 = gr->members[0];
      IterArgs one;
      build_iteration(r0->v, 0, 0, 0, &one);
      for (int j = 0; j < chunk; ++j)
        HMC_CHECK_HIP(launch_iteration(gr->g, (hmc_prec)prm.inner_prec, 1, &t, one, (int)gr->members.size(),
                                       r0->v.nbD, r0->v.nbR, gr->J + j, gr->stream));
      gr->J += chunk;
    }
    HMC_CHECK_HIP(sync_all());
    HMC_CHECK_HIP(read_states());
    // (c) stops: reliable updates / convergence
    std::vector<std::pair<Req*, Group*>> stopped;
    for (auto& gr : groups)
      for (Req* r : gr->members) {
        const SolverState& s = h_states[r->idx];
        if (s.stop_at != INT_MAX || s.iters >= prm.maxiter) stopped.push_back({r, gr.get()});
      }
    if (stopped.empty()) return HMC_OK;
    for (auto& [r, gr] : stopped) {
      if (r->v.prec == HMC_F64)
        HMC_CHECK_HIP(true_residual(r->v, gr->stream));
      else
        HMC_CHECK_HIP(reliable_update(r->v, gr->stream));
    }
    HMC_CHECK_HIP(sync_all());
    HMC_CHECK_HIP(read_states());
    std::vector<std::pair<Req*, Group*>> finishing;
    std::vector<int> fstatus;
    for (auto& [r, gr] : stopped) {
      const double rr64 = h_slots[2 * r->idx + 1];
      const SolverState& s = h_states[r->idx];
      if (r->v.prec != HMC_F64) r->reliable++;
      // FP64 stops on the recursive residual (as the single solve does);
      // mixed precision on the FP64 true residual of the reliable update
      const bool conv = r->v.prec == HMC_F64 ? s.reason == 1 : rr64 <= r->thr;
      const bool dead = !conv && (r->v.prec == HMC_F64 || !(rr64 == rr64) || s.iters >= prm.maxiter ||
                                  r->reliable >= kMaxReliable);
      if (conv || dead) {
        finishing.push_back({r, gr});
        fstatus.push_back(conv ? HMC_OK : HMC_E_NOCONV);
        HMC_CHECK_HIP(finalize_enqueue(r, gr->stream));
      } else {
        // the search direction restarts as in the single solve's device-driven
        // update: the recursion lost track of the FP64 residual, or a cycle
        // made no progress
        const bool restart_p = rr64 > 2.0 * s.rr || (r->reliable > 1 && rr64 >= r->last_rr64);
        r->last_rr64 = rr64;
        HMC_CHECK_HIP(start_inner(r, gr->J + r->iter0, gr->stream, restart_p));
      }
    }
    if (!finishing.empty()) {
      HMC_CHECK_HIP(sync_all());
      HMC_CHECK_HIP(read_states());
      for (size_t i = 0; i < finishing.size(); ++i)
        retire(finishing[i].first, finishing[i].second, fstatus[i], h_slots[2 * finishing[i].first->idx + 1]);
    }
    return HMC_OK;
  }

  // Drops empty groups so their table slot and stream can serve a new volume.
  void drop_empty_groups() {
    for (auto it = groups.begin(); it != groups.end();) {
      if ((*it)->members.empty()) {
        group_slot_used[(*it)->slot] = false;
        it = groups.erase(it);
      } else {
        ++it;
      }
    }
  }

  hmc_status step(int* pending_out) {
    std::lock_guard<std::mutex> lk(step_mu);
    hmc_status s = fatal ? fatal : round();
    drop_empty_groups();
    if (s != HMC_OK) fatal = s;
    if (pending_out) {
      std::lock_guard<std::mutex> l2(mu);
      *pending_out = pending;
    }
    return s;
  }

  void loop() {
    while (true) {
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || pending > 0; });
        if (stop) return;
      }
      if (step(nullptr) != HMC_OK) {
        std::lock_guard<std::mutex> lk(mu);
        cv_done.notify_all();
        return;
      }
    }
  }
};

}  // namespace hmc

using namespace hmc;

extern "C" {

hmc_status hmc_request_bytes(const hmc_solve_request* req, int32_t inner_prec, size_t* bytes) {
  HMC_REQUIRE(req && bytes, "null argument");
  HMC_REQUIRE(inner_prec >= HMC_F64 && inner_prec <= HMC_BF16, "bad precision");
  LatArg g;
  long long V = 1;
  for (int k = 0; k < 4; ++k) {
    HMC_REQUIRE(req->L[k] >= 2 && req->L[k] % 2 == 0, "lattice extent L[%d] = %d must be even and >= 2", k,
                req->L[k]);
    g.L[k] = req->L[k];
    V *= req->L[k];
  }
  HMC_REQUIRE(V / 2 < (1LL << 31) / 12, "lattice too large");
  g.Vh = (int)(V / 2);
  g.stride = g.Vh;
  void *u, *b, *x;
  *bytes = carve_request(nullptr, g, inner_prec, nullptr, &u, &b, &x);
  return HMC_OK;
}

hmc_status hmc_service_create(const hmc_service_params* p, hmc_service** out) {
  HMC_REQUIRE(p && out && p->arena, "null argument");
  HMC_REQUIRE(((uintptr_t)p->arena & 255) == 0, "arena must be 256-byte aligned");
  HMC_REQUIRE(p->max_batch >= 1 && p->max_batch <= kMaxBatch, "max_batch must be in [1, %d]", kMaxBatch);
  HMC_REQUIRE(p->inner_prec >= HMC_F64 && p->inner_prec <= HMC_BF16, "bad precision");
  HMC_REQUIRE(p->tol > 0 && p->maxiter >= 1, "bad tolerance or maxiter");
  HMC_REQUIRE(p->n_streams >= 1 && p->n_streams <= HMC_SERVICE_MAX_STREAMS, "n_streams must be in [1, %d]",
              HMC_SERVICE_MAX_STREAMS);
  static_assert(kMaxGroups == HMC_SERVICE_MAX_STREAMS, "one stream slot per volume group");
  auto S = std::make_unique<Service>();
  S->prm = *p;
  S->chunk = p->chunk > 0 ? p->chunk : 16;
  // the single solve's default delta (0.01 for FP32 storage, 0.1 for FP16 / BF16)
  const double delta = p->reliable_delta > 0 ? p->reliable_delta : p->inner_prec == HMC_F32 ? 0.01 : 0.1;
  S->delta2 = delta * delta;
  S->t0 = std::chrono::steady_clock::now();
  S->table_region = a256(4 * kMaxBatch * sizeof(DslashArgs) + 2 * kMaxBatch * sizeof(CgArgs));
  Carve c((char*)p->arena);
  S->states = (SolverState*)c.take(sizeof(SolverState) * kMaxActive);
  S->slots = (double*)c.take(sizeof(double) * 2 * kMaxActive);
  S->tables = (char*)c.take(S->table_region * kMaxGroups);
  if (c.off >= p->arena_bytes) {
    set_error("arena of %zu bytes cannot hold the service header (%zu bytes)", p->arena_bytes, c.off);
    return HMC_E_OOM;
  }
  S->heap = (char*)p->arena + c.off;
  S->heap_bytes = p->arena_bytes - c.off;
  S->free_list[0] = S->heap_bytes;
  if (hipHostMalloc((void**)&S->h_states, sizeof(SolverState) * kMaxActive) != hipSuccess ||
      hipHostMalloc((void**)&S->h_slots, sizeof(double) * 2 * kMaxActive) != hipSuccess ||
      hipHostMalloc((void**)&S->h_tables, S->table_region * kMaxGroups) != hipSuccess) {
    set_error("hipHostMalloc of the service staging buffers failed");
    return HMC_E_HIP;
  }
  for (int k = 0; k < kMaxGroups; ++k) S->streams[k] = (hipStream_t)p->streams[k % p->n_streams];
  Service* raw = S.release();
  if (!p->manual) raw->worker = std::thread([raw] { raw->loop(); });
  *out = reinterpret_cast<hmc_service*>(raw);
  return HMC_OK;
}

hmc_status hmc_service_submit(hmc_service* svc, const hmc_solve_request* req, uint64_t* ticket) {
  HMC_REQUIRE(svc && req && ticket, "null argument");
  Service* S = reinterpret_cast<Service*>(svc);
  const double t = S->now();
  size_t bytes;
  hmc_status st = hmc_request_bytes(req, S->prm.inner_prec, &bytes);
  if (st) return st;
  HMC_REQUIRE(req->kappa > 0 && req->kappa < 0.25, "kappa %g out of range", req->kappa);
  HMC_REQUIRE(req->source_kind >= 0 && req->source_kind <= 2, "bad source kind");
  if (bytes > S->heap_bytes) {
    set_error("request needs %zu bytes; the arena heap has %zu", bytes, S->heap_bytes);
    return HMC_E_OOM;
  }
  auto r = std::make_unique<Req>();
  r->q = *req;
  for (int k = 0; k < 4; ++k) r->g.L[k] = req->L[k];
  long long V = (long long)req->L[0] * req->L[1] * req->L[2] * req->L[3];
  r->g.Vh = (int)(V / 2);
  r->g.stride = r->g.Vh;
  r->bytes = bytes;
  r->res.t_submit = t;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->inbox.push_back(r.get());
    S->reqs[r->ticket] = std::move(r);
    S->pending++;
  }
  S->cv_work.notify_one();
  return HMC_OK;
}

hmc_status hmc_service_poll(hmc_service* svc, uint64_t ticket, hmc_solve_result* res) {
  HMC_REQUIRE(svc, "null service");
  Service* S = reinterpret_cast<Service*>(svc);
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  HMC_REQUIRE(it != S->reqs.end(), "unknown ticket %llu", (unsigned long long)ticket);
  if (S->fatal) {
    set_error("service stopped after a device error");
    return S->fatal;
  }
  if (it->second->phase != Phase::Done) return HMC_E_BUSY;
  if (res) *res = it->second->res;
  return it->second->res.status;
}

hmc_status hmc_service_step(hmc_service* svc, int32_t* pending) {
  HMC_REQUIRE(svc, "null service");
  Service* S = reinterpret_cast<Service*>(svc);
  HMC_REQUIRE(S->prm.manual, "hmc_service_step needs manual mode");
  int p = 0;
  hmc_status s = S->step(&p);
  if (pending) *pending = p;
  return s;
}

hmc_status hmc_service_wait(hmc_service* svc, uint64_t ticket, hmc_solve_result* res) {
  HMC_REQUIRE(svc, "null service");
  Service* S = reinterpret_cast<Service*>(svc);
  while (true) {
    hmc_status s = hmc_service_poll(svc, ticket, res);
    if (s != HMC_E_BUSY) return s;
    if (S->prm.manual) {
      hmc_status e = S->step(nullptr);
      if (e != HMC_OK) return e;
    } else {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_done.wait_for(lk, std::chrono::milliseconds(50));
    }
  }
}

hmc_status hmc_service_destroy(hmc_service* svc) {
  HMC_REQUIRE(svc, "null service");
  Service* S = reinterpret_cast<Service*>(svc);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (int k = 0; k < kMaxGroups && k < S->prm.n_streams; ++k) (void)hipStreamSynchronize(S->streams[k]);
  if (S->h_states) (void)hipHostFree(S->h_states);
  if (S->h_slots) (void)hipHostFree(S->h_slots);
  if (S->h_tables) (void)hipHostFree(S->h_tables);
  delete S;
  return HMC_OK;
}

}  // extern "C"
