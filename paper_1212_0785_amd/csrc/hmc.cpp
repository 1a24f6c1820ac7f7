// C-ABI entry points of libhmc: fields objects in caller-owned arenas,
// layout conversion, the Dslash / Mhat / M operators, global sums, forces,
// the link update, refresh, the leapfrog integrator and the HMC trajectory
// (the HMC step list of the paper's Sec. 1, run entirely on the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <complex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fields.h"

namespace hmc {

// ------------------------------------------------------------ errors

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}
const char* last_error() { return g_err.c_str(); }

// ------------------------------------------------------------ timing

namespace {
struct TimingRec {
  int kernel;
  int pair;
  double bytes;  // algorithmic
  double moved;  // as implemented
  int launches;  // launches the pair brackets (a group shares one pair)
};
struct Timing {
  std::mutex mu;
  int sample_every = 0;
  std::vector<hipEvent_t> events;  // 2 per pair
  std::vector<TimingRec> recs;
  long long counter[TK_COUNT] = {};
  long long launches[TK_COUNT] = {};
  long long calls[TK_COUNT] = {};  // every launch while enabled
  double ms[TK_COUNT] = {};
  double bytes[TK_COUNT] = {};
  double moved[TK_COUNT] = {};
  int open_pair = -1;
  // open group: family, launches still to come, its record (-1: unsampled)
  int group_kernel = -1, group_left = 0, group_rec = -1;
};
Timing& timing() {
  static Timing t;
  return t;
}
constexpr int kMaxPairs = 8192;
// Launches recorded into a graph on this thread take no timing events;
// while t_every is set, every launch of this thread is sampled.
thread_local bool t_recording = false;
thread_local bool t_every = false;
}  // namespace

void timing_set_recording(bool on) { t_recording = on; }
void timing_sample_all(bool on) { t_every = on; }
int timing_sample_every() { return timing().sample_every; }

void timing_count(int kernel, long long n) {
  Timing& T = timing();
  if (T.sample_every <= 0 || n <= 0) return;
  std::lock_guard<std::mutex> lk(T.mu);
  T.calls[kernel] += n;
}

bool timing_enabled() { return timing().sample_every > 0; }

const char* timed_kernel_name(int k) {
  static const char* names[TK_COUNT] = {"dslash", "cg_blas", "reduce", "gauge_force", "fermion_force",
                                        "exp_update", "refresh", "plaquette", "other"};
  return (k >= 0 && k < TK_COUNT) ? names[k] : "?";
}

bool timing_begin(int kernel, hipStream_t st, double bytes, double moved) {
  Timing& T = timing();
  if (T.sample_every <= 0 || t_recording) return false;
  std::lock_guard<std::mutex> lk(T.mu);
  ++T.calls[kernel];
  if (T.counter[kernel]++ % T.sample_every && !t_every) return false;
  int pair = (int)T.recs.size();
  if (pair >= kMaxPairs) return false;
  while ((int)T.events.size() < 2 * (pair + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return false;
    T.events.push_back(e);
  }
  if (hipEventRecord(T.events[2 * pair], st) != hipSuccess) return false;
  T.recs.push_back({kernel, pair, bytes, moved < 0 ? bytes : moved, 1});
  T.open_pair = pair;
  return true;
}

// A free event pair for a new record, or -1 (pool exhausted / HIP error).
static int new_pair(Timing& T) {
  const int pair = (int)T.recs.size();
  if (pair >= kMaxPairs) return -1;
  while ((int)T.events.size() < 2 * (pair + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    T.events.push_back(e);
  }
  return pair;
}

KernelEvents timing_kernel_events(int kernel, double bytes, double moved) {
  KernelEvents ev;
  if (moved < 0) moved = bytes;
  Timing& T = timing();
  if (T.sample_every <= 0 || t_recording) return ev;
  std::lock_guard<std::mutex> lk(T.mu);
  ++T.calls[kernel];
  if (T.group_left > 0 && T.group_kernel == kernel) {  // inside a group
    const bool first = T.group_rec == -2, last = T.group_left == 1;
    --T.group_left;
    if (first) {  // the group's sampling decision, on its first launch
      T.group_rec = -1;
      if (T.counter[kernel]++ % T.sample_every == 0 || t_every) {
        const int pair = new_pair(T);
        if (pair >= 0) {
          T.recs.push_back({kernel, pair, 0.0, 0.0, 0});
          T.group_rec = (int)T.recs.size() - 1;
          ev.start = T.events[2 * pair];
        }
      }
    }
    if (T.group_rec >= 0) {
      TimingRec& r = T.recs[T.group_rec];
      r.bytes += bytes;
      r.moved += moved;
      r.launches += 1;
      if (last) ev.stop = T.events[2 * r.pair + 1];
    }
    if (last) T.group_kernel = -1;
    return ev;
  }
  if (T.counter[kernel]++ % T.sample_every && !t_every) return ev;
  const int pair = new_pair(T);
  if (pair < 0) return ev;
  T.recs.push_back({kernel, pair, bytes, moved, 1});
  ev.start = T.events[2 * pair];
  ev.stop = T.events[2 * pair + 1];
  return ev;
}

void timing_group_end() {
  Timing& T = timing();
  std::lock_guard<std::mutex> lk(T.mu);
  // an unfinished group (a launch failed) has no stop event: drop its record
  if (T.group_left > 0 && T.group_rec >= 0 && T.group_rec == (int)T.recs.size() - 1) T.recs.pop_back();
  T.group_kernel = -1;
  T.group_left = 0;
  T.group_rec = -1;
}

void timing_group_begin(int kernel, int n) {
  Timing& T = timing();
  std::lock_guard<std::mutex> lk(T.mu);
  if (T.sample_every <= 0 || n <= 0 || t_recording) return;
  T.group_kernel = kernel;
  T.group_left = n;
  T.group_rec = -2;  // decided on the first launch
}

void timing_end(int kernel, hipStream_t st) {
  (void)kernel;
  Timing& T = timing();
  std::lock_guard<std::mutex> lk(T.mu);
  if (T.open_pair >= 0) hipEventRecord(T.events[2 * T.open_pair + 1], st);
  T.open_pair = -1;
}

// --------------------------------------------------------- geometry

static hmc_status check_geom(const hmc_geom* geom, LatArg* g, long long* V) {
  HMC_REQUIRE(geom, "null geometry");
  long long v = 1;
  for (int k = 0; k < 4; ++k) {
    int L = geom->L[k];
    HMC_REQUIRE(L >= 2 && L % 2 == 0, "lattice extent L[%d] = %d must be even and >= 2", k, L);
    v *= L;
  }
  HMC_REQUIRE(v / 2 < (1LL << 31) / 12, "lattice too large for 32-bit component indexing");
  for (int k = 0; k < 4; ++k) g->L[k] = geom->L[k];
  g->Vh = (int)(v / 2);
  g->stride = g->Vh;
  *V = v;
  return HMC_OK;
}

static size_t half_bytes(int Vh, hmc_prec p) {
  switch (p) {
    case HMC_F64: return (size_t)Vh * 192;
    case HMC_F32: return (size_t)Vh * 96;
    case HMC_F16: return (size_t)Vh * 52;
    case HMC_BF16: return (size_t)Vh * 48;
  }
  return 0;
}
static size_t gauge_bytes(int Vh, hmc_prec p) {
  switch (p) {
    case HMC_F64: return (size_t)Vh * 8 * 144;
    case HMC_F32: return (size_t)Vh * 8 * 72;
    case HMC_F16:
    case HMC_BF16: return (size_t)Vh * 8 * 36;
  }
  return 0;
}
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Arena plan; with base == nullptr only the size is computed.
static size_t plan_fields(Fields* F, char* base, const LatArg& g, uint32_t flags) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const int Vh = g.Vh;
  const size_t h64 = half_bytes(Vh, HMC_F64);
  const int nbD = dslash_blocks(g, HMC_F64), nbR = blas_blocks(Vh);
  const int npart = 2 * std::max(dslash_blocks_max(Vh), nbR);
  const int nb_multi = std::min(nbR, 1024);
  const size_t multi = (size_t)nb_multi * 2 * 1024 + 1024;
  Fields tmp;
  Fields* f = F ? F : &tmp;
  f->half64 = h64;
  f->halflow = half_bytes(Vh, HMC_F32);
  f->nbD = nbD;
  f->nbR = nbR;
  f->npart = npart;
  f->multi_doubles = multi;
  f->U = take(gauge_bytes(Vh, HMC_F64));
  f->U_old = take(gauge_bytes(Vh, HMC_F64));
  f->P = (double*)take((size_t)Vh * 8 * 8 * 8);
  f->eta = take(h64);
  f->phi = take(h64);
  f->Xe = take(h64);
  f->Xo = take(h64);
  f->Ye = take(h64);
  f->Yo = take(h64);
  f->eta2 = take(h64);
  f->phi2 = take(h64);
  f->chi = take(h64);
  f->X2 = take(h64);
  for (int k = 0; k < Fields::kChronoMax; ++k) f->hist[k] = take(h64);
  f->n_hist = 0;
  f->r = take(h64);
  f->p = take(h64);
  f->q = take(h64);
  f->s = take(h64);
  f->t = take(h64);
  f->bhat = take(h64);
  f->tmp = take(2 * h64);
  for (int k = 0; k < kNumPart; ++k) f->part[k] = (double*)take((size_t)npart * 8);
  f->multi = (double*)take(multi * 8);
  f->state = (SolverState*)take(sizeof(SolverState) * 4);
  f->slots = (double*)take(SL_COUNT * 8);
  for (int k = 0; k < 4; ++k) f->Ulow[k] = nullptr;
  f->lr = f->lp = f->lq = f->ls = f->lt = f->lx = nullptr;
  if (flags & HMC_FIELDS_LOWPREC) {
    f->Ulow[HMC_F32] = take(gauge_bytes(Vh, HMC_F32));
    f->Ulow[HMC_F16] = take(gauge_bytes(Vh, HMC_F16));
    f->Ulow[HMC_BF16] = take(gauge_bytes(Vh, HMC_BF16));
    const size_t hl = f->halflow;
    f->lr = take(hl);
    f->lp = take(hl);
    f->lq = take(hl);
    f->ls = take(hl);
    f->lt = take(hl);
    f->lx = take(half_bytes(Vh, HMC_F32));
  }
  return off;
}

hipError_t read_slots(Fields* F, int first, int n, double* out, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(F->pinned, F->slots + first, n * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  for (int k = 0; k < n; ++k) out[k] = F->pinned[k];
  return hipSuccess;
}

hipError_t dslash_f64(Fields* F, void* out, const void* in, int out_par, int dag, int epi, const void* y, double a,
                      double b, double* partial, const int* stop_at, int iter, hipStream_t st) {
  DslashArgs d{};
  d.U = F->U;
  d.in = in;
  d.out = out;
  d.y = y;
  d.a = a;
  d.b = b;
  d.partial = partial;
  d.stop_at = stop_at;
  d.iter0 = iter;
  d.su3 = F->su3;
  return launch_dslash(HMC_F64, dag, epi, F->g, out_par, nullptr, 1, d, st);
}

void* low_links(Fields* F, hmc_prec prec) { return (prec == HMC_F64) ? F->U : F->Ulow[prec]; }

hipError_t ensure_lowprec(Fields* F, hmc_prec prec, hipStream_t st) {
  if (prec == HMC_F64) return hipSuccess;
  if (!F->Ulow[prec]) return hipErrorInvalidValue;
  if (F->low_version[prec] == F->u_version) return hipSuccess;
  hipError_t e = launch_convert_gauge(F->g, F->U, F->Ulow[prec], prec, st);
  if (e == hipSuccess) F->low_version[prec] = F->u_version;
  return e;
}

// Largest |stored - rebuilt| third-row component for which the two-row
// loads are taken to reproduce the link (links have entries of modulus <= 1).
constexpr double kSu3Tol = 1e-14;

hipError_t check_su3(Fields* F, hipStream_t st) {
  hipError_t e = launch_su3_check(F->g, F->U, kSu3Tol, F->part[4], F->nbR, st);
  if (e != hipSuccess) return e;
  if ((e = launch_finalize(F->part[4], F->nbR, 1, F->slots + SL_RED, 1.0, 0, st))) return e;
  double bad = -1;
  if ((e = read_slots(F, SL_RED, 1, &bad, st))) return e;
  F->su3 = bad == 0.0;
  return hipSuccess;
}

// Mhat (dag) on F64 half spinors: out = in - kappa^2 D_eo D_oe in.
hipError_t mhat_f64(Fields* F, void* out, const void* in, int dag, double* partial, hipStream_t st) {
  hipError_t e = dslash_f64(F, F->t, in, 1, dag, EPI_PLAIN, nullptr, 0, 1, nullptr, nullptr, 0, st);
  if (e != hipSuccess) return e;
  return dslash_f64(F, out, F->t, 0, dag, partial ? EPI_AXPY_NORM : EPI_AXPY, in, 1.0, -F->kappa * F->kappa, partial,
                    nullptr, 0, st);
}

static hipError_t finalize_to_slot(Fields* F, const double* part, int n, int nvals, int slot, hipStream_t st) {
  return launch_finalize(part, n, nvals, F->slots + slot, 1.0, 0, st);
}

// Sum over x, mu < nu of Re Tr U_mu nu(x) into a slot (partials in part[0]).
static hipError_t plaquette_to_slot(Fields* F, int slot, hipStream_t st) {
  hipError_t e = launch_plaquette_partials(F->g, F->U, F->part[0], st, F->su3);
  if (e != hipSuccess) return e;
  return finalize_to_slot(F, F->part[0], plaquette_blocks(F->g, F->su3), 1, slot, st);
}

}  // namespace hmc

using namespace hmc;

// Partial sums of hmc_norm2_static: a file-scope device array, one copy per
// GPU, held until the process ends.  In host code `scratch` names a
// host-side stand-in, never the device array: kernels receive the address
// hipGetSymbolAddress returns, looked up once per device on the first call.
// Every partial is written before the final sum reads it, so the array
// needs no clearing between calls.
constexpr int kStaticPartials = 4096;  // two halves x the largest BLAS grid
static __device__ __align__(256) double scratch[kStaticPartials];

namespace hmc {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
hmc_status static_partials(double** out) {
  int dev = -1;
  HMC_CHECK_HIP(hipGetDevice(&dev));
  HMC_REQUIRE(dev >= 0 && dev < kMaxDevices, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HMC_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    HMC_REQUIRE(p != nullptr, "no device address for the static partial-sum array");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return HMC_OK;
}
}  // namespace
}  // namespace hmc

#define ST(s) reinterpret_cast<hipStream_t>(s)
#define FIELDS(f)                                 \
  HMC_REQUIRE((f) != nullptr, "null fields");     \
  Fields* F = as_fields(f);

extern "C" {

const char* hmc_last_error(void) { return last_error(); }

hmc_status hmc_get_version(int32_t* major, int32_t* minor) {
  HMC_REQUIRE(major && minor, "null output");
  *major = 1;
  *minor = 0;
  return HMC_OK;
}

hmc_status hmc_field_bytes(const hmc_geom* geom, hmc_prec prec, hmc_kind kind, size_t* bytes) {
  LatArg g;
  long long V;
  hmc_status s = check_geom(geom, &g, &V);
  if (s) return s;
  HMC_REQUIRE(bytes, "null output");
  HMC_REQUIRE(prec >= HMC_F64 && prec <= HMC_BF16, "bad precision %d", (int)prec);
  switch (kind) {
    case HMC_KIND_HALF_SPINOR: *bytes = half_bytes(g.Vh, prec); break;
    case HMC_KIND_FULL_SPINOR: *bytes = 2 * half_bytes(g.Vh, prec); break;
    case HMC_KIND_GAUGE: *bytes = gauge_bytes(g.Vh, prec); break;
    case HMC_KIND_MOMENTA:
      HMC_REQUIRE(prec == HMC_F64, "momenta are stored in F64 only");
      *bytes = (size_t)g.Vh * 8 * 8 * 8;
      break;
    default: HMC_REQUIRE(false, "bad field kind %d", (int)kind);
  }
  return HMC_OK;
}

hmc_status hmc_fields_bytes(const hmc_geom* geom, uint32_t flags, size_t* bytes) {
  LatArg g;
  long long V;
  hmc_status s = check_geom(geom, &g, &V);
  if (s) return s;
  HMC_REQUIRE(bytes, "null output");
  *bytes = plan_fields(nullptr, nullptr, g, flags);
  return HMC_OK;
}

hmc_status hmc_alloc_fields(const hmc_geom* geom, const hmc_action* action, uint32_t flags, void* arena,
                            size_t arena_bytes, hmc_fields** out) {
  LatArg g;
  long long V;
  hmc_status s = check_geom(geom, &g, &V);
  if (s) return s;
  HMC_REQUIRE(action && arena && out, "null argument");
  HMC_REQUIRE(((uintptr_t)arena & 255) == 0, "arena must be 256-byte aligned");
  size_t need = plan_fields(nullptr, nullptr, g, flags);
  if (arena_bytes < need) {
    set_error("arena of %zu bytes is smaller than the %zu bytes needed", arena_bytes, need);
    return HMC_E_OOM;
  }
  Fields* F = new Fields();
  F->g = g;
  F->V = V;
  F->beta = action->beta;
  F->kappa = action->kappa;
  F->flags = flags;
  F->arena = (char*)arena;
  F->arena_bytes = arena_bytes;
  plan_fields(F, (char*)arena, g, flags);
  F->u_version = 1;
  for (int k = 0; k < 4; ++k) F->low_version[k] = 0;
  F->su3 = F->su3_old = false;  // U holds whatever the arena held
  F->state_ev[0] = F->state_ev[1] = nullptr;
  if (hipEventCreateWithFlags(&F->state_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&F->state_ev[1], hipEventDisableTiming) != hipSuccess) {
    for (hipEvent_t e : F->state_ev)
      if (e) hipEventDestroy(e);
    delete F;
    set_error("hipEventCreate failed");
    return HMC_E_HIP;
  }
  if (hipHostMalloc((void**)&F->pinned, (SL_COUNT + 64) * sizeof(double)) != hipSuccess) {
    for (hipEvent_t e : F->state_ev) hipEventDestroy(e);
    delete F;
    set_error("hipHostMalloc of the scalar read-back buffer failed");
    return HMC_E_HIP;
  }
  *out = reinterpret_cast<hmc_fields*>(F);
  return HMC_OK;
}

hmc_status hmc_free_fields(hmc_fields* f) {
  FIELDS(f);
  for (Fields::Recorded& r : F->recorded) hipGraphExecDestroy(r.exec);
  if (F->record_stream) hipStreamDestroy(F->record_stream);
  if (F->pinned) hipHostFree(F->pinned);
  for (hipEvent_t e : F->state_ev)
    if (e) hipEventDestroy(e);
  delete F;
  return HMC_OK;
}

hmc_status hmc_set_action(hmc_fields* f, const hmc_action* action) {
  FIELDS(f);
  HMC_REQUIRE(action, "null action");
  F->beta = action->beta;
  F->kappa = action->kappa;
  return HMC_OK;
}

hmc_status hmc_field_pointer(hmc_fields* f, hmc_field_id which, void** ptr) {
  FIELDS(f);
  HMC_REQUIRE(ptr, "null output");
  switch (which) {
    case HMC_FIELD_GAUGE:  // the caller may write U: full-link loads until hmc_sync_lowprec
      *ptr = F->U;
      F->su3 = false;
      break;
    case HMC_FIELD_MOMENTA: *ptr = F->P; break;
    case HMC_FIELD_ETA: *ptr = F->eta; break;
    case HMC_FIELD_PHI: *ptr = F->phi; break;
    case HMC_FIELD_XE: *ptr = F->Xe; break;
    default: HMC_REQUIRE(false, "bad field id %d", (int)which);
  }
  return HMC_OK;
}

hmc_status hmc_links_two_row(hmc_fields* f, int32_t* on) {
  FIELDS(f);
  HMC_REQUIRE(on, "null output");
  *on = (F->su3 && dslash_link_form(F->g, HMC_F64) != LINK_FULL) ? 1 : 0;
  return HMC_OK;
}

hmc_status hmc_import_gauge(hmc_fields* f, const void* canon, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(canon, "null buffer");
  HMC_CHECK_HIP(launch_pack_gauge(F->g, canon, F->U, ST(stream)));
  F->u_version++;
  HMC_CHECK_HIP(check_su3(F, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_export_gauge(hmc_fields* f, void* canon, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(canon, "null buffer");
  HMC_CHECK_HIP(launch_unpack_gauge(F->g, F->U, canon, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_import_momenta(hmc_fields* f, const void* canon, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(canon, "null buffer");
  HMC_CHECK_HIP(launch_pack_momenta(F->g, canon, F->P, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_export_momenta(hmc_fields* f, void* canon, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(canon, "null buffer");
  HMC_CHECK_HIP(launch_unpack_momenta(F->g, F->P, canon, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_import_spinor(hmc_fields* f, void* dst, const void* canon, int32_t parity, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(dst && canon, "null buffer");
  HMC_REQUIRE(parity >= -1 && parity <= 1, "parity must be -1, 0 or 1");
  HMC_CHECK_HIP(launch_pack_spinor(F->g, canon, dst, parity, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_export_spinor(hmc_fields* f, void* canon, const void* src, int32_t parity, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(src && canon, "null buffer");
  HMC_REQUIRE(parity >= -1 && parity <= 1, "parity must be -1, 0 or 1");
  HMC_CHECK_HIP(launch_unpack_spinor(F->g, src, canon, parity, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_convert_spinor(hmc_fields* f, void* dst, hmc_prec dst_prec, const void* src, hmc_prec src_prec,
                              void* stream) {
  FIELDS(f);
  HMC_REQUIRE(dst && src, "null buffer");
  HMC_REQUIRE(dst_prec >= HMC_F64 && dst_prec <= HMC_BF16 && src_prec >= HMC_F64 && src_prec <= HMC_BF16,
              "bad precision");
  HMC_CHECK_HIP(launch_convert_spinor(F->g, src, src_prec, dst, dst_prec, 1, nullptr, nullptr, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_sync_lowprec(hmc_fields* f, void* stream) {
  FIELDS(f);
  F->u_version++;
  HMC_CHECK_HIP(check_su3(F, ST(stream)));
  if (F->flags & HMC_FIELDS_LOWPREC)
    for (int p = HMC_F32; p <= HMC_BF16; ++p) HMC_CHECK_HIP(ensure_lowprec(F, (hmc_prec)p, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_wilson_dslash(hmc_fields* f, void* out, const void* in, int32_t out_parity, int32_t dagger,
                             hmc_prec prec, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(out && in, "null buffer");
  HMC_REQUIRE(out != in, "out and in must not alias");
  HMC_REQUIRE(out_parity == 0 || out_parity == 1, "out_parity must be 0 or 1");
  HMC_REQUIRE(prec >= HMC_F64 && prec <= HMC_BF16, "bad precision");
  HMC_REQUIRE(prec == HMC_F64 || (F->flags & HMC_FIELDS_LOWPREC), "low precision needs HMC_FIELDS_LOWPREC");
  HMC_CHECK_HIP(ensure_lowprec(F, prec, ST(stream)));
  DslashArgs d{};
  d.U = low_links(F, prec);
  d.su3 = F->su3;
  d.in = in;
  d.out = out;
  d.b = 1.0;
  HMC_CHECK_HIP(launch_dslash(prec, dagger ? 1 : 0, EPI_PLAIN, F->g, out_parity, nullptr, 1, d, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_mhat(hmc_fields* f, void* out, const void* in, int32_t dagger, hmc_prec prec, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(out && in, "null buffer");
  HMC_REQUIRE(out != in, "out and in must not alias");
  HMC_REQUIRE(prec >= HMC_F64 && prec <= HMC_BF16, "bad precision");
  HMC_REQUIRE(prec == HMC_F64 || (F->flags & HMC_FIELDS_LOWPREC), "low precision needs HMC_FIELDS_LOWPREC");
  hipStream_t st = ST(stream);
  if (prec == HMC_F64) {
    HMC_CHECK_HIP(mhat_f64(F, out, in, dagger ? 1 : 0, nullptr, st));
    return HMC_OK;
  }
  HMC_CHECK_HIP(ensure_lowprec(F, prec, st));
  DslashArgs d{};
  d.U = low_links(F, prec);
  d.su3 = F->su3;
  d.in = in;
  d.out = F->lt;
  d.b = 1.0;
  HMC_CHECK_HIP(launch_dslash(prec, dagger ? 1 : 0, EPI_PLAIN, F->g, 1, nullptr, 1, d, st));
  d.in = F->lt;
  d.out = out;
  d.y = in;
  d.a = 1.0;
  d.b = -F->kappa * F->kappa;
  HMC_CHECK_HIP(launch_dslash(prec, dagger ? 1 : 0, EPI_AXPY, F->g, 0, nullptr, 1, d, st));
  return HMC_OK;
}

hmc_status hmc_wilson_m(hmc_fields* f, void* out, const void* in, int32_t dagger, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(out && in, "null buffer");
  HMC_REQUIRE(out != in, "out and in must not alias");
  hipStream_t st = ST(stream);
  const char* ie = (const char*)in;
  char* oe = (char*)out;
  const int dag = dagger ? 1 : 0;
  // out_e = in_e - kappa D_eo in_o ; out_o = in_o - kappa D_oe in_e
  HMC_CHECK_HIP(dslash_f64(F, oe, ie + F->half64, 0, dag, EPI_AXPY, ie, 1.0, -F->kappa, nullptr, nullptr, 0, st));
  HMC_CHECK_HIP(dslash_f64(F, oe + F->half64, ie, 1, dag, EPI_AXPY, ie + F->half64, 1.0, -F->kappa, nullptr, nullptr,
                           0, st));
  return HMC_OK;
}

hmc_status hmc_norm2(hmc_fields* f, const void* x, int32_t nhalves, hmc_prec prec, double* out, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(x && out, "null argument");
  HMC_REQUIRE(nhalves == 1 || nhalves == 2, "nhalves must be 1 or 2");
  HMC_REQUIRE(prec >= HMC_F64 && prec <= HMC_BF16, "bad precision");
  hipStream_t st = ST(stream);
  const int nb = F->nbR;
  size_t hb = half_bytes(F->g.Vh, prec);
  for (int h = 0; h < nhalves; ++h)
    HMC_CHECK_HIP(launch_norm2_partials(F->g, prec, (const char*)x + h * hb, F->part[0] + h * nb, nb, st));
  HMC_CHECK_HIP(finalize_to_slot(F, F->part[0], nb * nhalves, 1, SL_RED, st));
  HMC_CHECK_HIP(read_slots(F, SL_RED, 1, out, st));
  return HMC_OK;
}

hmc_status hmc_norm2_static(const hmc_geom* geom, const void* x, int32_t nhalves, hmc_prec prec, double* out_dev,
                            void* stream) {
  LatArg g;
  long long V;
  hmc_status s = check_geom(geom, &g, &V);
  if (s) return s;
  HMC_REQUIRE(x && out_dev, "null argument");
  HMC_REQUIRE(nhalves == 1 || nhalves == 2, "nhalves must be 1 or 2");
  HMC_REQUIRE(prec >= HMC_F64 && prec <= HMC_BF16, "bad precision");
  const int nb = blas_blocks(g.Vh);
  HMC_REQUIRE(nb * nhalves <= kStaticPartials, "%d partial sums exceed the static array of %d", nb * nhalves,
              kStaticPartials);
  double* part = nullptr;
  if ((s = static_partials(&part))) return s;
  hipStream_t st = ST(stream);
  const size_t hb = half_bytes(g.Vh, prec);
  for (int h = 0; h < nhalves; ++h)
    HMC_CHECK_HIP(launch_norm2_partials(g, prec, (const char*)x + h * hb, part + h * nb, nb, st));
  HMC_CHECK_HIP(launch_finalize(part, nb * nhalves, 1, out_dev, 1.0, 0, st));
  return HMC_OK;
}

hmc_status hmc_inner(hmc_fields* f, const void* a, const void* b, int32_t nhalves, double* out, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(a && b && out, "null argument");
  HMC_REQUIRE(nhalves == 1 || nhalves == 2, "nhalves must be 1 or 2");
  hipStream_t st = ST(stream);
  const int nb = F->nbR;
  // partial layout per half: [re: nb][im: nb]; rearranged by two finalisations
  for (int h = 0; h < nhalves; ++h)
    HMC_CHECK_HIP(launch_inner_partials(F->g, (const char*)a + h * F->half64, (const char*)b + h * F->half64,
                                        F->part[1 + h], nb, st));
  double res[2] = {0, 0};
  for (int h = 0; h < nhalves; ++h) {
    HMC_CHECK_HIP(launch_finalize(F->part[1 + h], nb, 2, F->slots + SL_RED, 1.0, h > 0, st));
  }
  HMC_CHECK_HIP(read_slots(F, SL_RED, 2, res, st));
  out[0] = res[0];
  out[1] = res[1];
  return HMC_OK;
}

hmc_status hmc_sum_multi(hmc_fields* f, const void* x, int32_t nhalves, const int32_t* subset, int32_t nsub,
                         double* out, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(x && subset && out, "null argument");
  HMC_REQUIRE(nhalves == 1 || nhalves == 2, "nhalves must be 1 or 2");
  HMC_REQUIRE(nsub >= 1 && nsub <= 1024, "nsub must be in [1, 1024]");
  hipStream_t st = ST(stream);
  const int nb = std::min(F->nbR, 1024);
  std::vector<double> host(nsub);
  // rows of partials first, the nsub results in the last 1024 doubles
  double* res = F->multi + F->multi_doubles - 1024;
  HMC_CHECK_HIP(launch_sum_multi(F->g, x, nhalves, subset, nsub, F->multi, nb, res, st));
  HMC_CHECK_HIP(hipMemcpyAsync(host.data(), res, nsub * sizeof(double), hipMemcpyDeviceToHost, st));
  HMC_CHECK_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < nsub; ++k) out[k] = host[k];
  return HMC_OK;
}

hmc_status hmc_plaquette(hmc_fields* f, double* out, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(out, "null output");
  hipStream_t st = ST(stream);
  double sum;
  HMC_CHECK_HIP(plaquette_to_slot(F, SL_RED, st));
  HMC_CHECK_HIP(read_slots(F, SL_RED, 1, &sum, st));
  *out = sum / (18.0 * F->V);
  return HMC_OK;
}

hmc_status hmc_gauge_action(hmc_fields* f, double* out, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(out, "null output");
  hipStream_t st = ST(stream);
  double sum;
  HMC_CHECK_HIP(plaquette_to_slot(F, SL_RED, st));
  HMC_CHECK_HIP(read_slots(F, SL_RED, 1, &sum, st));
  *out = F->beta * (6.0 * F->V - sum / 3.0);
  return HMC_OK;
}

hmc_status hmc_kinetic_energy(hmc_fields* f, double* out, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(out, "null output");
  hipStream_t st = ST(stream);
  HMC_CHECK_HIP(launch_kinetic_partials(F->g, F->P, F->part[0], F->nbR, st));
  HMC_CHECK_HIP(finalize_to_slot(F, F->part[0], F->nbR, 1, SL_RED, st));
  HMC_CHECK_HIP(read_slots(F, SL_RED, 1, out, st));
  return HMC_OK;
}

hmc_status hmc_gauge_force(hmc_fields* f, double coef, void* stream) {
  FIELDS(f);
  HMC_CHECK_HIP(launch_gauge_force(F->g, F->U, F->P, coef * F->beta, ST(stream), F->su3));
  return HMC_OK;
}

static hipError_t fermion_force_impl(Fields* F, const void* Xe, double coef, hipStream_t st) {
  const double k2 = F->kappa * F->kappa;
  hipError_t e;
  // X_o = D_oe X_e ; Y_e = X_e - kappa^2 D_eo X_o ; Y_o = (D^dag)_oe Y_e
  if ((e = dslash_f64(F, F->Xo, Xe, 1, 0, EPI_PLAIN, nullptr, 0, 1, nullptr, nullptr, 0, st))) return e;
  if ((e = dslash_f64(F, F->Ye, F->Xo, 0, 0, EPI_AXPY, Xe, 1.0, -k2, nullptr, nullptr, 0, st))) return e;
  if ((e = dslash_f64(F, F->Yo, F->Ye, 1, 1, EPI_PLAIN, nullptr, 0, 1, nullptr, nullptr, 0, st))) return e;
  return launch_fermion_force(F->g, F->U, Xe, F->Xo, F->Ye, F->Yo, F->P, coef * k2, st, F->su3);
}

hmc_status hmc_fermion_force(hmc_fields* f, const void* X_e, double coef, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(X_e, "null X_e");
  HMC_CHECK_HIP(fermion_force_impl(F, X_e, coef, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_exp_update_reunit(hmc_fields* f, double eps, void* stream) {
  FIELDS(f);
  HMC_CHECK_HIP(launch_exp_update(F->g, F->U, F->P, eps, ST(stream), F->su3));
  F->u_version++;
  F->su3 = true;  // third row rebuilt by the reunitarisation
  return HMC_OK;
}

static hipError_t refresh_pf(Fields* F, uint64_t seed, uint64_t traj, hipStream_t st) {
  hipError_t e;
  if ((e = launch_eta(F->g, seed, traj, 0, F->eta, st))) return e;
  return mhat_f64(F, F->phi, F->eta, 1, nullptr, st);
}

hmc_status hmc_refresh(hmc_fields* f, uint64_t seed, uint64_t traj, uint32_t what, void* stream) {
  FIELDS(f);
  HMC_REQUIRE((what & ~(HMC_REFRESH_MOM | HMC_REFRESH_PF)) == 0 && what, "bad refresh flags");
  hipStream_t st = ST(stream);
  if (what & HMC_REFRESH_MOM) HMC_CHECK_HIP(launch_refresh_momenta(F->g, seed, traj, F->P, st));
  if (what & HMC_REFRESH_PF) HMC_CHECK_HIP(refresh_pf(F, seed, traj, st));
  return HMC_OK;
}

hmc_status hmc_weak_field_start(hmc_fields* f, uint64_t seed, double eps, void* stream) {
  FIELDS(f);
  HMC_CHECK_HIP(launch_weak_field(F->g, seed, eps, F->U, ST(stream)));
  F->u_version++;
  F->su3 = true;
  return HMC_OK;
}

hmc_status hmc_make_source(hmc_fields* f, void* b, int32_t kind, uint64_t seed, uint64_t epoch, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(b, "null buffer");
  HMC_REQUIRE(kind >= 0 && kind <= 2, "bad source kind %d", kind);
  HMC_CHECK_HIP(launch_source(F->g, kind, seed, epoch, b, (char*)b + F->half64, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_random_words(uint64_t seed, uint64_t rng_stream, uint64_t epoch, const int64_t* sites,
                            int32_t nsites, int32_t nblocks, uint64_t* out, void* stream) {
  HMC_REQUIRE(sites && out, "null buffer");
  HMC_REQUIRE(nsites >= 0 && nblocks >= 1 && nblocks <= 64, "bad sizes");
  if (nsites == 0) return HMC_OK;
  HMC_CHECK_HIP(launch_site_words(seed, rng_stream, epoch, (const long long*)sites, nsites, nblocks, out, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_random_gaussians(uint64_t seed, uint64_t rng_stream, uint64_t epoch, const int64_t* sites,
                                int32_t nsites, int32_t n, double* out, void* stream) {
  HMC_REQUIRE(sites && out, "null buffer");
  HMC_REQUIRE(nsites >= 0 && n >= 2 && n <= 32 && n % 4 == 0, "n must be a multiple of 4 in [4, 32]");
  if (nsites == 0) return HMC_OK;
  HMC_CHECK_HIP(launch_site_gaussians(seed, rng_stream, epoch, (const long long*)sites, nsites, n, out, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_cg_solve(hmc_fields* f, void* x, const void* b, const hmc_cg_params* params, hmc_cg_stats* stats,
                        void* stream) {
  FIELDS(f);
  HMC_REQUIRE(x && b && params, "null argument");
  return cg_solve_impl(F, x, b, params, stats, ST(stream));
}

// One force evaluation: P -= coef (F_g + F_f) with the fermion force from a
// fresh solve of phi_e into X_e.
// Chronological guess into x: the Galerkin projection of A x = phi onto the
// span of the stored solutions F->hist[0..n_hist) (Brower, Ivanenko, Levi,
// Orginos, Nucl. Phys. B 484 (1997) 353).  G_jk = <y_j, A y_k>, f_j =
// <y_j, phi>, G c = f by Gaussian elimination with partial pivoting on the
// host, x = sum_k c_k y_k.  *ok is false (x untouched) when G is singular.
static hmc_status chrono_guess(Fields* F, const void* phi, void* x, bool* ok, hipStream_t st) {
  const int m = F->n_hist, nb = F->nbR;
  *ok = false;
  if (m < 1) return HMC_OK;
  for (int k = 0; k < m; ++k) {
    HMC_CHECK_HIP(mhat_f64(F, F->s, F->hist[k], 0, nullptr, st));
    HMC_CHECK_HIP(mhat_f64(F, F->q, F->s, 1, nullptr, st));
    for (int j = 0; j < m; ++j) {
      HMC_CHECK_HIP(launch_inner_partials(F->g, F->hist[j], F->q, F->part[1], nb, st));
      HMC_CHECK_HIP(finalize_to_slot(F, F->part[1], nb, 2, SL_CHRONO + 2 * (j * m + k), st));
    }
  }
  for (int j = 0; j < m; ++j) {
    HMC_CHECK_HIP(launch_inner_partials(F->g, F->hist[j], phi, F->part[1], nb, st));
    HMC_CHECK_HIP(finalize_to_slot(F, F->part[1], nb, 2, SL_CHRONO + 2 * (m * m + j), st));
  }
  double v[2 * (Fields::kChronoMax * Fields::kChronoMax + Fields::kChronoMax)];
  HMC_CHECK_HIP(read_slots(F, SL_CHRONO, 2 * (m * m + m), v, st));
  using C = std::complex<double>;
  C G[Fields::kChronoMax][Fields::kChronoMax], f[Fields::kChronoMax], c[Fields::kChronoMax];
  for (int j = 0; j < m; ++j) {
    for (int k = 0; k < m; ++k) G[j][k] = C(v[2 * (j * m + k)], v[2 * (j * m + k) + 1]);
    f[j] = C(v[2 * (m * m + j)], v[2 * (m * m + j) + 1]);
  }
  for (int col = 0; col < m; ++col) {
    int piv = col;
    for (int r = col + 1; r < m; ++r)
      if (std::abs(G[r][col]) > std::abs(G[piv][col])) piv = r;
    if (!(std::abs(G[piv][col]) > 0)) return HMC_OK;
    if (piv != col) {
      for (int k = 0; k < m; ++k) std::swap(G[col][k], G[piv][k]);
      std::swap(f[col], f[piv]);
    }
    for (int r = col + 1; r < m; ++r) {
      const C l = G[r][col] / G[col][col];
      for (int k = col; k < m; ++k) G[r][k] -= l * G[col][k];
      f[r] -= l * f[col];
    }
  }
  for (int r = m - 1; r >= 0; --r) {
    C s = f[r];
    for (int k = r + 1; k < m; ++k) s -= G[r][k] * c[k];
    c[r] = s / G[r][r];
  }
  double cc[2 * Fields::kChronoMax];
  for (int k = 0; k < m; ++k) {
    if (!std::isfinite(c[k].real()) || !std::isfinite(c[k].imag())) return HMC_OK;
    cc[2 * k] = c[k].real();
    cc[2 * k + 1] = c[k].imag();
  }
  HMC_CHECK_HIP(launch_lincomb(F->g, F->hist, cc, m, x, st));
  *ok = true;
  return HMC_OK;
}

// Appends the solution x to the history (the oldest drops out at n_chrono).
static hmc_status chrono_push(Fields* F, const void* x, int n_chrono, hipStream_t st) {
  if (F->n_hist == n_chrono) {
    void* oldest = F->hist[0];
    for (int k = 1; k < n_chrono; ++k) F->hist[k - 1] = F->hist[k];
    F->hist[n_chrono - 1] = oldest;
    --F->n_hist;
  }
  HMC_CHECK_HIP(launch_copy(F->hist[F->n_hist], x, F->half64, st));
  ++F->n_hist;
  return HMC_OK;
}

static hmc_status force_kick(Fields* F, double coef, const hmc_cg_params* cg, hmc_md_stats* ms, hipStream_t st,
                             int n_chrono = 0) {
  HMC_CHECK_HIP(launch_gauge_force(F->g, F->U, F->P, coef * F->beta, st, F->su3));
  hmc_cg_params p = *cg;
  p.mode = HMC_CG_NORMAL_MHAT;
  p.initial_guess = 0;
  if (n_chrono > 0) {
    bool ok = false;
    hmc_status g = chrono_guess(F, F->phi, F->Xe, &ok, st);
    if (g) return g;
    p.initial_guess = ok ? 1 : 0;
  }
  hmc_cg_stats cs;
  hmc_status s = cg_solve_impl(F, F->Xe, F->phi, &p, &cs, st);
  if (s != HMC_OK && s != HMC_E_NOCONV && s != HMC_E_NAN) return s;
  const hmc_status solved = s;
  if (n_chrono > 0 && (s = chrono_push(F, F->Xe, n_chrono, st))) return s;
  ms->solves++;
  ms->iters_total += cs.iters;
  ms->iters_max = std::max(ms->iters_max, cs.iters);
  if (solved != HMC_OK) ms->nonconverged++;
  if (solved == HMC_E_NAN) ms->nonfinite++;
  HMC_CHECK_HIP(fermion_force_impl(F, F->Xe, coef, st));
  return HMC_OK;
}

static hmc_status leapfrog_impl(Fields* F, double tau, int nsteps, const hmc_cg_params* cg, hmc_md_stats* ms,
                                hipStream_t st, int n_chrono = 0) {
  const double eps = tau / nsteps;
  *ms = hmc_md_stats{};
  F->n_hist = 0;
  hmc_status s = force_kick(F, 0.5 * eps, cg, ms, st, n_chrono);
  if (s) return s;
  for (int k = 1; k <= nsteps; ++k) {
    HMC_CHECK_HIP(launch_exp_update(F->g, F->U, F->P, eps, st, F->su3));
    F->u_version++;
    F->su3 = true;
    s = force_kick(F, k < nsteps ? eps : 0.5 * eps, cg, ms, st, n_chrono);
    if (s) return s;
  }
  return HMC_OK;
}

hmc_status hmc_md_leapfrog(hmc_fields* f, double tau, int32_t nsteps, const hmc_cg_params* cg, hmc_md_stats* stats,
                           void* stream) {
  FIELDS(f);
  HMC_REQUIRE(cg && stats, "null argument");
  HMC_REQUIRE(nsteps >= 1, "nsteps must be >= 1");
  hipStream_t st = ST(stream);
  hmc_status s = leapfrog_impl(F, tau, nsteps, cg, stats, st);
  if (s) return s;
  HMC_CHECK_HIP(hipStreamSynchronize(st));
  if (stats->nonfinite) {
    set_error("%d of %d solves met a non-finite residual", stats->nonfinite, stats->solves);
    return HMC_E_NAN;
  }
  if (stats->nonconverged) {
    set_error("%d of %d solves did not converge", stats->nonconverged, stats->solves);
    return HMC_E_NOCONV;
  }
  return HMC_OK;
}

hmc_status hmc_trajectory(hmc_fields* f, uint64_t seed, uint64_t traj, const hmc_traj_params* params,
                          hmc_traj_result* res, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(params && res, "null argument");
  HMC_REQUIRE(params->nsteps >= 1, "nsteps must be >= 1");
  HMC_REQUIRE(params->n_chrono >= 0 && params->n_chrono <= Fields::kChronoMax, "n_chrono must be in 0..%d",
              Fields::kChronoMax);
  hipStream_t st = ST(stream);
  auto t0 = std::chrono::steady_clock::now();
  const size_t ub = gauge_bytes(F->g.Vh, HMC_F64);
  HMC_CHECK_HIP(launch_copy(F->U_old, F->U, ub, st));
  F->su3_old = F->su3;
  HMC_CHECK_HIP(launch_refresh_momenta(F->g, seed, traj, F->P, st));
  HMC_CHECK_HIP(refresh_pf(F, seed, traj, st));
  const int nb = F->nbR;
  HMC_CHECK_HIP(launch_kinetic_partials(F->g, F->P, F->part[0], nb, st));
  HMC_CHECK_HIP(finalize_to_slot(F, F->part[0], nb, 1, SL_KE_OLD, st));
  HMC_CHECK_HIP(plaquette_to_slot(F, SL_PLAQ_OLD, st));
  HMC_CHECK_HIP(launch_norm2_partials(F->g, HMC_F64, F->eta, F->part[0], nb, st));
  HMC_CHECK_HIP(finalize_to_slot(F, F->part[0], nb, 1, SL_ETA2, st));

  hmc_md_stats ms;
  hmc_status s = leapfrog_impl(F, params->tau, params->nsteps, &params->cg, &ms, st, params->n_chrono);
  if (s) return s;

  HMC_CHECK_HIP(launch_kinetic_partials(F->g, F->P, F->part[0], nb, st));
  HMC_CHECK_HIP(finalize_to_slot(F, F->part[0], nb, 1, SL_KE_NEW, st));
  HMC_CHECK_HIP(plaquette_to_slot(F, SL_PLAQ_NEW, st));
  HMC_CHECK_HIP(launch_inner_partials(F->g, F->phi, F->Xe, F->part[1], nb, st));
  HMC_CHECK_HIP(finalize_to_slot(F, F->part[1], nb, 2, SL_PHIX, st));
  HMC_CHECK_HIP(launch_metropolis(seed, traj, F->beta, (double)F->V, F->slots, st));
  double sl[13];
  HMC_CHECK_HIP(read_slots(F, 0, 13, sl, st));

  const bool finite = std::isfinite(sl[SL_DH]) && ms.nonfinite == 0;
  bool accepted = sl[SL_ACC] != 0.0 && ms.nonconverged == 0 && finite;
  if (!accepted) {
    HMC_CHECK_HIP(launch_copy(F->U, F->U_old, ub, st));
    F->u_version++;
    F->su3 = F->su3_old;
  }
  double plaq_sum;
  HMC_CHECK_HIP(plaquette_to_slot(F, SL_RED, st));
  HMC_CHECK_HIP(read_slots(F, SL_RED, 1, &plaq_sum, st));

  res->KE_old = sl[SL_KE_OLD];
  res->KE_new = sl[SL_KE_NEW];
  res->S_f_old = sl[SL_ETA2];
  res->S_g_old = sl[SL_SG_OLD];
  res->S_g_new = sl[SL_SG_NEW];
  res->H_old = sl[SL_H_OLD];
  res->H_new = sl[SL_H_NEW];
  res->dH = sl[SL_DH];
  res->u = sl[SL_U];
  res->S_f_new = sl[SL_PHIX];
  res->accepted = accepted ? 1 : 0;
  res->plaquette = plaq_sum / (18.0 * F->V);
  res->cg_iters_total = ms.iters_total;
  res->cg_iters_max = ms.iters_max;
  res->nonconverged = ms.nonconverged;
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  // a non-finite energy change (or solve) explains any non-convergence it caused
  if (!finite) {
    set_error("non-finite energy change (%d of %d solves non-finite); trajectory rejected", ms.nonfinite, ms.solves);
    return HMC_E_NAN;
  }
  if (ms.nonconverged) {
    set_error("%d of %d solves did not converge; trajectory rejected", ms.nonconverged, ms.solves);
    return HMC_E_NOCONV;
  }
  return HMC_OK;
}

hmc_status hmc_timing_enable(int32_t sample_every) {
  Timing& T = timing();
  std::lock_guard<std::mutex> lk(T.mu);
  T.sample_every = sample_every > 0 ? sample_every : 0;
  return HMC_OK;
}

hmc_status hmc_timing_reset(void) {
  Timing& T = timing();
  std::lock_guard<std::mutex> lk(T.mu);
  T.recs.clear();
  T.open_pair = -1;
  for (int k = 0; k < TK_COUNT; ++k) {
    T.counter[k] = 0;
    T.launches[k] = 0;
    T.calls[k] = 0;
    T.ms[k] = 0;
    T.bytes[k] = 0;
    T.moved[k] = 0;
  }
  return HMC_OK;
}

hmc_status hmc_timing_probe(int32_t n, void* stream) {
  HMC_REQUIRE(n >= 0, "n = %d < 0", n);
  for (int i = 0; i < n; ++i) HMC_CHECK_HIP(launch_empty_timed(ST(stream)));
  return HMC_OK;
}

hmc_status hmc_timing_read(hmc_timing_entry* out, int32_t max_entries, int32_t* n_entries) {
  HMC_REQUIRE(n_entries, "null output");
  Timing& T = timing();
  std::lock_guard<std::mutex> lk(T.mu);
  for (const TimingRec& r : T.recs) {
    hipEvent_t a = T.events[2 * r.pair], b = T.events[2 * r.pair + 1];
    HMC_CHECK_HIP(hipEventSynchronize(b));
    float ms = 0;
    HMC_CHECK_HIP(hipEventElapsedTime(&ms, a, b));
    T.launches[r.kernel] += r.launches;
    T.ms[r.kernel] += ms;
    T.bytes[r.kernel] += r.bytes;
    T.moved[r.kernel] += r.moved;
  }
  T.recs.clear();
  int n = 0;
  for (int k = 0; k < TK_COUNT; ++k) {
    if (!T.launches[k] && !T.calls[k]) continue;
    if (out && n < max_entries) {
      std::snprintf(out[n].name, sizeof out[n].name, "%s", timed_kernel_name(k));
      out[n].launches = T.launches[k];
      out[n].total_ms = T.ms[k];
      out[n].bytes = T.bytes[k];
      out[n].calls = T.calls[k];
      out[n].bytes_moved = T.moved[k];
    }
    ++n;
  }
  *n_entries = n;
  return HMC_OK;
}

}  // extern "C"

// ------------------------------------------------ mass preconditioning

namespace hmc {
namespace {

// out = Mhat(kappa_c) in (dag: Mhat^dag) on F64 half spinors (uses F->t).
hipError_t mhat_k(Fields* F, void* out, const void* in, int dag, double kappa_c, hipStream_t st) {
  hipError_t e = dslash_f64(F, F->t, in, 1, dag, EPI_PLAIN, nullptr, 0, 1, nullptr, nullptr, 0, st);
  if (e != hipSuccess) return e;
  return dslash_f64(F, out, F->t, 0, dag, EPI_AXPY, in, 1.0, -kappa_c * kappa_c, nullptr, nullptr, 0, st);
}

// P -= coef F for the bilinear of X = (X_e, D_oe X_e), Y = (Y_e, D^dag_oe Y_e)
// at kappa_c (F->Xo / F->Yo are the odd halves; Y_e is read in place).
hipError_t force_bilinear(Fields* F, const void* Xe, const void* Ye, double kappa_c, double coef, hipStream_t st) {
  hipError_t e;
  if ((e = dslash_f64(F, F->Xo, Xe, 1, 0, EPI_PLAIN, nullptr, 0, 1, nullptr, nullptr, 0, st))) return e;
  if ((e = dslash_f64(F, F->Yo, Ye, 1, 1, EPI_PLAIN, nullptr, 0, 1, nullptr, nullptr, 0, st))) return e;
  return launch_fermion_force(F->g, F->U, Xe, F->Xo, Ye, F->Yo, F->P, coef * kappa_c * kappa_c, st, F->su3);
}

// x = (Mhat^dag Mhat)^-1 b at kappa_c.
hmc_status solve_at(Fields* F, double kappa_c, void* x, const void* b, const hmc_cg_params* cg, int* iters,
                    int* nonconv, int* nonfinite, hipStream_t st) {
  hmc_cg_params p = *cg;
  p.mode = HMC_CG_NORMAL_MHAT;
  p.initial_guess = 0;
  hmc_cg_stats cs{};
  const double k0 = F->kappa;
  F->kappa = kappa_c;
  hmc_status s = cg_solve_impl(F, x, b, &p, &cs, st);
  F->kappa = k0;
  if (s != HMC_OK && s != HMC_E_NOCONV && s != HMC_E_NAN) return s;
  *iters += cs.iters;
  if (s != HMC_OK) ++*nonconv;
  if (s == HMC_E_NAN) ++*nonfinite;
  return HMC_OK;
}

// Nested leapfrog, flattened: per stretch between two link updates the
// summed kick of each level (ratio, heavy, gauge) and the update's eps.
struct Stretch {
  double coef[3];
  double eps;
};

void mts_emit_level(const int* steps, int level, double t, std::vector<Stretch>* out, double* pend) {
  const int n = steps[level];
  const double e = t / n;
  pend[level] += 0.5 * e;
  for (int k = 1; k <= n; ++k) {
    if (level == 2) {
      Stretch s;
      for (int l = 0; l < 3; ++l) s.coef[l] = pend[l], pend[l] = 0;
      s.eps = e;
      out->push_back(s);
    } else {
      mts_emit_level(steps, level + 1, e, out, pend);
    }
    pend[level] += k < n ? e : 0.5 * e;
  }
}

std::vector<Stretch> mts_schedule(int n_ratio, int n_heavy, int n_gauge, double tau) {
  const int steps[3] = {n_ratio, n_heavy, n_gauge};
  std::vector<Stretch> out;
  double pend[3] = {0, 0, 0};
  mts_emit_level(steps, 0, tau, &out, pend);
  Stretch last;
  for (int l = 0; l < 3; ++l) last.coef[l] = pend[l];
  last.eps = 0;
  out.push_back(last);
  return out;
}

hmc_status mts_integrate(Fields* F, const hmc_mts_params* p, hmc_mts_stats* ms, hipStream_t st) {
  const double k = F->kappa, kh = p->kappa_h;
  int nc = 0, nf = 0;
  for (const Stretch& s : mts_schedule(p->n_ratio, p->n_heavy, p->n_gauge, p->tau)) {
    if (s.coef[0] != 0) {  // ratio: chi = Mhat_h^dag phi_2, X_2 = A^-1 chi
      HMC_CHECK_HIP(mhat_k(F, F->chi, F->phi2, 1, kh, st));
      hmc_status r = solve_at(F, k, F->X2, F->chi, &p->cg, &ms->iters_ratio, &nc, &nf, st);
      if (r) return r;
      ms->solves_ratio++;
      HMC_CHECK_HIP(mhat_k(F, F->Ye, F->X2, 0, k, st));
      HMC_CHECK_HIP(force_bilinear(F, F->X2, F->Ye, k, s.coef[0], st));
      HMC_CHECK_HIP(force_bilinear(F, F->X2, F->phi2, kh, -s.coef[0], st));
    }
    if (s.coef[1] != 0) {  // heavy: X_1 = A_h^-1 phi_1
      hmc_status r = solve_at(F, kh, F->Xe, F->phi, &p->cg, &ms->iters_heavy, &nc, &nf, st);
      if (r) return r;
      ms->solves_heavy++;
      HMC_CHECK_HIP(mhat_k(F, F->Ye, F->Xe, 0, kh, st));
      HMC_CHECK_HIP(force_bilinear(F, F->Xe, F->Ye, kh, s.coef[1], st));
    }
    if (s.coef[2] != 0) {
      HMC_CHECK_HIP(launch_gauge_force(F->g, F->U, F->P, s.coef[2] * F->beta, st, F->su3));
      ms->gauge_forces++;
    }
    if (s.eps != 0) {
      HMC_CHECK_HIP(launch_exp_update(F->g, F->U, F->P, s.eps, st, F->su3));
      F->u_version++;
      F->su3 = true;
      ms->link_updates++;
    }
  }
  ms->nonconverged = nc;
  ms->nonfinite = nf;
  return HMC_OK;
}

hmc_status check_mts(const Fields* F, const hmc_mts_params* p) {
  HMC_REQUIRE(p, "null parameters");
  HMC_REQUIRE(p->n_ratio >= 1 && p->n_heavy >= 1 && p->n_gauge >= 1, "step counts must be >= 1");
  HMC_REQUIRE((long long)p->n_ratio * p->n_heavy * p->n_gauge <= 1000000, "too many link updates");
  HMC_REQUIRE(p->kappa_h > 0 && p->kappa_h <= F->kappa, "need 0 < kappa_h <= kappa");
  HMC_REQUIRE(p->cg.prec == HMC_F64 || (F->flags & HMC_FIELDS_LOWPREC), "mixed precision needs HMC_FIELDS_LOWPREC");
  return HMC_OK;
}

}  // namespace
}  // namespace hmc

using namespace hmc;

hmc_status hmc_fermion_force_bilinear(hmc_fields* f, const void* X_e, const void* Y_e, double kappa_c, double coef,
                                      void* stream) {
  FIELDS(f);
  HMC_REQUIRE(X_e && Y_e, "null buffer");
  HMC_CHECK_HIP(force_bilinear(F, X_e, Y_e, kappa_c, coef, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_md_mts(hmc_fields* f, const void* phi2, const hmc_mts_params* p, hmc_mts_stats* stats,
                      void* stream) {
  FIELDS(f);
  hmc_status s = check_mts(F, p);
  if (s) return s;
  HMC_REQUIRE(phi2 && stats, "null argument");
  hipStream_t st = ST(stream);
  HMC_CHECK_HIP(launch_copy(F->phi2, phi2, F->half64, st));
  *stats = hmc_mts_stats{};
  s = mts_integrate(F, p, stats, st);
  if (s) return s;
  HMC_CHECK_HIP(hipStreamSynchronize(st));
  if (stats->nonfinite) {
    set_error("%d solves met a non-finite residual", stats->nonfinite);
    return HMC_E_NAN;
  }
  if (stats->nonconverged) {
    set_error("%d solves did not converge", stats->nonconverged);
    return HMC_E_NOCONV;
  }
  return HMC_OK;
}

hmc_status hmc_trajectory_mts(hmc_fields* f, uint64_t seed, uint64_t traj, const hmc_mts_params* p,
                              hmc_traj_result* res, hmc_mts_stats* stats, void* stream) {
  FIELDS(f);
  hmc_status s = check_mts(F, p);
  if (s) return s;
  HMC_REQUIRE(res && stats, "null argument");
  hipStream_t st = ST(stream);
  auto t0 = std::chrono::steady_clock::now();
  const double k = F->kappa, kh = p->kappa_h;
  *stats = hmc_mts_stats{};
  const size_t ub = gauge_bytes(F->g.Vh, HMC_F64);
  HMC_CHECK_HIP(launch_copy(F->U_old, F->U, ub, st));
  F->su3_old = F->su3;
  HMC_CHECK_HIP(launch_refresh_momenta(F->g, seed, traj, F->P, st));
  // phi_1 = Mhat_h^dag eta_1;  phi_2 = Mhat_h A_h^-1 Mhat^dag eta_2
  HMC_CHECK_HIP(launch_eta(F->g, seed, traj, 0, F->eta, st, 0));
  HMC_CHECK_HIP(launch_eta(F->g, seed, traj, 0, F->eta2, st, 1));
  HMC_CHECK_HIP(mhat_k(F, F->phi, F->eta, 1, kh, st));
  HMC_CHECK_HIP(mhat_k(F, F->chi, F->eta2, 1, k, st));
  int nc = 0, nf = 0;
  s = solve_at(F, kh, F->Xe, F->chi, &p->cg, &stats->iters_heavy, &nc, &nf, st);
  if (s) return s;
  stats->solves_heavy++;
  HMC_CHECK_HIP(mhat_k(F, F->phi2, F->Xe, 0, kh, st));

  const int nb = F->nbR;
  HMC_CHECK_HIP(launch_kinetic_partials(F->g, F->P, F->part[0], nb, st));
  HMC_CHECK_HIP(finalize_to_slot(F, F->part[0], nb, 1, SL_KE_OLD, st));
  HMC_CHECK_HIP(plaquette_to_slot(F, SL_PLAQ_OLD, st));
  // S_1 + S_2 = |eta_1|^2 + |eta_2|^2 into SL_ETA2 (parts in SL_RED + 0, + 1)
  HMC_CHECK_HIP(launch_norm2_partials(F->g, HMC_F64, F->eta, F->part[0], nb, st));
  HMC_CHECK_HIP(finalize_to_slot(F, F->part[0], nb, 1, SL_RED + 0, st));
  HMC_CHECK_HIP(launch_finalize(F->part[0], nb, 1, F->slots + SL_ETA2, 1.0, 0, st));
  HMC_CHECK_HIP(launch_norm2_partials(F->g, HMC_F64, F->eta2, F->part[0], nb, st));
  HMC_CHECK_HIP(finalize_to_slot(F, F->part[0], nb, 1, SL_RED + 1, st));
  HMC_CHECK_HIP(launch_finalize(F->part[0], nb, 1, F->slots + SL_ETA2, 1.0, 1, st));

  s = mts_integrate(F, p, stats, st);
  if (s) return s;
  stats->nonconverged += nc;
  stats->nonfinite += nf;

  HMC_CHECK_HIP(launch_kinetic_partials(F->g, F->P, F->part[0], nb, st));
  HMC_CHECK_HIP(finalize_to_slot(F, F->part[0], nb, 1, SL_KE_NEW, st));
  HMC_CHECK_HIP(plaquette_to_slot(F, SL_PLAQ_NEW, st));
  // S_1 = <phi_1, X_1>, S_2 = <chi, X_2> at the final links (SL_RED + 2.., + 4..)
  HMC_CHECK_HIP(launch_inner_partials(F->g, F->phi, F->Xe, F->part[1], nb, st));
  HMC_CHECK_HIP(finalize_to_slot(F, F->part[1], nb, 2, SL_RED + 2, st));
  HMC_CHECK_HIP(launch_finalize(F->part[1], nb, 2, F->slots + SL_PHIX, 1.0, 0, st));
  HMC_CHECK_HIP(launch_inner_partials(F->g, F->chi, F->X2, F->part[1], nb, st));
  HMC_CHECK_HIP(finalize_to_slot(F, F->part[1], nb, 2, SL_RED + 4, st));
  HMC_CHECK_HIP(launch_finalize(F->part[1], nb, 2, F->slots + SL_PHIX, 1.0, 1, st));
  HMC_CHECK_HIP(launch_metropolis(seed, traj, F->beta, (double)F->V, F->slots, st));
  double sl[13], parts[6];
  HMC_CHECK_HIP(read_slots(F, 0, 13, sl, st));
  HMC_CHECK_HIP(read_slots(F, SL_RED, 6, parts, st));

  const bool converged = stats->nonconverged == 0;
  const bool finite = std::isfinite(sl[SL_DH]) && stats->nonfinite == 0;
  bool accepted = sl[SL_ACC] != 0.0 && converged && finite;
  if (!accepted) {
    HMC_CHECK_HIP(launch_copy(F->U, F->U_old, ub, st));
    F->u_version++;
    F->su3 = F->su3_old;
  }
  double plaq_sum;
  HMC_CHECK_HIP(plaquette_to_slot(F, SL_RED, st));
  HMC_CHECK_HIP(read_slots(F, SL_RED, 1, &plaq_sum, st));

  stats->S1_old = parts[0];
  stats->S2_old = parts[1];
  stats->S1_new = parts[2];
  stats->S2_new = parts[4];
  res->KE_old = sl[SL_KE_OLD];
  res->KE_new = sl[SL_KE_NEW];
  res->S_f_old = sl[SL_ETA2];
  res->S_g_old = sl[SL_SG_OLD];
  res->S_g_new = sl[SL_SG_NEW];
  res->H_old = sl[SL_H_OLD];
  res->H_new = sl[SL_H_NEW];
  res->dH = sl[SL_DH];
  res->u = sl[SL_U];
  res->S_f_new = sl[SL_PHIX];
  res->accepted = accepted ? 1 : 0;
  res->plaquette = plaq_sum / (18.0 * F->V);
  res->cg_iters_total = stats->iters_ratio + stats->iters_heavy;
  res->cg_iters_max = 0;
  res->nonconverged = stats->nonconverged;
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (!finite) {
    set_error("non-finite energy change (%d solves non-finite); trajectory rejected", stats->nonfinite);
    return HMC_E_NAN;
  }
  if (!converged) {
    set_error("%d solves did not converge; trajectory rejected", stats->nonconverged);
    return HMC_E_NOCONV;
  }
  return HMC_OK;
}

// ------------------------------------------------------- auto-tuning

hmc_status hmc_autotune(hmc_fields* f, const char* db_path, void* stream) {
  FIELDS(f);
  HMC_REQUIRE(!tune_env_forced(), "HMC_DSLASH_SPLIT or HMC_GFORCE_PLANES forces the launch shapes; unset it to tune");
  hipStream_t st = ST(stream);
  hipEvent_t e0, e1;
  HMC_CHECK_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    set_error("hipEventCreate failed");
    return HMC_E_HIP;
  }
  auto elapsed_us = [&](auto&& work) -> double {  // GPU time of work() on st, gaps included
    if (hipEventRecord(e0, st) != hipSuccess) return -1;
    if (!work()) return -1;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1;
    float ms = 0;
    return hipEventElapsedTime(&ms, e0, e1) == hipSuccess ? 1e3 * ms : -1;
  };
  hmc_status status = HMC_OK;
  const std::string err0 = "a timed launch failed during tuning";
  std::string err = err0;
  // Dslash: each (shape, link form) timed where it runs, inside a solve (CG
  // on Mhat^dag Mhat from Gaussian noise, tolerance 1e-10 or kIters
  // iterations; FP64 CG, else mixed precision with the storage inside), per
  // iteration.  The candidate is installed as the table entries, since a
  // solve takes its shapes from the table when it starts; FP64 goes first
  // because the mixed-precision solves run their FP64 steps with the FP64
  // choice.  Link forms are tuned on SU(3) fields only (others read every
  // entry).
  constexpr int kIters = 100, kReps = 3;
  const std::vector<int> forms = F->su3 ? std::vector<int>{LINK_ROWS2, LINK_ROWCOL} : std::vector<int>{0};
  if (launch_eta(F->g, 1, 0, 0, F->eta, st) != hipSuccess) status = HMC_E_HIP;
  const int nprec = (F->flags & HMC_FIELDS_LOWPREC) ? 4 : 1;
  for (int pi = 0; pi < nprec && status == HMC_OK; ++pi) {
    const hmc_prec prec = (hmc_prec)pi;
    hmc_cg_params prm{};
    prm.tol = 1e-10;
    prm.maxiter = kIters;
    prm.mode = HMC_CG_NORMAL_MHAT;
    prm.prec = prec;
    // one timed candidate: installs its table entries, returns us per
    // iteration (< 0 after a failure; status / err say which)
    auto time_candidate = [&](int shape, int form, int stream, int order, int occ) -> double {
      tune_store(F->g.L, TUNE_DSLASH, prec, shape, 0);
      if (form) tune_store(F->g.L, TUNE_DSLASH_LINKS, prec, form, 0);
      if (form) tune_store(F->g.L, TUNE_DSLASH_STREAM, prec, stream, 0);
      tune_store(F->g.L, TUNE_DSLASH_ORDER, prec, order, 0);
      tune_store(F->g.L, TUNE_DSLASH_OCC, prec, occ, 0);
      double us = -1;
      for (int r = 0; r <= kReps; ++r) {  // r = 0 warms up
        hmc_cg_stats cs{};
        hmc_status s = HMC_OK;
        const double t = elapsed_us([&] {
          s = cg_solve_impl(F, F->Xe, F->eta, &prm, &cs, st);
          return s == HMC_OK || s == HMC_E_NOCONV;
        });
        if (t < 0 || cs.iters <= 0) {
          status = s != HMC_OK && s != HMC_E_NOCONV ? s : HMC_E_HIP;
          if (s != HMC_OK && s != HMC_E_NOCONV) err = hmc_last_error();
          return -1;
        }
        if (r > 0 && (us < 0 || t / cs.iters < us)) us = t / cs.iters;
      }
      return us;
    };
    // shapes x link forms (linear order, no streaming), then streaming and
    // the tiled orders x workgroups per CU for the best pair
    int best = 0, best_form = 0, best_stream = 0, best_order = 0, best_occ = 2;
    double best_us = 0;
    for (int form : forms) {
      for (int shape : {1, 2, 4}) {
        const double us = time_candidate(shape, form, 0, 0, 2);
        if (us < 0) break;
        if (!best || us < best_us) best = shape, best_form = form, best_us = us;
      }
      if (status != HMC_OK) break;
    }
    if (status == HMC_OK && best_form) {
      const double us = time_candidate(best, best_form, 1, 0, 2);
      if (us >= 0 && us < best_us) best_stream = 1, best_us = us;
    }
    if (status == HMC_OK && best == 1 && tiled_order_valid(F->g)) {
      // whole z-planes, then y-blocks of a few chunks
      for (int order : {1, 2, 3, 4, 6}) {
        if (!tiled_order_valid(F->g, order) || (order > 1 && order >= F->g.L[0] * F->g.L[1] / 128)) continue;
        for (int occ : {2, 0}) {
          const double us = time_candidate(best, best_form, best_stream, order, occ);
          if (us < 0) break;
          if (us < best_us) best_order = order, best_occ = occ, best_us = us;
        }
        if (status != HMC_OK) break;
      }
    }
    if (status == HMC_OK) {
      tune_store(F->g.L, TUNE_DSLASH, prec, best, best_us);
      tune_store(F->g.L, TUNE_DSLASH_ORDER, prec, best_order, best_us);
      tune_store(F->g.L, TUNE_DSLASH_OCC, prec, best_occ, best_us);
      if (best_form) {
        tune_store(F->g.L, TUNE_DSLASH_LINKS, prec, best_form, best_us);
        tune_store(F->g.L, TUNE_DSLASH_STREAM, prec, best_stream, best_us);
      }
    }
  }
  // staple force: the launch alone (coef 0 leaves P unchanged), each shape
  // and link form
  if (status == HMC_OK) {
    int best = -1, best_form = 0;
    double best_us = 0;
    for (int form : forms) {
      for (int shape : {0, 1, 2}) {
        auto launch = [&] {
          return launch_gauge_force(F->g, F->U, F->P, 0.0, st, F->su3, shape, form) == hipSuccess;
        };
        double us = -1;
        if (launch() && launch()) us = elapsed_us([&] {
          for (int r = 0; r < 5; ++r)
            if (!launch()) return false;
          return true;
        }) / 5;
        if (us < 0) {
          status = HMC_E_HIP;
          break;
        }
        if (best < 0 || us < best_us) best = shape, best_form = form, best_us = us;
      }
      if (status != HMC_OK) break;
    }
    if (status == HMC_OK) {
      tune_store(F->g.L, TUNE_GFORCE, HMC_F64, best, best_us);
      if (best_form) tune_store(F->g.L, TUNE_GFORCE_LINKS, HMC_F64, best_form, best_us);
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (status != HMC_OK) {
    set_error("%s", err.c_str());
    return status;
  }
  if (db_path && tune_save(db_path) < 0) {
    set_error("could not write the tuning table to %s", db_path);
    return HMC_E_ARG;
  }
  return HMC_OK;
}

hmc_status hmc_stream_triad(void* a, const void* b, const void* c, double s, uint64_t n, int32_t nontemporal,
                            void* stream) {
  HMC_REQUIRE(a && b && c, "null buffer");
  HMC_REQUIRE(n % 2 == 0, "n = %llu must be even", (unsigned long long)n);
  HMC_REQUIRE(((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) % 16 == 0, "buffers must be 16-byte aligned");
  if (n == 0) return HMC_OK;
  HMC_CHECK_HIP(launch_triad(a, b, c, s, n / 2, nontemporal != 0, ST(stream)));
  return HMC_OK;
}

hmc_status hmc_tune_load(const char* path, int32_t* n_entries) {
  HMC_REQUIRE(path, "null path");
  const int n = tune_load(path);
  HMC_REQUIRE(n >= 0, "cannot read %s", path);
  if (n_entries) *n_entries = n;
  return HMC_OK;
}

hmc_status hmc_tune_save(const char* path, int32_t* n_entries) {
  HMC_REQUIRE(path, "null path");
  const int n = tune_save(path);
  HMC_REQUIRE(n >= 0, "cannot write %s", path);
  if (n_entries) *n_entries = n;
  return HMC_OK;
}

hmc_status hmc_tune_query(const int32_t* L, int32_t kind, int32_t prec, int32_t* choice, int32_t* tuned) {
  HMC_REQUIRE(L && choice, "null argument");
  HMC_REQUIRE(kind >= HMC_TUNE_DSLASH && kind <= HMC_TUNE_DSLASH_OCC, "bad kind %d", kind);
  HMC_REQUIRE(prec >= HMC_F64 && prec <= HMC_BF16, "bad precision %d", prec);
  hmc_geom geom;
  for (int k = 0; k < 4; ++k) geom.L[k] = L[k];
  LatArg g;
  long long V;
  hmc_status s = check_geom(&geom, &g, &V);
  if (s) return s;
  const int ints[4] = {L[0], L[1], L[2], L[3]};
  const bool per_prec = kind == HMC_TUNE_DSLASH || kind == HMC_TUNE_DSLASH_LINKS || kind == HMC_TUNE_DSLASH_STREAM ||
                        kind == HMC_TUNE_DSLASH_ORDER || kind == HMC_TUNE_DSLASH_OCC;
  const int t = tune_lookup(ints, kind, per_prec ? prec : HMC_F64);
  switch (kind) {
    case HMC_TUNE_DSLASH: *choice = dslash_shape(g, (hmc_prec)prec); break;
    case HMC_TUNE_GAUGE_FORCE: *choice = gauge_force_shape(g); break;
    case HMC_TUNE_DSLASH_LINKS: *choice = dslash_link_form(g, (hmc_prec)prec); break;
    case HMC_TUNE_DSLASH_STREAM: *choice = dslash_link_stream(g, (hmc_prec)prec) ? 1 : 0; break;
    case HMC_TUNE_DSLASH_ORDER: *choice = dslash_tiled_order(g, (hmc_prec)prec); break;
    case HMC_TUNE_DSLASH_OCC: *choice = dslash_tiled_occupancy(g, (hmc_prec)prec); break;
    default: *choice = staple_link_form(g); break;
  }
  if (tuned) *tuned = t >= 0 ? 1 : 0;
  return HMC_OK;
}
