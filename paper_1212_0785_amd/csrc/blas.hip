// Global sums (the QDP++ sum / innerProduct / sumMulti functions named in
// the paper's QDP-JIT feature list, Sec. 1) and the fused vector updates
// of the Krylov solvers.
//
// Every reduction is deterministic and independent of other work in the
// same launch: a work-item accumulates its sites in a fixed grid-stride
// order, a wave64 butterfly and a fixed wave order give one partial per
// block, and consumers sum the partials in index order.  The solver
// kernels re-sum the partials they need in every block (the same bits in
// every block), which removes the separate finalisation launches from the
// iteration.
#include <hip/hip_ext.h>

#include <algorithm>
#include <climits>

#include "device.h"
#include "internal.h"

namespace hmc {


// ------------------------------------------------------------- sums

// Longest run of inner iterations between two device-driven reliable updates.
constexpr int kMaxInner = 48;

// The kernels taking `gate` do nothing while *gate == 0 (gate may be null).
__device__ __forceinline__ bool gate_closed(const int* gate) { return gate && *gate == 0; }

template <class SP>
__global__ void __launch_bounds__(kBlock) k_norm2_partials(Lat g, const void* x, double* part, const int* gate) {
  if (gate_closed(gate)) return;
  double v[1] = {0.0};
  for (int s = blockIdx.x * kBlock + threadIdx.x; s < g.Vh; s += gridDim.x * kBlock) {
    cx<typename SP::R> a[12];
    SP::load(x, g.stride, s, a);
#pragma unroll
    for (int k = 0; k < 12; ++k) v[0] += (double)a[k].re * a[k].re + (double)a[k].im * a[k].im;
  }
  block_sum<1>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(kBlock) k_inner_partials(Lat g, const double2* a, const double2* b, double* part) {
  double v[2] = {0.0, 0.0};
  const size_t n = (size_t)12 * g.stride;
  for (size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (size_t)gridDim.x * kBlock) {
    if ((int)(j % g.stride) >= g.Vh) continue;
    double2 x = a[j], y = b[j];
    v[0] += x.x * y.x + x.y * y.y;  // Re conj(x) y
    v[1] += x.x * y.y - x.y * y.x;  // Im conj(x) y
  }
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = v[0];
    part[gridDim.x + blockIdx.x] = v[1];
  }
}

__global__ void __launch_bounds__(kBlock) k_finalize(const double* part, int n, int nvals, double* out, double scale,
                                                     int accumulate, const int* gate) {
  if (gate_closed(gate)) return;
  for (int v = 0; v < nvals; ++v) {
    double s = sum_partials(part + (size_t)v * n, n);
    if (threadIdx.x == 0) out[v] = (accumulate ? out[v] : 0.0) + scale * s;
  }
}

// sumMulti: per-block histogram of |x|^2 over subsets, accumulated in
// site order by one work-item per block (deterministic), then summed over
// blocks in block order.
constexpr int kMaxSub = 1024;

__global__ void __launch_bounds__(kBlock) k_sum_multi_partials(Lat g, const double2* x, const int* subset, int nsub,
                                                               double* part) {
  __shared__ double bins[kMaxSub];
  __shared__ double vals[kBlock];
  __shared__ int subs[kBlock];
  for (int k = threadIdx.x; k < nsub; k += kBlock) bins[k] = 0.0;
  const int half = blockIdx.y;
  const double2* xh = x + (size_t)half * 12 * g.stride;
  const int* sh = subset + (size_t)half * g.Vh;
  for (int base = blockIdx.x * kBlock; base < g.Vh; base += gridDim.x * kBlock) {
    int s = base + threadIdx.x;
    double v = 0.0;
    int sub = 0;
    if (s < g.Vh) {
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        double2 a = xh[(size_t)k * g.stride + s];
        v += a.x * a.x + a.y * a.y;
      }
      sub = sh[s];
    }
    __syncthreads();
    vals[threadIdx.x] = v;
    subs[threadIdx.x] = sub;
    __syncthreads();
    if (threadIdx.x == 0) {
      int n = min(kBlock, g.Vh - base);
      for (int k = 0; k < n; ++k)
        if (subs[k] >= 0 && subs[k] < nsub) bins[subs[k]] += vals[k];  // ids outside [0, nsub) are ignored
    }
  }
  __syncthreads();
  double* out = part + ((size_t)half * gridDim.x + blockIdx.x) * nsub;
  for (int k = threadIdx.x; k < nsub; k += kBlock) out[k] = bins[k];
}

__global__ void k_sum_multi_final(const double* part, int nrows, int nsub, double* out) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= nsub) return;
  double s = 0.0;
  for (int r = 0; r < nrows; ++r) s += part[(size_t)r * nsub + k];
  out[k] = s;
}

// ------------------------------------------------------- element-wise

// STREAM triad a = b + s c over n2 double2 elements, four per work-item
// (all loads before the stores), optionally with non-temporal hints: the
// attainable streaming rate of this chip for the access pattern of the
// field kernels (16-byte lanes, contiguous waves).
template <bool NT>
__global__ void __launch_bounds__(kBlock) k_triad(void* a, const void* b, const void* c, double sc, size_t n2) {
  constexpr int U = 4;
  const size_t step = (size_t)gridDim.x * kBlock;
  for (size_t j0 = (size_t)blockIdx.x * kBlock + threadIdx.x; j0 < n2; j0 += step * U) {
    v2d x[U], y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t j = j0 + u * step;
      if (j < n2) {
        x[u] = gld_link<v2d, NT>((const char*)b + j * 16, 0);
        y[u] = gld_link<v2d, NT>((const char*)c + j * 16, 0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t j = j0 + u * step;
      if (j < n2) gput<NT>((char*)a + j * 16, 0, v2d{fma(sc, y[u].x, x[u].x), fma(sc, y[u].y, x[u].y)});
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_xmy_norm(Lat g, const double2* b, const double2* q, double2* r,
                                                    double* part, const int* gate) {
  if (gate_closed(gate)) return;
  double v[1] = {0.0};
  for (int s = blockIdx.x * kBlock + threadIdx.x; s < g.Vh; s += gridDim.x * kBlock) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      size_t j = (size_t)k * g.stride + s;
      double2 d = make_double2(b[j].x - q[j].x, b[j].y - q[j].y);
      r[j] = d;
      v[0] += d.x * d.x + d.y * d.y;
    }
  }
  block_sum<1>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ void k_zero(uint4* p, size_t n16, unsigned char* tail, size_t ntail) {
  for (size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x; j < n16; j += (size_t)gridDim.x * kBlock)
    p[j] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

__global__ void k_copy(uint4* d, const uint4* s, size_t n16, unsigned char* dt, const unsigned char* st,
                       size_t ntail, const int* gate) {
  if (gate && *gate == 0) return;
  for (size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x; j < n16; j += (size_t)gridDim.x * kBlock) d[j] = s[j];
  if (blockIdx.x == 0 && threadIdx.x < ntail) dt[threadIdx.x] = st[threadIdx.x];
}

// ------------------------------------------------------------ solvers

// x = 0, r = p = b, partials of |b|^2 (FP64 vectors).
__global__ void __launch_bounds__(kBlock) k_cg_init(Lat g, const double2* b, double2* x, double2* r, double2* p,
                                                    double* part) {
  double v[1] = {0.0};
  for (int s = blockIdx.x * kBlock + threadIdx.x; s < g.Vh; s += gridDim.x * kBlock) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      size_t j = (size_t)k * g.stride + s;
      double2 a = b[j];
      x[j] = make_double2(0.0, 0.0);
      r[j] = a;
      p[j] = a;
      v[0] += a.x * a.x + a.y * a.y;
    }
  }
  block_sum<1>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// The arguments of this block's solve: entry blockIdx.y of a batch table,
// or the single entry passed by value.  Chosen at compile time, so the
// by-value entry is read in place from the kernel arguments (a run-time
// choice copies the struct to per-lane scratch memory).
template <bool BATCH>
__device__ __forceinline__ const CgArgs& cg_args(const CgArgs* table, const CgArgs& one) {
  if constexpr (BATCH)
    return table[blockIdx.y];
  else
    return one;
}

// One solver iteration with label k = iter0 + j; cur = k & 1, nxt = cur ^ 1.
//   update:  alpha = sum(pp[cur]) / sum(pq);  x += alpha p;  r -= alpha q;
//            per-block |r|^2 -> pp[nxt] (CG) or pr (CGLS)
//   pupdate: beta = sum(pp[nxt]) / sum(pp[cur]);  p = src + beta p with
//            src = r (CG) or s (CGLS); convergence measure |r|^2 =
//            sum(pp[nxt]) (CG) or sum(pr) (CGLS).
// (CG: pp holds |r|^2, pq = <p, A p> = |Mhat p|^2.  CGLS: pp holds
// |s|^2 = |Mhat^dag r|^2, pq = |q|^2 = |Mhat p|^2.)
// Fused CG (CgArgs::fused): the update kernel is not launched; the
// preceding Dslash computes alpha (block 0, into the solver state) and
// r -= alpha q in its epilogue, and the p-update also does x += alpha p.
template <class SP, class SX, bool BATCH>
__global__ void __launch_bounds__(kBlock) k_cg_update(Lat g, const CgArgs* table, CgArgs one, int j) {
  const CgArgs& a = cg_args<BATCH>(table, one);
  const int k = a.iter0 + a.state->base + j;
  if (k >= a.state->stop_at) return;
  using R = typename SP::R;
  const int cur = k & 1;
  const double* part[2] = {a.pp[cur], a.pq};
  const int n[2] = {a.n_pp, a.n_pq};
  double sums[2];
  sum_partials_n<kBlock / 64, 2>(part, n, sums);
  const double alpha = sums[0] / sums[1];
  const R al = (R)alpha;
  double v[1] = {0.0};
  for (int s = blockIdx.x * kBlock + threadIdx.x; s < g.Vh; s += gridDim.x * kBlock) {
    cx<R> p[12], q[12], r[12];
    cx<typename SX::R> x[12];
    SP::load(a.p, g.stride, s, p);
    SP::load(a.q, g.stride, s, q);
    SP::load(a.r, g.stride, s, r);
    SX::load(a.x, g.stride, s, x);
#pragma unroll
    for (int m = 0; m < 12; ++m) {
      x[m].re = fma((typename SX::R)alpha, (typename SX::R)p[m].re, x[m].re);
      x[m].im = fma((typename SX::R)alpha, (typename SX::R)p[m].im, x[m].im);
      r[m].re = fma(-al, q[m].re, r[m].re);
      r[m].im = fma(-al, q[m].im, r[m].im);
      v[0] += (double)r[m].re * r[m].re + (double)r[m].im * r[m].im;
    }
    SX::store(a.x, g.stride, s, x);
    SP::store(a.r, g.stride, s, r);
  }
  block_sum<1>(v);
  double* out = a.cgls ? a.pr : a.pp[cur ^ 1];
  if (threadIdx.x == 0) out[blockIdx.x] = v[0];
}

// Block 0 records the iteration and, when |r|^2 <= thr (or, in mixed
// precision, when the inner residual fell by delta since the last FP64
// update), sets stop_at = k + 1; blocks of this launch compare k only, so
// none of them can observe a change that concerns it.
//
// NP work-items share a site: work-item (part, s) updates the colour
// vectors 12/NP * part .. of site s (NP = 4 only for storages without a
// per-site scale).  Every input of an element is loaded before any output
// is stored (x, p and r are distinct arrays), so a work-item makes one
// round trip to memory.
template <class SP, class SX, int NP, bool BATCH>
__global__ void __launch_bounds__(kBlock) k_cg_pupdate(Lat g, const CgArgs* table, CgArgs one, int j) {
  static_assert(NP == 1 || (NP == 4 && !SP::kScaled), "parts need an unscaled storage");
  const CgArgs& a = cg_args<BATCH>(table, one);
  SolverState* stt = a.state;
  const int k = a.iter0 + stt->base + j;
  if (k >= stt->stop_at) return;
  using R = typename SP::R;
  using XR = typename SX::R;
  constexpr int NC = 12 / NP;  // components per work-item
  const int cur = k & 1, nxt = cur ^ 1;
  const void* src = a.cgls ? a.s : a.r;
  // XCD x (hardware blocks b with b % 8 == x; gridDim.x is a multiple of
  // 8) updates the sites [x Vh / 8, (x + 1) Vh / 8), the range the Dslash's
  // XCD-aware block order gives the same XCD, so p, r and x stay in the L2
  // of the XCD that reads them next.
  const int xcd = blockIdx.x & 7, nbx = gridDim.x >> 3;
  const int lo = (int)((long long)g.Vh * xcd / 8), nsx = (int)((long long)g.Vh * (xcd + 1) / 8) - lo;
  const int nwork = nsx * NP;
  cx<R> p[NC], q[NC];
  cx<XR> x[NC];
  auto load = [&](int i) {
    const int part = NP == 1 ? 0 : i / nsx;
    const int s = lo + i - part * nsx;
    if constexpr (NP == 1) {
      SP::load(a.p, g.stride, s, p);
      if (a.fused) SX::load(a.x, g.stride, s, x);
      SP::load(src, g.stride, s, q);
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) p[c] = SP::load_one(a.p, g.stride, s, NC * part + c);
      if (a.fused)
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = SX::load_one(a.x, g.stride, s, NC * part + c);
#pragma unroll
      for (int c = 0; c < NC; ++c) q[c] = SP::load_one(src, g.stride, s, NC * part + c);
    }
  };
  // The first element's loads do not depend on the sums: issued before the
  // reduction, their latency overlaps it.
  const int i0 = (blockIdx.x >> 3) * kBlock + threadIdx.x;
  if (i0 < nwork) load(i0);
  // the three sums of this step in one block reduction (same order, hence
  // the same bits, in every block)
  __shared__ double bc[3];
  __shared__ int fold_sh;
  {
    // each work-item adds its partials in index order; the loads of up to
    // eight of them are issued together
    constexpr int U = 8;
    double v[3] = {0.0, 0.0, 0.0};
    for (int base = threadIdx.x; base < a.n_pp; base += U * kBlock) {
      double t0[U], t1[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = base + u * kBlock;
        t0[u] = i < a.n_pp ? a.pp[nxt][i] : 0.0;
        t1[u] = i < a.n_pp ? a.pp[cur][i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) v[0] += t0[u], v[1] += t1[u];
    }
    if (a.cgls)
      for (int base = threadIdx.x; base < a.n_pr; base += U * kBlock) {
        double t2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = base + u * kBlock;
          t2[u] = i < a.n_pr ? a.pr[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) v[2] += t2[u];
      }
    block_sum<3>(v);
    if (threadIdx.x == 0) {
      bc[0] = v[0], bc[1] = v[1], bc[2] = v[2];
      // mixed precision with device-driven updates: does this iteration ask
      // for one?  (Block 0 may already have raised maxrr to max(maxrr, rr):
      // every block gets the same answer.)
      const double r2 = a.cgls ? v[2] : v[0];
      // (ru_iter and ru_label change only between chunks, so every block
      // counts the same iterations.)
      const int done_after = stt->ru_iter + (k + 1 - stt->ru_label);
      fold_sh = a.x64 && (r2 <= stt->thr || r2 < a.delta2 * fmax(stt->maxrr, r2) || !(r2 == r2) ||
                          k + 1 - stt->ru_label >= kMaxInner || (a.max_iters > 0 && done_after >= a.max_iters));
    }
    __syncthreads();
  }
  const double nw = bc[0], old = bc[1];
  const double rr = a.cgls ? bc[2] : nw;
  const bool conv = rr <= stt->thr;
  const double alpha = a.fused ? stt->alpha : 0.0;
  // the iteration that asks for an update folds the inner solution into
  // the FP64 one (x64 += xl, xl = 0) for the update that follows
  const bool fold = fold_sh != 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    stt->iters += 1;
    stt->last = k;
    stt->rr = rr;
    if (a.mixed) {
      double mx = fmax(stt->maxrr, rr);
      stt->maxrr = mx;
      // updates also come every kMaxInner iterations, so a low-precision
      // recursion that stagnates cannot run away (the host-driven updates
      // of the solve service: since the restart at ru_label), and, device
      // driven, at the iteration limit
      if (a.x64 ? fold : (conv || rr < a.delta2 * mx || !(rr == rr) || k + 1 - stt->ru_label >= kMaxInner)) {
        stt->reason = 2;
        stt->stop_at = k + 1;
        stt->ru_gate = INT_MAX;  // a device-driven solve updates next
      }
    } else if (conv || !(rr == rr)) {
      stt->reason = conv ? 1 : 3;
      stt->stop_at = k + 1;
    }
  }
  const bool p_done = conv && !a.mixed;  // converged: the search direction is not needed
  if (p_done && !a.fused) return;
  const R beta = (R)(nw / old);
  for (int i = i0; i < nwork; i += nbx * kBlock) {
    const int part = NP == 1 ? 0 : i / nsx;
    const int s = lo + i - part * nsx;
    if (i != i0) load(i);
    if (a.fused) {  // x += alpha p with the p of this iteration
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        x[m].re = fma((XR)alpha, (XR)p[m].re, x[m].re);
        x[m].im = fma((XR)alpha, (XR)p[m].im, x[m].im);
      }
    } else if (fold) {  // CGLS: x was updated by the update kernel
      if constexpr (NP == 1)
        SX::load(a.x, g.stride, s, x);
      else
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = SX::load_one(a.x, g.stride, s, NC * part + c);
    }
    if (fold) {
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        double2* h = (double2*)a.x64 + (size_t)(NP == 1 ? m : NC * part + m) * g.stride + s;
        const double2 v = *h;
        *h = make_double2(v.x + (double)x[m].re, v.y + (double)x[m].im);
        x[m] = {(XR)0, (XR)0};
      }
    }
    if (a.fused || fold) {
      if constexpr (NP == 1)
        SX::store(a.x, g.stride, s, x);
      else
        SX::store_part(a.x, g.stride, s, part, x);
    }
    if (p_done) continue;
#pragma unroll
    for (int m = 0; m < NC; ++m) {
      p[m].re = fma(beta, p[m].re, q[m].re);
      p[m].im = fma(beta, p[m].im, q[m].im);
    }
    if constexpr (NP == 1)
      SP::store(a.p, g.stride, s, p);
    else
      SP::store_part(a.p, g.stride, s, part, p);
  }
}

// Start or resume a solve: stop_at = INT_MAX, reason = 0, no reliable
// update pending, maxrr from a device slot (null -> 0), threshold thr; a
// start also clears the counts and the label base.
__global__ void k_state_reset(SolverState* st, const double* maxrr, int nbatch, int reset_iters, double thr,
                              int label) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= nbatch) return;
  st[k].stop_at = INT_MAX;
  st[k].reason = 0;
  st[k].ru_gate = 0;
  st[k].thr = thr;
  if (reset_iters) {
    st[k].iters = 0;
    st[k].last = -1;
    st[k].rr = 0.0;
    st[k].base = 0;
    st[k].done = 0;
    st[k].nru = 0;
    st[k].ru_iter = 0;
    st[k].ru_label = 0;
    st[k].rr64 = 0.0;
  }
  st[k].maxrr = maxrr ? maxrr[k] : 0.0;
  if (label >= 0) st[k].ru_label = label;
}

// dst = src over n doubles while *gate != 0.
__global__ void k_copy_doubles_gated(double* dst, const double* src, int n, const int* gate) {
  if (*gate == 0) return;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) dst[i] = src[i];
}

__global__ void k_advance_base(SolverState* st, int n) {
  if (threadIdx.x == 0) st->base += n;
}

__global__ void k_ru_request(SolverState* st) {
  if (threadIdx.x != 0) return;
  st->ru_gate = INT_MAX;
  st->stop_at = min(st->stop_at, st->base);
}

// The end of a device-driven reliable update (see launch_ru_finish).  One
// block; every thread reads the gate before thread 0 clears it (the sum
// synchronises the block in between).
__global__ void __launch_bounds__(kBlock) k_ru_finish(SolverState* st, const double* part64, int n, double* slot,
                                                     int max_ru, int max_iters) {
  if (st->ru_gate == 0) {
    if (threadIdx.x == 0) st->restart = 0;
    return;
  }
  const double rr64 = sum_partials(part64, n);
  if (threadIdx.x != 0) return;
  *slot = rr64;
  // The reliable update keeps the search direction p, which is conjugate
  // for the recursive residual it replaces.  Where the two differ by more
  // than a factor 2 in |r|^2, or a whole cycle of inner iterations did not
  // lower the FP64 residual, the low-precision recursion has lost track
  // (BF16 storage with a small delta does this) and keeping p makes the
  // iteration diverge: p restarts from the new residual instead.
  st->restart = rr64 > 2.0 * st->rr || (st->nru > 0 && rr64 >= st->rr64);
  st->nru += 1;
  st->ru_iter = st->iters;
  st->ru_label = st->base;
  st->rr64 = rr64;
  if (rr64 <= st->thr) {
    st->done = 1;
  } else if (!isfinite(rr64)) {
    st->done = 3;
  } else if (st->nru >= max_ru || st->iters >= max_iters) {
    st->done = 4;
  } else {  // resume: the iterations of the next chunk run
    st->stop_at = INT_MAX;
    st->reason = 0;
    st->maxrr = rr64;
  }
  st->ru_gate = 0;
}

// Device-driven reliable update after q = A x (see launch_ru_residual).  The
// |r|^2 of the stored low-precision r is summed from its stored values, as
// the norm of a freshly converted vector is.
template <class SP>
__global__ void __launch_bounds__(kBlock) k_ru_residual(Lat g, const double2* rhs, const double2* q, double2* r64,
                                                        void* rlow, double* part64, double* pp0, double* pp1,
                                                        const int* gate) {
  if (*gate == 0) return;
  using R = typename SP::R;
  double v[2] = {0.0, 0.0};
  for (int s = blockIdx.x * kBlock + threadIdx.x; s < g.Vh; s += gridDim.x * kBlock) {
    cx<R> a[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const size_t j = (size_t)k * g.stride + s;
      const double2 d = make_double2(rhs[j].x - q[j].x, rhs[j].y - q[j].y);
      r64[j] = d;
      v[0] += d.x * d.x + d.y * d.y;
      a[k] = {(R)d.x, (R)d.y};
    }
    SP::store(rlow, g.stride, s, a);
    if (pp0) {
      SP::load(rlow, g.stride, s, a);
#pragma unroll
      for (int k = 0; k < 12; ++k) v[1] += (double)a[k].re * a[k].re + (double)a[k].im * a[k].im;
    }
  }
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    part64[blockIdx.x] = v[0];
    if (pp0) pp0[blockIdx.x] = v[1], pp1[blockIdx.x] = v[1];
  }
}

// x64 += x32; x32 = 0 (mixed precision accumulator hand-over).
__global__ void k_add_low_to_f64(Lat g, double2* x64, float2* x32, const int* gate) {
  if (gate_closed(gate)) return;
  const size_t n = (size_t)12 * g.stride;
  for (size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (size_t)gridDim.x * kBlock) {
    float2 l = x32[j];
    double2 h = x64[j];
    x64[j] = make_double2(h.x + (double)l.x, h.y + (double)l.y);
    x32[j] = make_float2(0.f, 0.f);
  }
}

// ------------------------------------------------------------ launchers

// One wavefront that does nothing: the floor of a launch timed through a
// kernel-stamped event pair.
__global__ void k_empty() {}

hipError_t launch_empty_timed(hipStream_t st) {
  const KernelEvents ev = timing_kernel_events(TK_OTHER, 0.0);
  hipExtLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, st, ev.start, ev.stop, 0);
  return hipGetLastError();
}

hipError_t launch_triad(void* a, const void* b, const void* c, double sc, size_t n2, bool nt, hipStream_t st) {
  TimedScope ts(TK_OTHER, st, 48.0 * n2);
  const int nb = (int)std::min<size_t>((n2 + 4 * kBlock - 1) / (4 * kBlock), 65536);
  if (nt)
    hipLaunchKernelGGL(k_triad<true>, dim3(nb), dim3(kBlock), 0, st, a, b, c, sc, n2);
  else
    hipLaunchKernelGGL(k_triad<false>, dim3(nb), dim3(kBlock), 0, st, a, b, c, sc, n2);
  return hipGetLastError();
}

hipError_t launch_norm2_partials(const LatArg& g, hmc_prec prec, const void* x, double* part, int nb,
                                 hipStream_t st, const int* gate) {
  const double kb[4] = {SpF64::kBytes, SpF32::kBytes, SpF16::kBytes, SpBF16::kBytes};
  TimedScope ts(TK_REDUCE, st, kb[prec] * g.Vh);
  switch (prec) {
    case HMC_F64: hipLaunchKernelGGL(k_norm2_partials<SpF64>, dim3(nb), dim3(kBlock), 0, st, to_lat(g), x, part, gate); break;
    case HMC_F32: hipLaunchKernelGGL(k_norm2_partials<SpF32>, dim3(nb), dim3(kBlock), 0, st, to_lat(g), x, part, gate); break;
    case HMC_F16: hipLaunchKernelGGL(k_norm2_partials<SpF16>, dim3(nb), dim3(kBlock), 0, st, to_lat(g), x, part, gate); break;
    case HMC_BF16: hipLaunchKernelGGL(k_norm2_partials<SpBF16>, dim3(nb), dim3(kBlock), 0, st, to_lat(g), x, part, gate); break;
  }
  return hipGetLastError();
}

hipError_t launch_inner_partials(const LatArg& g, const void* a, const void* b, double* part, int nb,
                                 hipStream_t st) {
  TimedScope ts(TK_REDUCE, st, 2.0 * SpF64::kBytes * g.Vh);
  hipLaunchKernelGGL(k_inner_partials, dim3(nb), dim3(kBlock), 0, st, to_lat(g), (const double2*)a,
                     (const double2*)b, part);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* part, int n, int nvals, double* out, double scale, int accumulate,
                           hipStream_t st, const int* gate) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, st, part, n, nvals, out, scale, accumulate, gate);
  return hipGetLastError();
}

hipError_t launch_sum_multi(const LatArg& g, const void* x, int nhalves, const int* subset, int nsub, double* part,
                            int nb, double* out, hipStream_t st) {
  if (nsub > kMaxSub || nsub < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sum_multi_partials, dim3(nb, nhalves), dim3(kBlock), 0, st, to_lat(g), (const double2*)x,
                     subset, nsub, part);
  hipLaunchKernelGGL(k_sum_multi_final, dim3(ceil_div(nsub, kBlock)), dim3(kBlock), 0, st, part, nb * nhalves, nsub,
                     out);
  return hipGetLastError();
}

// out = sum_k c_k y_k over n <= 4 F64 half spinors (complex coefficients).
struct LinComb {
  const double2* y[4];
  double2 c[4];
  int n;
};

__global__ void __launch_bounds__(kBlock) k_lincomb(Lat g, LinComb a, double2* out) {
  const size_t total = (size_t)12 * g.stride;
  for (size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x; j < total; j += (size_t)gridDim.x * kBlock) {
    double re = 0.0, im = 0.0;
    for (int k = 0; k < a.n; ++k) {
      const double2 v = a.y[k][j];
      re += a.c[k].x * v.x - a.c[k].y * v.y;
      im += a.c[k].x * v.y + a.c[k].y * v.x;
    }
    out[j] = make_double2(re, im);
  }
}

hipError_t launch_lincomb(const LatArg& g, const void* const* y, const double* c, int n, void* out, hipStream_t st) {
  if (n < 1 || n > 4) return hipErrorInvalidValue;
  LinComb a{};
  for (int k = 0; k < n; ++k) {
    a.y[k] = (const double2*)y[k];
    a.c[k] = make_double2(c[2 * k], c[2 * k + 1]);
  }
  a.n = n;
  hipLaunchKernelGGL(k_lincomb, dim3(blas_blocks(g.Vh)), dim3(kBlock), 0, st, to_lat(g), a, (double2*)out);
  return hipGetLastError();
}

hipError_t launch_xmy_norm(const LatArg& g, const void* b, const void* q, void* r, double* part, int nb,
                           hipStream_t st, const int* gate) {
  hipLaunchKernelGGL(k_xmy_norm, dim3(nb), dim3(kBlock), 0, st, to_lat(g), (const double2*)b, (const double2*)q,
                     (double2*)r, part, gate);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  size_t n16 = bytes / 16, nt = bytes % 16;
  int nb = (int)std::min<size_t>(std::max<size_t>((n16 + kBlock - 1) / kBlock, 1), 4096);
  hipLaunchKernelGGL(k_zero, dim3(nb), dim3(kBlock), 0, st, (uint4*)p, n16, (unsigned char*)p + n16 * 16, nt);
  return hipGetLastError();
}

hipError_t launch_copy_gated(void* dst, const void* src, size_t bytes, const int* gate, hipStream_t st) {
  size_t n16 = bytes / 16, nt = bytes % 16;
  int nb = (int)std::min<size_t>(std::max<size_t>((n16 + kBlock - 1) / kBlock, 1), 4096);
  hipLaunchKernelGGL(k_copy, dim3(nb), dim3(kBlock), 0, st, (uint4*)dst, (const uint4*)src, n16,
                     (unsigned char*)dst + n16 * 16, (const unsigned char*)src + n16 * 16, nt, gate);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
  return launch_copy_gated(dst, src, bytes, nullptr, st);
}

hipError_t launch_cg_init(const LatArg& g, hmc_prec prec, const void* b, void* x, void* r, void* p, double* part,
                          int nb, hipStream_t st) {
  if (prec != HMC_F64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(kBlock), 0, st, to_lat(g), (const double2*)b, (double2*)x,
                     (double2*)r, (double2*)p, part);
  return hipGetLastError();
}

// Bytes of a solver-vector update per site: x read and written in its own
// storage, `nsp` reads or writes of vectors of the iteration's storage.
static double cg_vec_bytes(hmc_prec prec, bool with_x, int nsp) {
  const double sp = prec == HMC_F64 ? SpF64::kBytes : prec == HMC_F32 ? SpF32::kBytes
                    : prec == HMC_F16 ? SpF16::kBytes : SpBF16::kBytes;
  const double sx = prec == HMC_F64 ? SpF64::kBytes : SpF32::kBytes;
  return (with_x ? 2 * sx : 0.0) + nsp * sp;
}

hipError_t launch_cg_update(const LatArg& g, hmc_prec prec, const CgArgs& a, int nb, const CgArgs* table,
                            int nbatch, int j, hipStream_t st) {
  // x += alpha p, r -= alpha q: x read + written, p and q read, r read + written
  TimedScope ts(TK_CG_BLAS, st, cg_vec_bytes(prec, true, 4) * g.Vh * nbatch);
  const dim3 grid(nb, nbatch), block(kBlock);
  auto go = [&](auto kernel_single, auto kernel_batch) {
    if (table)
      hipLaunchKernelGGL(kernel_batch, grid, block, 0, st, to_lat(g), table, a, j);
    else
      hipLaunchKernelGGL(kernel_single, grid, block, 0, st, to_lat(g), table, a, j);
  };
  switch (prec) {
    case HMC_F64: go(k_cg_update<SpF64, SpF64, false>, k_cg_update<SpF64, SpF64, true>); break;
    case HMC_F32: go(k_cg_update<SpF32, SpF32, false>, k_cg_update<SpF32, SpF32, true>); break;
    case HMC_F16: go(k_cg_update<SpF16, SpF32, false>, k_cg_update<SpF16, SpF32, true>); break;
    case HMC_BF16: go(k_cg_update<SpBF16, SpF32, false>, k_cg_update<SpBF16, SpF32, true>); break;
  }
  return hipGetLastError();
}

hipError_t launch_cg_pupdate(const LatArg& g, hmc_prec prec, const CgArgs& a, int nb, const CgArgs* table,
                             int nbatch, int j, hipStream_t st) {
  // p = r + beta p: p read + written, r read (fused: x += alpha p as well)
  TimedScope ts(TK_CG_BLAS, st, cg_vec_bytes(prec, a.fused != 0, 3) * g.Vh * nbatch);
  (void)nb;  // the update writes no partial sums: its grid is its own
  // multiples of 8 blocks (one share per XCD)
  const int nb4 = std::min(8 * ceil_div(4LL * g.Vh, 8 * kBlock), 2048);
  const int nb1 = std::min(8 * ceil_div(g.Vh, 8 * kBlock), 2048);
  const dim3 block(kBlock);
  auto go = [&](int nb_, auto kernel_single, auto kernel_batch) {
    const dim3 grid(nb_, nbatch);
    if (table)
      hipLaunchKernelGGL(kernel_batch, grid, block, 0, st, to_lat(g), table, a, j);
    else
      hipLaunchKernelGGL(kernel_single, grid, block, 0, st, to_lat(g), table, a, j);
  };
  switch (prec) {
    case HMC_F64: go(nb4, k_cg_pupdate<SpF64, SpF64, 4, false>, k_cg_pupdate<SpF64, SpF64, 4, true>); break;
    case HMC_F32: go(nb4, k_cg_pupdate<SpF32, SpF32, 4, false>, k_cg_pupdate<SpF32, SpF32, 4, true>); break;
    case HMC_F16: go(nb1, k_cg_pupdate<SpF16, SpF32, 1, false>, k_cg_pupdate<SpF16, SpF32, 1, true>); break;
    case HMC_BF16: go(nb4, k_cg_pupdate<SpBF16, SpF32, 4, false>, k_cg_pupdate<SpBF16, SpF32, 4, true>); break;
  }
  return hipGetLastError();
}

hipError_t launch_state_reset(SolverState* st_dev, const double* maxrr, int nbatch, int reset_iters, double thr,
                              hipStream_t st, int label) {
  hipLaunchKernelGGL(k_state_reset, dim3(ceil_div(nbatch, kBlock)), dim3(kBlock), 0, st, st_dev, maxrr, nbatch,
                     reset_iters, thr, label);
  return hipGetLastError();
}

hipError_t launch_advance_base(SolverState* st_dev, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_advance_base, dim3(1), dim3(64), 0, st, st_dev, n);
  return hipGetLastError();
}

hipError_t launch_copy_doubles_gated(double* dst, const double* src, int n, const int* gate, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_doubles_gated, dim3(std::max(1, std::min(ceil_div(n, kBlock), 64))), dim3(kBlock), 0, st,
                     dst, src, n, gate);
  return hipGetLastError();
}

hipError_t launch_ru_request(SolverState* st_dev, hipStream_t st) {
  hipLaunchKernelGGL(k_ru_request, dim3(1), dim3(64), 0, st, st_dev);
  return hipGetLastError();
}

hipError_t launch_ru_finish(SolverState* st_dev, const double* part64, int n, double* rr64_slot, int max_ru,
                            int max_iters, hipStream_t st) {
  hipLaunchKernelGGL(k_ru_finish, dim3(1), dim3(kBlock), 0, st, st_dev, part64, n, rr64_slot, max_ru, max_iters);
  return hipGetLastError();
}

hipError_t launch_ru_residual(const LatArg& g, hmc_prec prec, const void* rhs, const void* q, void* r64, void* rlow,
                              double* part64, double* pp0, double* pp1, int nb, const int* gate, hipStream_t st) {
  const dim3 grid(nb), block(kBlock);
  const Lat lat = to_lat(g);
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, grid, block, 0, st, lat, (const double2*)rhs, (const double2*)q, (double2*)r64, rlow,
                       part64, pp0, pp1, gate);
  };
  switch (prec) {
    case HMC_F64: return hipErrorInvalidValue;  // FP64 solves need no update
    case HMC_F32: go(k_ru_residual<SpF32>); break;
    case HMC_F16: go(k_ru_residual<SpF16>); break;
    case HMC_BF16: go(k_ru_residual<SpBF16>); break;
  }
  return hipGetLastError();
}

hipError_t launch_add_low_to_f64(const LatArg& g, void* x64, void* xlow, hipStream_t st, const int* gate) {
  hipLaunchKernelGGL(k_add_low_to_f64, dim3(blas_blocks(g.Vh)), dim3(kBlock), 0, st, to_lat(g), (double2*)x64,
                     (float2*)xlow, gate);
  return hipGetLastError();
}

}  // namespace hmc
