// Kernels and launchers of the Wilson hopping term, instantiated once per
// storage precision (dslash_f64.hip, dslash_f32.hip, dslash_f16.hip,
// dslash_bf16.hip; dslash.hip dispatches).
//
// Wilson hopping term on one checkerboard (the dominant kernel of the
// fermion-matrix inversion that the paper's introduction singles out as
// the bulk of the floating-point work):
//   (D psi)(x) = sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu)
//                      + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)]
// with -1 on hops across the time boundary; the dagger swaps the
// projectors.  One work-item per output site (Sec. 3's site-per-thread
// mapping); the 4x4 spin structure is applied through the rank-2
// projections (1 +- gamma_mu), so each hop multiplies only two colour
// vectors by the link.
//
// The kernel is HBM-bound (about 0.86 flop per byte in FP64).  Fields are
// stored component-major so every load instruction of a wave covers one
// contiguous 1 KiB (FP64) span; neighbour spinors are re-read through L2,
// and the XCD-aware block order keeps the +-y/+-z neighbours of a block on
// the XCD that owns it.
#pragma once

#include <hip/hip_ext.h>

#include "device.h"
#include "internal.h"

namespace hmc {

#ifndef HMC_DSLASH_WAVES
#define HMC_DSLASH_WAVES
#endif
#ifndef HMC_HOP_CHAIN
#define HMC_HOP_CHAIN 1
#endif

// Makes `idx` depend on every accumulator without changing either.  The
// loads of a hop use indices chained to the accumulators left by the
// previous hop, so the compiler cannot issue all sixteen hops' loads up
// front (that needs ~600 registers and spills); a wave keeps one hop
// (HMC_HOP_CHAIN = 1) or one direction (= 2) of loads in flight and
// occupancy supplies the memory parallelism.
template <typename R>
__device__ __forceinline__ int chain(int idx, cx<R>* acc) {
#if HMC_HOP_CHAIN
#pragma unroll
  for (int k = 0; k < 12; ++k) asm volatile("" : "+v"(acc[k].re), "+v"(acc[k].im));
  asm volatile("" : "+v"(idx));
#endif
  return idx;
}

template <class SP, class LK, int MU, bool DAG>
__device__ __forceinline__ void hop_dir(const Lat& g, const Site& st, int out_par, int s, const void* U,
                                        const void* in, cx<typename SP::R>* acc) {
  using R = typename SP::R;
  constexpr int SF = DAG ? +1 : -1;  // forward hop carries (1 + SF gamma_mu)
  constexpr int SB = -SF;
  bool wf, wb;
  const int lf = neighbour_lex<MU, +1>(g, st, &wf);
  const int lb = neighbour_lex<MU, -1>(g, st, &wb);
  {
    cx<R> psi[12], h[6], uh[6];
    const int sn = chain(lf >> 1, acc), sl = chain(s, acc);
    SP::load(in, g.stride, sn, psi);
    spin_project<MU, SF>(psi, h);
    if (MU == 3) {  // antiperiodic time boundary
      const R sg = wf ? R(-1) : R(1);
#pragma unroll
      for (int k = 0; k < 6; ++k) h[k] = sg * h[k];
    }
    const mat3<R> u = LK::load(U, g.stride, MU, out_par, sl);
    mv(u, h, uh);
    mv(u, h + 3, uh + 3);
    spin_accum<MU, SF>(acc, uh);
  }
  {
    cx<R> psi[12], h[6], uh[6];
    const int sn = HMC_HOP_CHAIN == 1 ? chain(lb >> 1, acc) : lb >> 1;
    SP::load(in, g.stride, sn, psi);
    spin_project<MU, SB>(psi, h);
    if (MU == 3) {
      const R sg = wb ? R(-1) : R(1);
#pragma unroll
      for (int k = 0; k < 6; ++k) h[k] = sg * h[k];
    }
    const mat3<R> u = LK::load(U, g.stride, MU, out_par ^ 1, sn);
    mdv(u, h, uh);
    mdv(u, h + 3, uh + 3);
    spin_accum<MU, SB>(acc, uh);
  }
}

// Block 0 computes the solver step length from the partial sums of the
// previous kernels (see DslashArgs::alpha_out); the other blocks skip it.
template <int W = kBlock / 64>
__device__ __forceinline__ void alpha_prologue(const DslashArgs& e, int label) {
  if (!e.alpha_out || blockIdx.x != 0) return;
  const double* part[2] = {e.alpha_pp[label & 1], e.alpha_den};
  const int n[2] = {e.alpha_n_pp, e.alpha_n_den};
  double s[2];
  sum_partials_n<W, 2>(part, n, s);
  if (threadIdx.x == 0) *(HMC_GLOBAL double*)e.alpha_out = s[0] / s[1];
}

// BATCH: blockIdx.y selects an entry of `table` (same-volume requests share
// one launch); otherwise the single entry `one` is read from the kernel
// arguments.
template <class SP, class LK, bool DAG, int EPI, bool BATCH>
__global__ void __launch_bounds__(kBlock) HMC_DSLASH_WAVES k_dslash(Lat g, int out_par,
                                                                    const DslashArgs* __restrict__ table,
                                                                    DslashArgs one, int j) {
  using R = typename SP::R;
  const DslashArgs* ep;
  if constexpr (BATCH)
    ep = table + blockIdx.y;
  else
    ep = &one;
  const DslashArgs& e = *ep;
  const int label = e.iter0 + j + (e.label_base ? *(const HMC_GLOBAL int*)e.label_base : 0);
  if (e.stop_at && label >= *(const HMC_GLOBAL int*)e.stop_at) return;
  alpha_prologue(e, label);
  int b;
  const int s = dslash_site(g, &b);
  double nrm[1] = {0.0};
  if (s < g.Vh) {
    const Site st = cb_site(g, out_par, s);
    cx<R> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
    hop_dir<SP, LK, 0, DAG>(g, st, out_par, s, e.U, e.in, acc);
    hop_dir<SP, LK, 1, DAG>(g, st, out_par, s, e.U, e.in, acc);
    hop_dir<SP, LK, 2, DAG>(g, st, out_par, s, e.U, e.in, acc);
    hop_dir<SP, LK, 3, DAG>(g, st, out_par, s, e.U, e.in, acc);
    if (EPI != EPI_PLAIN) {
      const R a = (R)e.a, bb = (R)e.b;
      if (e.y) {
        cx<R> y[12];
        SP::load(e.y, g.stride, s, y);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {fma(bb, acc[k].re, a * y[k].re), fma(bb, acc[k].im, a * y[k].im)};
      } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = bb * acc[k];
      }
    }
    if (EPI == EPI_CG) {  // acc = q = A p;  r <- r - alpha q
      const R al = (R)(*(const HMC_GLOBAL double*)e.alpha_in);
      cx<R> r[12];
      SP::load(e.r, g.stride, s, r);
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = {fma(-al, acc[k].re, r[k].re), fma(-al, acc[k].im, r[k].im)};
    }
    if (EPI == EPI_AXPY_NORM || EPI == EPI_CG)
#pragma unroll
      for (int k = 0; k < 12; ++k) nrm[0] += (double)acc[k].re * acc[k].re + (double)acc[k].im * acc[k].im;
    SP::template store<LK::kStream>(e.out, g.stride, s, acc);
  }
  if (EPI == EPI_AXPY_NORM || EPI == EPI_CG) {
    block_sum<1>(nrm);
    double* dst = e.partial_pp[0] ? e.partial_pp[(label + 1) & 1] : e.partial;
    if (threadIdx.x == 0) ((HMC_GLOBAL double*)dst)[b] = nrm[0];
  }
}

// Direction-split variant: a block covers 64 sites with NW wavefronts
// (NW = 2 or 4); wave w computes the hops along directions
// w*4/NW .. (w+1)*4/NW - 1 for those sites and parks its partial sum in
// LDS; after a barrier each work-item combines the NW partials of 12/NW of
// the 12 components of one site (coalesced stores).  NW times the
// wavefronts of the one-site-per-work-item kernel at the same registers per
// work-item, and 1/NW of its serial hop chain per wavefront.
template <class SP, class LK, bool DAG, int EPI, bool BATCH, int NW>
__global__ void __launch_bounds__(NW * 64) k_dslash_split(Lat g, int out_par, const DslashArgs* __restrict__ table,
                                                          DslashArgs one, int j) {
  using R = typename SP::R;
  constexpr int kSites = 64;
  constexpr int kDirs = 4 / NW;    // directions per wavefront
  constexpr int kParts = 4 / NW;   // groups of 3 components per work-item in the combine
  __shared__ cx<R> part[NW][12][kSites];
  const DslashArgs* ep;
  if constexpr (BATCH)
    ep = table + blockIdx.y;
  else
    ep = &one;
  const DslashArgs& e = *ep;
  const int label = e.iter0 + j + (e.label_base ? *(const HMC_GLOBAL int*)e.label_base : 0);
  if (e.stop_at && label >= *(const HMC_GLOBAL int*)e.stop_at) return;
  alpha_prologue<NW>(e, label);
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int w = threadIdx.x >> 6;  // wave index (uniform per wave)
  const int ls = threadIdx.x & (kSites - 1);
  const int s = b * kSites + ls;
  {
    cx<R> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
    if (s < g.Vh) {
      const Site st = cb_site(g, out_par, s);
      if constexpr (NW == 4) {
        switch (w) {
          case 0: hop_dir<SP, LK, 0, DAG>(g, st, out_par, s, e.U, e.in, acc); break;
          case 1: hop_dir<SP, LK, 1, DAG>(g, st, out_par, s, e.U, e.in, acc); break;
          case 2: hop_dir<SP, LK, 2, DAG>(g, st, out_par, s, e.U, e.in, acc); break;
          default: hop_dir<SP, LK, 3, DAG>(g, st, out_par, s, e.U, e.in, acc); break;
        }
      } else {
        if (w == 0) {
          hop_dir<SP, LK, 0, DAG>(g, st, out_par, s, e.U, e.in, acc);
          hop_dir<SP, LK, 1, DAG>(g, st, out_par, s, e.U, e.in, acc);
        } else {
          hop_dir<SP, LK, 2, DAG>(g, st, out_par, s, e.U, e.in, acc);
          hop_dir<SP, LK, 3, DAG>(g, st, out_par, s, e.U, e.in, acc);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) part[w][k][ls] = acc[k];
  }
  (void)kDirs;
  __syncthreads();
  // work-item (ls, w) now owns components 3*kParts*w .. 3*kParts*(w+1)-1 of site s
  double nrm[1] = {0.0};
  cx<R> o[3 * kParts];
  const bool active = s < g.Vh;
  if (active) {
#pragma unroll
    for (int c = 0; c < 3 * kParts; ++c) {
      const int k = 3 * kParts * w + c;
      cx<R> t = part[0][k][ls];
#pragma unroll
      for (int q = 1; q < NW; ++q) t = t + part[q][k][ls];
      o[c] = t;
    }
    if (EPI != EPI_PLAIN) {
      const R a = (R)e.a, bb = (R)e.b;
#pragma unroll
      for (int c = 0; c < 3 * kParts; ++c) {
        if (e.y) {
          const cx<R> y = SP::load_one(e.y, g.stride, s, 3 * kParts * w + c);
          o[c] = {fma(bb, o[c].re, a * y.re), fma(bb, o[c].im, a * y.im)};
        } else {
          o[c] = bb * o[c];
        }
      }
    }
    if (EPI == EPI_CG) {
      const R al = (R)(*(const HMC_GLOBAL double*)e.alpha_in);
#pragma unroll
      for (int c = 0; c < 3 * kParts; ++c) {
        const cx<R> rv = SP::load_one(e.r, g.stride, s, 3 * kParts * w + c);
        o[c] = {fma(-al, o[c].re, rv.re), fma(-al, o[c].im, rv.im)};
      }
    }
    if (EPI == EPI_AXPY_NORM || EPI == EPI_CG)
#pragma unroll
      for (int c = 0; c < 3 * kParts; ++c) nrm[0] += (double)o[c].re * o[c].re + (double)o[c].im * o[c].im;
  }
  if constexpr (SP::kScaled) {
    // the per-site scale needs the largest |re|, |im| over all 12 components
    __shared__ float smax[NW][kSites];
    float m = 0.f;
    if (active)
#pragma unroll
      for (int c = 0; c < 3 * kParts; ++c) m = fmaxf(m, fmaxf(fabsf((float)o[c].re), fabsf((float)o[c].im)));
    smax[w][ls] = m;
    __syncthreads();
    m = smax[0][ls];
#pragma unroll
    for (int q = 1; q < NW; ++q) m = fmaxf(m, smax[q][ls]);
    if (active)
#pragma unroll
      for (int q = 0; q < kParts; ++q)
        SP::template store_part_scaled<LK::kStream>(e.out, g.stride, s, kParts * w + q, o + 3 * q, m);
  } else {
    if (active)
#pragma unroll
      for (int q = 0; q < kParts; ++q) SP::template store_part<LK::kStream>(e.out, g.stride, s, kParts * w + q, o + 3 * q);
  }
  if (EPI == EPI_AXPY_NORM || EPI == EPI_CG) {
    block_sum<1, NW>(nrm);
    double* dst = e.partial_pp[0] ? e.partial_pp[(label + 1) & 1] : e.partial;
    if (threadIdx.x == 0) ((HMC_GLOBAL double*)dst)[b] = nrm[0];
  }
}

template <class SP, class LK>
static hipError_t launch_typed(hmc_prec prec, int dagger, int epi, const LatArg& ga, int out_par,
                               const DslashArgs* table, int nbatch, const DslashArgs& one, hipStream_t st, int j,
                               KernelEvents ev) {
  Lat g = to_lat(ga);
  const int shape = one.shape ? one.shape : dslash_shape(ga, prec);
  const int order = shape == 1 ? dslash_tiled_order(ga, prec) : 0;
  if (order) {
    g.tiled = 1;
    g.plane = ga.L[0] * ga.L[1] / 2;
    g.slice = g.plane * ga.L[2];
    g.tile_r = g.plane % 64 == 0 ? g.plane / 64 : 0;
    g.tile_t = ga.L[3] / 8;
    g.tile_y = order == 1 ? g.tile_r : order;  // 0: chunks of the t-slices
  }
  const int ways = shape == 1 ? 0 : shape;
  const dim3 grid(dslash_shape_blocks(ga.Vh, shape), nbatch);
  const dim3 block(ways ? 64 * ways : kBlock);
  // The tiled order may reserve LDS it does not use: 54,000 bytes per block
  // leave room for two blocks per CU (2 wavefronts per SIMD), so an XCD's
  // wavefronts in flight span a few (z, t) rows instead of dozens and the
  // neighbours they share are still in its L2 (measured at 48^3x96 with
  // whole z-planes: FP64 1.36 ms without the cap, 1.24 ms with it, 1.27-1.31
  // ms for the linear order; with y-blocks the FP32 and FP16 kernels run
  // faster without it).
  const size_t lds_cap = g.tiled && dslash_tiled_occupancy(ga, prec) == 2 ? 54000 : 0;
#define HMC_LAUNCH(KERNEL) \
  hipExtLaunchKernelGGL(KERNEL, grid, block, lds_cap, st, ev.start, ev.stop, 0, g, out_par, table, one, j)
#define HMC_DS_B(D, E, B)                                  \
  do {                                                     \
    if (ways == 4)                                         \
      HMC_LAUNCH((k_dslash_split<SP, LK, D, E, B, 4>));    \
    else if (ways == 2)                                    \
      HMC_LAUNCH((k_dslash_split<SP, LK, D, E, B, 2>));    \
    else                                                   \
      HMC_LAUNCH((k_dslash<SP, LK, D, E, B>));             \
  } while (0)
#define HMC_DS(D, E)            \
  do {                          \
    if (table)                  \
      HMC_DS_B(D, E, true);     \
    else                        \
      HMC_DS_B(D, E, false);    \
  } while (0)
  if (epi == EPI_CG) {  // last hop of a CG iteration: dagger, one solve
    if (table || !dagger) return hipErrorInvalidValue;
    HMC_DS_B(true, EPI_CG, false);
    return hipGetLastError();
  }
  if (dagger) {
    if (epi == EPI_PLAIN) HMC_DS(true, EPI_PLAIN);
    else if (epi == EPI_AXPY) HMC_DS(true, EPI_AXPY);
    else HMC_DS(true, EPI_AXPY_NORM);
  } else {
    if (epi == EPI_PLAIN) HMC_DS(false, EPI_PLAIN);
    else if (epi == EPI_AXPY) HMC_DS(false, EPI_AXPY);
    else HMC_DS(false, EPI_AXPY_NORM);
  }
#undef HMC_DS
#undef HMC_DS_B
#undef HMC_LAUNCH
  return hipGetLastError();
}

// Link form (SU(3) fields: the tuned compact form and streaming choice,
// else all entries), then shape and epilogue.
template <class SP, class LK>
hipError_t launch_links(hmc_prec prec, int dagger, int epi, const LatArg& g, int out_par, const DslashArgs* table,
                        int nbatch, const DslashArgs& one, hipStream_t st, int j) {
  const int form = link_form_for(one.su3, dslash_link_form(g, prec));
  const bool stream = form != LINK_FULL && dslash_link_stream(g, prec);
  const int link_bytes = form == LINK_ROWCOL ? LkRowCol<LK>::kBytes : form == LINK_ROWS2 ? LkRows2<LK>::kBytes
                                                                                          : LK::kBytes;
  // bytes per site: 8 links + 1 input + 1 output spinor (+1 for y, +1 more
  // for the residual read by the CG epilogue); algorithmic with whole links,
  // moved with the stored reals of the link form
  const double spinor_bytes = 2 * SP::kBytes + (epi ? SP::kBytes : 0) + (epi == EPI_CG ? SP::kBytes : 0);
  const double alg = (8.0 * LK::kBytes + spinor_bytes) * g.Vh * nbatch;
  const double moved = (8.0 * link_bytes + spinor_bytes) * g.Vh * nbatch;
  const KernelEvents ev = timing_kernel_events(TK_DSLASH, alg, moved);
  if (form == LINK_ROWCOL) {
    if (stream)
      return launch_typed<SP, LkRowCol<LK, true>>(prec, dagger, epi, g, out_par, table, nbatch, one, st, j, ev);
    return launch_typed<SP, LkRowCol<LK>>(prec, dagger, epi, g, out_par, table, nbatch, one, st, j, ev);
  }
  if (form == LINK_ROWS2) {
    if (stream)
      return launch_typed<SP, LkRows2<LK, true>>(prec, dagger, epi, g, out_par, table, nbatch, one, st, j, ev);
    return launch_typed<SP, LkRows2<LK>>(prec, dagger, epi, g, out_par, table, nbatch, one, st, j, ev);
  }
  return launch_typed<SP, LK>(prec, dagger, epi, g, out_par, table, nbatch, one, st, j, ev);
}

}  // namespace hmc
