// Random fields of the HMC (the "random number generator", momentum and
// pseudofermion refresh of the paper's Sec. 1), from a counter-based
// generator so that every site draws independently and the result does not
// depend on the launch shape: Philox4x64-10 with counter (block, lexicographic
// site, stream, epoch) and key (seed, 0).  Streams: 0 weak-field start,
// 1 momenta, 2 pseudofermion noise, 3 Metropolis, 4 solver sources.
#include "device.h"
#include "internal.h"

namespace hmc {


enum { ST_WEAKFIELD = 0, ST_MOMENTA = 1, ST_ETA = 2, ST_ACCEPT = 3, ST_SOURCE = 4, ST_ETA2 = 5 };

// n (even, <= 32) Gaussians of one site, consecutive word pairs through
// Box-Muller.
template <int N>
__device__ __forceinline__ void site_gaussians(uint64_t seed, uint64_t site, uint64_t stream, uint64_t epoch,
                                               double* g) {
#pragma unroll
  for (int b = 0; b < N / 4; ++b) {
    uint64_t w[4];
    philox4x64_10(b, site, stream, epoch, seed, 0, w);
    box_muller(w[0], w[1], &g[4 * b], &g[4 * b + 1]);
    box_muller(w[2], w[3], &g[4 * b + 2], &g[4 * b + 3]);
  }
}

// sum_a w_a T^a (T^a = lambda^a/2) in compact form.
__device__ __forceinline__ void algebra_compact(const double* w, double* c) {
  const double inv_sqrt3 = 0.57735026918962576451;
  c[0] = 0.5 * (w[2] + inv_sqrt3 * w[7]);
  c[1] = 0.5 * (-w[2] + inv_sqrt3 * w[7]);
  c[2] = 0.5 * w[0];
  c[3] = -0.5 * w[1];
  c[4] = 0.5 * w[3];
  c[5] = -0.5 * w[4];
  c[6] = 0.5 * w[5];
  c[7] = -0.5 * w[6];
}

// One work-item per link (blockIdx.y = mu): the eight Gaussians of
// direction mu are the words of Philox blocks 2 mu and 2 mu + 1 of the
// site's stream, so every value is the one a whole-site work-item would
// draw, with a quarter of its registers.
__global__ void __launch_bounds__(kBlock) k_refresh_momenta(Lat g, uint64_t seed, uint64_t epoch, double* P) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= 2 * g.Vh) return;
  int par = j >= g.Vh, s = j - par * g.Vh;
  const int mu = blockIdx.y;
  Site x = cb_site(g, par, s);
  double gs[8];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    uint64_t w[4];
    philox4x64_10(2 * mu + b, (uint64_t)x.lex, ST_MOMENTA, epoch, seed, 0, w);
    box_muller(w[0], w[1], &gs[4 * b], &gs[4 * b + 1]);
    box_muller(w[2], w[3], &gs[4 * b + 2], &gs[4 * b + 3]);
  }
  double c[8];
  algebra_compact(gs, c);
  store_compact(P, g.stride, mu, par, s, c);
}

__global__ void __launch_bounds__(kBlock) k_weak_field(Lat g, uint64_t seed, double eps, void* U) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= 2 * g.Vh) return;
  int par = j >= g.Vh, s = j - par * g.Vh;
  Site x = cb_site(g, par, s);
  double gs[32];
  site_gaussians<32>(seed, (uint64_t)x.lex, ST_WEAKFIELD, 0, gs);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    double c[8];
    algebra_compact(&gs[8 * mu], c);
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] *= eps;
    mat3<double> u = exp_iQ(herm_from_compact(c));
    reunitarise(u);
    LkF64::store(U, g.stride, mu, par, s, u);
  }
}

// eta on the sites of parity par: complex Gaussian with E|eta_k|^2 = 1.
// Three work-items per site (blockIdx.y = q): components 4q .. 4q+3 from
// Philox blocks 2q and 2q + 1 of the site's stream, the values a
// whole-site work-item would draw.
__global__ void __launch_bounds__(kBlock) k_eta(Lat g, uint64_t seed, uint64_t epoch, int par, double2* half,
                                                int rng_stream) {
  int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.Vh) return;
  const int q = blockIdx.y;
  Site x = cb_site(g, par, s);
  double gs[8];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    uint64_t w[4];
    philox4x64_10(2 * q + b, (uint64_t)x.lex, rng_stream, epoch, seed, 0, w);
    box_muller(w[0], w[1], &gs[4 * b], &gs[4 * b + 1]);
    box_muller(w[2], w[3], &gs[4 * b + 2], &gs[4 * b + 3]);
  }
  const double r = 0.70710678118654752440;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    half[(size_t)(4 * q + k) * g.stride + s] = make_double2(r * gs[2 * k], r * gs[2 * k + 1]);
}

// Sources on both parities (blockIdx.y = parity).
__global__ void __launch_bounds__(kBlock) k_source(Lat g, int kind, uint64_t seed, uint64_t epoch, double2* even,
                                                   double2* odd) {
  int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.Vh) return;
  int par = blockIdx.y;
  double2* out = par ? odd : even;
  Site x = cb_site(g, par, s);
  if (kind == 0) {
    double gs[24];
    site_gaussians<24>(seed, (uint64_t)x.lex, ST_SOURCE, epoch, gs);
#pragma unroll
    for (int k = 0; k < 12; ++k) out[(size_t)k * g.stride + s] = make_double2(gs[2 * k], gs[2 * k + 1]);
  } else if (kind == 1) {
    const double r = 0.70710678118654752440;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      uint64_t w[4];
      philox4x64_10(b, (uint64_t)x.lex, ST_SOURCE, epoch, seed, 0, w);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double re = (w[2 * h] >> 63) ? -r : r;
        double im = (w[2 * h + 1] >> 63) ? -r : r;
        out[(size_t)(2 * b + h) * g.stride + s] = make_double2(re, im);
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k)
      out[(size_t)k * g.stride + s] = make_double2((x.lex == 0 && k == 0) ? 1.0 : 0.0, 0.0);
  }
}

__global__ void k_site_words(uint64_t seed, uint64_t stream, uint64_t epoch, const long long* sites, int nsites,
                             int nblocks, uint64_t* out) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= nsites) return;
  for (int b = 0; b < nblocks; ++b) {
    uint64_t w[4];
    philox4x64_10(b, (uint64_t)sites[j], stream, epoch, seed, 0, w);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[((size_t)j * nblocks + b) * 4 + k] = w[k];
  }
}

__global__ void k_site_gaussians(uint64_t seed, uint64_t stream, uint64_t epoch, const long long* sites, int nsites,
                                 int n, double* out) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= nsites) return;
  double gs[32];
  switch (n) {
    case 4: site_gaussians<4>(seed, (uint64_t)sites[j], stream, epoch, gs); break;
    case 8: site_gaussians<8>(seed, (uint64_t)sites[j], stream, epoch, gs); break;
    case 12: site_gaussians<12>(seed, (uint64_t)sites[j], stream, epoch, gs); break;
    case 16: site_gaussians<16>(seed, (uint64_t)sites[j], stream, epoch, gs); break;
    case 20: site_gaussians<20>(seed, (uint64_t)sites[j], stream, epoch, gs); break;
    case 24: site_gaussians<24>(seed, (uint64_t)sites[j], stream, epoch, gs); break;
    case 28: site_gaussians<28>(seed, (uint64_t)sites[j], stream, epoch, gs); break;
    default: site_gaussians<32>(seed, (uint64_t)sites[j], stream, epoch, gs); break;
  }
  for (int k = 0; k < n; ++k) out[(size_t)j * n + k] = gs[k];
}

// Metropolis step on device.  Input slots: 0 sum Tr P^2 (old), 1 plaquette
// trace sum (old), 2 |eta|^2, 3 sum Tr P^2 (new), 4 plaquette trace sum
// (new), 5 Re <phi, X_e>.  Output: 6 H_old, 7 H_new, 8 dH, 9 u,
// 10 accepted (1/0), 11 S_g old, 12 S_g new.  S_g = beta (6V - sum/3).
__global__ void k_metropolis(uint64_t seed, uint64_t traj, double beta, double V, double* sl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double sg_old = beta * (6.0 * V - sl[1] / 3.0);
  double sg_new = beta * (6.0 * V - sl[4] / 3.0);
  double h_old = sl[0] + sg_old + sl[2];
  double h_new = sl[3] + sg_new + sl[5];
  double dh = h_new - h_old;
  uint64_t w[4];
  philox4x64_10(0, 0, ST_ACCEPT, traj, seed, 0, w);
  double u = u53(w[0]);
  bool acc = (dh == dh) && (dh <= 0.0 || u < exp(-dh));
  sl[6] = h_old;
  sl[7] = h_new;
  sl[8] = dh;
  sl[9] = u;
  sl[10] = acc ? 1.0 : 0.0;
  sl[11] = sg_old;
  sl[12] = sg_new;
}

hipError_t launch_refresh_momenta(const LatArg& g, uint64_t seed, uint64_t epoch, double* P, hipStream_t st) {
  TimedScope ts(TK_REFRESH, st, 2.0 * g.Vh * 4 * 64);
  hipLaunchKernelGGL(k_refresh_momenta, dim3(ceil_div(2LL * g.Vh, kBlock), 4), dim3(kBlock), 0, st, to_lat(g), seed,
                     epoch, P);
  return hipGetLastError();
}
hipError_t launch_weak_field(const LatArg& g, uint64_t seed, double eps, void* U, hipStream_t st) {
  hipLaunchKernelGGL(k_weak_field, dim3(ceil_div(2LL * g.Vh, kBlock)), dim3(kBlock), 0, st, to_lat(g), seed, eps, U);
  return hipGetLastError();
}
hipError_t launch_eta(const LatArg& g, uint64_t seed, uint64_t epoch, int par, void* half, hipStream_t st,
                      int second) {
  TimedScope ts(TK_REFRESH, st, (double)g.Vh * SpF64::kBytes);
  hipLaunchKernelGGL(k_eta, dim3(site_blocks(g.Vh), 3), dim3(kBlock), 0, st, to_lat(g), seed, epoch, par,
                     (double2*)half, second ? (int)ST_ETA2 : (int)ST_ETA);
  return hipGetLastError();
}
hipError_t launch_source(const LatArg& g, int kind, uint64_t seed, uint64_t epoch, void* even, void* odd,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_source, dim3(site_blocks(g.Vh), 2), dim3(kBlock), 0, st, to_lat(g), kind, seed, epoch,
                     (double2*)even, (double2*)odd);
  return hipGetLastError();
}
hipError_t launch_site_words(uint64_t seed, uint64_t stream, uint64_t epoch, const long long* sites, int nsites,
                             int nblocks, uint64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_site_words, dim3(ceil_div(nsites, kBlock)), dim3(kBlock), 0, st, seed, stream, epoch, sites,
                     nsites, nblocks, out);
  return hipGetLastError();
}
hipError_t launch_site_gaussians(uint64_t seed, uint64_t stream, uint64_t epoch, const long long* sites, int nsites,
                                 int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_site_gaussians, dim3(ceil_div(nsites, kBlock)), dim3(kBlock), 0, st, seed, stream, epoch,
                     sites, nsites, n, out);
  return hipGetLastError();
}
hipError_t launch_metropolis(uint64_t seed, uint64_t traj, double beta, double V, double* slots, hipStream_t st) {
  hipLaunchKernelGGL(k_metropolis, dim3(1), dim3(64), 0, st, seed, traj, beta, V, slots);
  return hipGetLastError();
}

}  // namespace hmc
