// Wilson fermion force fused with the momentum update (the "force term
// calculation" and "projection of fields" of the paper's Sec. 1 step list).
// For S_f = phi^dag (Mhat^dag Mhat)^-1 phi with X = (X_e, D_oe X_e) and
// Y = (Mhat X_e, (D^dag)_oe Mhat X_e) on the full lattice:
//   M1 = s tr_spin[(1 - gamma_mu) X(x+mu) Y(x)^dag]
//   M2 = s tr_spin[(1 + gamma_mu) X(x) Y(x+mu)^dag]
//   F  = (i kappa^2/2) TA(U_mu(x) M1 - M2 U_mu(x)^dag).
// Because P = 1 +- gamma_mu is Hermitian with P^2 = 2P, the spin trace
// tr[P a b^dag] equals sum over the two projected components h_j(a)
// h_j(b)^dag, so each trace is two colour outer products.
#include "device.h"
#include "internal.h"
#include "walk.h"

namespace hmc {


struct ForceVecs {
  const void* X[2];  // by parity
  const void* Y[2];
};

// sg * sum_{j=0,1} h_j(a) h_j(b)^dag for projected half spinors ha, hb.
__device__ __forceinline__ mat3<double> proj_outer(const cx<double>* ha, const cx<double>* hb, double sg) {
  mat3<double> m;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cx<double> v = ha[r] * conj(hb[c]);
      v = cmadd(v, ha[3 + r], conj(hb[3 + c]));
      m.m[3 * r + c] = sg * v;
    }
  return m;
}

template <class LK, int MU>
__device__ __forceinline__ void fermion_force_link(const Lat& g, const void* U, const ForceVecs& v, double* P,
                                                   double c_ta, int par, int s) {
  Site x = cb_site(g, par, s);
  bool w;
  const int sf = neighbour_lex<MU, +1>(g, x, &w) >> 1;
  const double sg = (MU == 3 && w) ? -1.0 : 1.0;
  cx<double> a[12], b[12], ha[6], hb[6];
  // M1 from X(x+mu) and Y(x), projector (1 - gamma_mu)
  SpF64::load(v.X[par ^ 1], g.stride, sf, a);
  SpF64::load(v.Y[par], g.stride, s, b);
  spin_project<MU, -1>(a, ha);
  spin_project<MU, -1>(b, hb);
  mat3<double> M1 = proj_outer(ha, hb, sg);
  // M2 from X(x) and Y(x+mu), projector (1 + gamma_mu)
  SpF64::load(v.X[par], g.stride, s, a);
  SpF64::load(v.Y[par ^ 1], g.stride, sf, b);
  spin_project<MU, +1>(a, ha);
  spin_project<MU, +1>(b, hb);
  mat3<double> M2 = proj_outer(ha, hb, sg);
  mat3<double> u = LK::load(U, g.stride, MU, par, s);
  mat3<double> W = msub(mmul(u, M1), mmul_nd(M2, u));
  double f[8], c[8];
  i_ta_compact(W, c_ta, f);
  load_compact(P, g.stride, MU, par, s, c);
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] += f[k];
  store_compact(P, g.stride, MU, par, s, c);
}

// A block of four wavefronts covers 64 sites of one parity, wavefront w the
// links U_w (walk_site with the block as the walk unit), so X and Y at a
// site and its neighbours are fetched once for all four directions.
template <class LK>
__global__ void __launch_bounds__(kBlock) k_fermion_force(Lat g, const void* U, ForceVecs v, double* P,
                                                          double c_ta) {
  int par, s;
  walk_site(g, blockIdx.x & 7, walk_unit(g, 1), &par, &s);
  if (s >= g.Vh) return;
  switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {  // the wavefront, as a scalar
    case 0: fermion_force_link<LK, 0>(g, U, v, P, c_ta, par, s); break;
    case 1: fermion_force_link<LK, 1>(g, U, v, P, c_ta, par, s); break;
    case 2: fermion_force_link<LK, 2>(g, U, v, P, c_ta, par, s); break;
    default: fermion_force_link<LK, 3>(g, U, v, P, c_ta, par, s); break;
  }
}

// P <- P - coef * F_f with F_f = (i kappa^2 / 2) TA(W): the kernel adds
// i c_ta TA(W) with c_ta = -coef kappa^2 / 2 (coef passed already times
// kappa^2 by the caller as `coef`).
hipError_t launch_fermion_force(const LatArg& g, const void* U, const void* Xe, const void* Xo, const void* Ye,
                                const void* Yo, double* P, double coef, hipStream_t st, bool su3) {
  // the link form of the FP64 hop kernels (same per-link work pattern)
  const int form = link_form_for(su3, dslash_link_form(g, HMC_F64));
  const int lb = form == LINK_ROWCOL ? LkRowCol<LkF64>::kBytes : form == LINK_ROWS2 ? LkRows2<LkF64>::kBytes
                                                                                     : LkF64::kBytes;
  // per site: 4 links, X and Y (both read once), momenta read + written
  TimedScope ts(TK_FERMION_FORCE, st, 2.0 * g.Vh * (4 * LkF64::kBytes + 2 * SpF64::kBytes + 2 * 4 * 64),
                2.0 * g.Vh * (4 * lb + 2 * SpF64::kBytes + 2 * 4 * 64));
  ForceVecs v;
  v.X[0] = Xe;
  v.X[1] = Xo;
  v.Y[0] = Ye;
  v.Y[1] = Yo;
  const dim3 grid(2 * ceil_div(g.Vh, 64)), block(kBlock);
  const double c = -0.5 * coef;
  const Lat lat = walk_lat(g);
  if (form == LINK_ROWCOL)
    hipLaunchKernelGGL(k_fermion_force<LkRowCol<LkF64>>, grid, block, 0, st, lat, U, v, P, c);
  else if (form == LINK_ROWS2)
    hipLaunchKernelGGL(k_fermion_force<LkRows2<LkF64>>, grid, block, 0, st, lat, U, v, P, c);
  else
    hipLaunchKernelGGL(k_fermion_force<LkF64>, grid, block, 0, st, lat, U, v, P, c);
  return hipGetLastError();
}

}  // namespace hmc
