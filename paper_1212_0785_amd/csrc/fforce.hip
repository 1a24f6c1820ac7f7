// Wilson fermion force fused with the momentum update (the "force term
// calculation" and "projection of fields" of the paper's Sec. 1 step list).
// For S_f = phi^dag (Mhat^dag Mhat)^-1 phi with X = (X_e, D_oe X_e) and
// Y = (Mhat X_e, (D^dag)_oe Mhat X_e) on the full lattice:
//   M1 = s tr_spin[(1 - gamma_mu) X(x+mu) Y(x)^dag]
//   M2 = s tr_spin[(1 + gamma_mu) X(x) Y(x+mu)^dag]
//   F  = (i kappa^2/2) TA(U_mu(x) M1 - M2 U_mu(x)^dag).
// Because P = 1 +- gamma_mu is Hermitian with P^2 = 2P, the spin trace
// tr[P a b^dag] equals sum over the two projected components h_j(a)
// h_j(b)^dag, so each trace is two colour outer products, and
// U M1 - M2 U^dag is assembled from the colour vectors U h_j without
// forming M1, M2 or a 3x3 product.
#include "device.h"
#include "internal.h"
#include "walk.h"

namespace hmc {


struct ForceVecs {
  const void* X[2];  // by parity
  const void* Y[2];
};

// X and Y at the block's own 64 sites, parked in LDS once for the four
// direction wavefronts.
struct OwnSpinors {
  cx<double> X[12][64];
  cx<double> Y[12][64];
};

template <class LK, int MU, bool NT>
__device__ __forceinline__ void fermion_force_link(const Lat& g, const void* U, const ForceVecs& v, double* P,
                                                   double c_ta, int par, int s, bool on, OwnSpinors& own) {
  const int w = MU, lane = threadIdx.x & 63;
  Site x = cb_site(g, on ? par : 0, on ? s : 0);
  bool wr;
  const int sf = neighbour_lex<MU, +1>(g, x, &wr) >> 1;
  const double sg = (MU == 3 && wr) ? -1.0 : 1.0;
  cx<double> xn[12], yn[12], ha[6], hb[6], t[12];
  mat3<double> u;
  double c[8];
  if (on) {
    // X and Y at x + mu and this wavefront's quarter of the block's X and Y,
    // issued together (the link and the momenta follow the barrier)
    SpF64::load(v.X[par ^ 1], g.stride, sf, xn);
    SpF64::load(v.Y[par ^ 1], g.stride, sf, yn);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      own.X[3 * w + k][lane] = SpF64::load_one(v.X[par], g.stride, s, 3 * w + k);
      own.Y[3 * w + k][lane] = SpF64::load_one(v.Y[par], g.stride, s, 3 * w + k);
    }
  }
  __syncthreads();
  if (!on) return;
  // the neighbour spinors projected first (half the registers)
  cx<double> hx[6], hy[6];
  spin_project<MU, -1>(xn, hx);
  spin_project<MU, +1>(yn, hy);
  // the link and the momenta: issuing them before the barrier as well
  // raises the registers past three wavefronts per SIMD (measured slower)
  u = LK::load(U, g.stride, MU, par, s);
  double* pm = P + (size_t)(MU * 2 + par) * 8 * g.stride;
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] = gld_link<double, NT>(pm, k * g.stride + s);
  // U M1 - M2 U^dag = sg sum_j [(U hx_j) hb_j^dag - ha_j (U hy_j)^dag]
  // (M1, M2 of rank two: no 3x3 product is formed)
  cx<double> ux[6], uy[6];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      cx<double> p = u.m[3 * r] * hx[3 * j];
      p = cmadd(p, u.m[3 * r + 1], hx[3 * j + 1]);
      ux[3 * j + r] = cmadd(p, u.m[3 * r + 2], hx[3 * j + 2]);
      cx<double> q = u.m[3 * r] * hy[3 * j];
      q = cmadd(q, u.m[3 * r + 1], hy[3 * j + 1]);
      uy[3 * j + r] = cmadd(q, u.m[3 * r + 2], hy[3 * j + 2]);
    }
#pragma unroll
  for (int k = 0; k < 12; ++k) t[k] = own.Y[k][lane];
  spin_project<MU, -1>(t, hb);  // Y(x), projector (1 - gamma_mu)
#pragma unroll
  for (int k = 0; k < 12; ++k) t[k] = own.X[k][lane];
  spin_project<MU, +1>(t, ha);  // X(x), projector (1 + gamma_mu)
  mat3<double> W;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      cx<double> e = ux[r] * conj(hb[q]);
      e = cmadd(e, ux[3 + r], conj(hb[3 + q]));
      e = e - ha[r] * conj(uy[q]);
      e = e - ha[3 + r] * conj(uy[3 + q]);
      W.m[3 * r + q] = sg * e;
    }
  double f[8];
  i_ta_compact(W, c_ta, f);
#pragma unroll
  for (int k = 0; k < 8; ++k) gput<NT>(pm, k * g.stride + s, c[k] + f[k]);
}

// A block of four wavefronts covers 64 sites of one parity, wavefront w the
// links U_w (walk_site with the block as the walk unit): X and Y at the
// block's sites are read from memory once into LDS, those at the
// neighbours once per direction.
template <class LK, bool NT>
__global__ void __launch_bounds__(kBlock) k_fermion_force(Lat g, const void* U, ForceVecs v, double* P,
                                                          double c_ta) {
  __shared__ OwnSpinors own;
  int par, s;
  walk_site(g, blockIdx.x & 7, walk_unit(g, 1), &par, &s);
  const bool on = s < g.Vh;
  // the wavefront, as a scalar: each case holds exactly one barrier, which
  // every wavefront (and every work-item, on or off the lattice) reaches once
  switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
    case 0: fermion_force_link<LK, 0, NT>(g, U, v, P, c_ta, par, s, on, own); break;
    case 1: fermion_force_link<LK, 1, NT>(g, U, v, P, c_ta, par, s, on, own); break;
    case 2: fermion_force_link<LK, 2, NT>(g, U, v, P, c_ta, par, s, on, own); break;
    default: fermion_force_link<LK, 3, NT>(g, U, v, P, c_ta, par, s, on, own); break;
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
  // non-temporal link and momentum accesses (each used once) where the
  // fields outgrow the last-level cache
  const bool nt = fermion_force_stream(g);
  if (form == LINK_ROWCOL && nt)
    hipLaunchKernelGGL((k_fermion_force<LkRowCol<LkF64, true>, true>), grid, block, 0, st, lat, U, v, P, c);
  else if (form == LINK_ROWCOL)
    hipLaunchKernelGGL((k_fermion_force<LkRowCol<LkF64>, false>), grid, block, 0, st, lat, U, v, P, c);
  else if (form == LINK_ROWS2 && nt)
    hipLaunchKernelGGL((k_fermion_force<LkRows2<LkF64, true>, true>), grid, block, 0, st, lat, U, v, P, c);
  else if (form == LINK_ROWS2)
    hipLaunchKernelGGL((k_fermion_force<LkRows2<LkF64>, false>), grid, block, 0, st, lat, U, v, P, c);
  else
    hipLaunchKernelGGL((k_fermion_force<LkF64, false>), grid, block, 0, st, lat, U, v, P, c);
  return hipGetLastError();
}

}  // namespace hmc
