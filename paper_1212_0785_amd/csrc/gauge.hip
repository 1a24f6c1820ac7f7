// Gauge-field kernels of the HMC step list (Sec. 1): the plaquette / gauge
// action sum, the staple force fused with the momentum update, the link
// update exp(i eps P) U with SU(3) reunitarisation, and the kinetic sum.
// One work-item per (site, direction) for the force and the link update:
// the direction is uniform in a wavefront and resolved at compile time
// (from blockIdx.y in the direction-major forms, from the wavefront in the
// site-blocked one); one work-item per site for the sums.
#include <cstdlib>

#include "device.h"
#include "internal.h"
#include "walk.h"


namespace hmc {


// The site one step along +-MU, with coordinates.
template <int MU, int DIR>
__device__ __forceinline__ Site shift(const Lat& g, const Site& st) {
  Site n = st;
  bool w;
  n.lex = neighbour_lex<MU, DIR>(g, st, &w);
  int c = st.c[MU] + DIR;
  n.c[MU] = w ? (DIR > 0 ? 0 : g.L[MU] - 1) : c;
  return n;
}

__device__ __forceinline__ int site_parity(const Site& st) { return (st.c[0] + st.c[1] + st.c[2] + st.c[3]) & 1; }

template <class LK>
__device__ __forceinline__ mat3<double> link(const Lat& g, const void* U, int mu, const Site& st) {
  return LK::load(U, g.stride, mu, site_parity(st), st.lex >> 1);
}

// Re Tr U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
template <class LK, int MU, int NU>
__device__ __forceinline__ double plaq(const Lat& g, const void* U, const Site& x) {
  Site xm = shift<MU, +1>(g, x), xn = shift<NU, +1>(g, x);
  mat3<double> a = mmul(link<LK>(g, U, MU, x), link<LK>(g, U, NU, xm));
  // U_mu(x+nu)^dag U_nu(x)^dag = b^dag with b = U_nu(x) U_mu(x+nu)
  mat3<double> b = mmul(link<LK>(g, U, NU, x), link<LK>(g, U, MU, xn));
  // Re Tr(a b^dag) = sum_ij Re(a_ij conj(b_ij))
  double s = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) s += a.m[k].re * b.m[k].re + a.m[k].im * b.m[k].im;
  return s;
}

// x, returned through an empty asm that also "reads" the running sum sp.
__device__ __forceinline__ Site plane_site(Site x, double& sp) {
  asm volatile("" : "+v"(sp), "+v"(x.lex), "+v"(x.c[0]), "+v"(x.c[1]), "+v"(x.c[2]), "+v"(x.c[3]));
  return x;
}

// Plaquette partial sums: a block of four wavefronts covers four walk
// units, one work-item per site (all six planes), one partial per block.
template <class LK>
__global__ void __launch_bounds__(kBlock) k_plaquette_partials(Lat g, const void* U, double* part) {
  int par, s;
  walk_site(g, blockIdx.x & 7, walk_unit(g, 4) + (threadIdx.x >> 6), &par, &s);
  double v[1] = {0.0};
  if (s < g.Vh) {
    Site x = cb_site(g, par, s);
    // one plane at a time: the site of each plane passes through an empty
    // asm that also takes the running sum, so the loads of a plane cannot
    // be issued before the previous plane is done (all 24 links in flight
    // at once exceed the register file)
    double sp = 0.0;
    sp += plaq<LK, 0, 1>(g, U, plane_site(x, sp));
    sp += plaq<LK, 0, 2>(g, U, plane_site(x, sp));
    sp += plaq<LK, 0, 3>(g, U, plane_site(x, sp));
    sp += plaq<LK, 1, 2>(g, U, plane_site(x, sp));
    sp += plaq<LK, 1, 3>(g, U, plane_site(x, sp));
    sp += plaq<LK, 2, 3>(g, U, plane_site(x, sp));
    v[0] = sp;
  }
  block_sum<1>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(kBlock) k_kinetic_partials(Lat g, const double* P, double* part) {
  double v[1] = {0.0};
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < 2 * g.Vh; j += gridDim.x * kBlock) {
    int par = j >= g.Vh, s = j - par * g.Vh;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      double c[8];
      load_compact(P, g.stride, mu, par, s, c);
      double p22 = -c[0] - c[1];
      v[0] += c[0] * c[0] + c[1] * c[1] + p22 * p22 +
              2.0 * (c[2] * c[2] + c[3] * c[3] + c[4] * c[4] + c[5] * c[5] + c[6] * c[6] + c[7] * c[7]);
    }
  }
  block_sum<1>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Orders the loads of successive staples after the accumulation of the
// previous one (see the same device in the Dslash): without it all 19 link
// loads of a (site, direction) are issued at once and the kernel spills.
__device__ __forceinline__ void chain_sites(Site& x, Site& xm, mat3<double>& A) {
#pragma unroll
  for (int k = 0; k < 9; ++k) asm volatile("" : "+v"(A.m[k].re), "+v"(A.m[k].im));
  asm volatile("" : "+v"(x.lex), "+v"(xm.lex));
}

// Staple pair of plane (MU, NU) for the link U_mu(x):
//   U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
// Same for the third link of a staple: its load waits for the product of
// the first two, so at most two links are in registers at a time.
__device__ __forceinline__ void chain_site(Site& x, mat3<double>& t) {
#pragma unroll
  for (int k = 0; k < 9; ++k) asm volatile("" : "+v"(t.m[k].re), "+v"(t.m[k].im));
  asm volatile("" : "+v"(x.lex));
}

// ---- staple pair on SU(3) links (the compact link forms).  Each staple
// and each partial product of two links is itself in SU(3), so two of its
// rows (or columns) fix the third as conj(row0 x row1) (conj(col0 x col1)):
// the products below form two rows or columns and rebuild the rest, which
// also spares rebuilding row 2 of the links that only enter through their
// first two rows.

template <class LK>
__device__ __forceinline__ mat3<double> link2(const Lat& g, const void* U, int mu, const Site& st) {
  return LK::load2(U, g.stride, mu, site_parity(st), st.lex >> 1);
}


// rows 0, 1 of r = a b (a: rows 0, 1; b: all rows)
__device__ __forceinline__ void mul_r01(const mat3<double>& a, const mat3<double>& b, mat3<double>& r) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> t = a.m[3 * i] * b.m[j];
      t = cmadd(t, a.m[3 * i + 1], b.m[3 + j]);
      r.m[3 * i + j] = cmadd(t, a.m[3 * i + 2], b.m[6 + j]);
    }
}

// rows 0, 1 of r = a b^dag (a: rows 0, 1; b: all rows)
__device__ __forceinline__ void mul_r01_nd(const mat3<double>& a, const mat3<double>& b, mat3<double>& r) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> t = a.m[3 * i] * conj(b.m[3 * j]);
      t = cmadd(t, a.m[3 * i + 1], conj(b.m[3 * j + 1]));
      r.m[3 * i + j] = cmadd(t, a.m[3 * i + 2], conj(b.m[3 * j + 2]));
    }
}

// columns 0, 1 of r = a^dag b (a: all rows; b: columns 0, 1)
__device__ __forceinline__ void mul_c01_dn(const mat3<double>& a, const mat3<double>& b, mat3<double>& r) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cx<double> t = cmadd_conj(cx<double>{0, 0}, a.m[i], b.m[j]);
      t = cmadd_conj(t, a.m[3 + i], b.m[3 + j]);
      r.m[3 * i + j] = cmadd_conj(t, a.m[6 + i], b.m[6 + j]);
    }
}

// acc + conj(a b - c d)
__device__ __forceinline__ cx<double> acc_conj_cross(cx<double> acc, cx<double> a, cx<double> b, cx<double> c,
                                                     cx<double> d) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.re = fma(-c.re, d.re, acc.re);
  acc.re = fma(c.im, d.im, acc.re);
  acc.im = fma(-a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
  acc.im = fma(c.re, d.im, acc.im);
  acc.im = fma(c.im, d.re, acc.im);
  return acc;
}

// Plaquette sum on SU(3) links, plane-paired: a block of three wavefronts
// covers one walk unit (64 sites of one parity); wavefront w takes the
// planes (0, w+1) and its complement, which together hold each direction
// once.  The block first parks rows 0 and 1 of its 256 own links U_mu(x)
// in LDS (each enters three planes); each wavefront issues the loads of the
// four links of its two planes that sit at x + mu and x + nu together, so
// twice the memory requests of a one-plane wavefront are in flight at the
// same occupancy (the sum is bound by the latency of those loads, not by
// its arithmetic or bandwidth).  With a = U_mu(x) U_nu(x+mu) and
// b = U_nu(x) U_mu(x+nu) both in SU(3), only rows 0 and 1 of each product
// are formed: with h_ij = sum_k conj(a_ik) b_jk, row 2 of each is the
// conjugate cross product of its rows 0 and 1, and the Binet-Cauchy
// identity gives its part of Re Tr(a b^dag) as Re(h00 h11 - h01 h10).
constexpr int kPlaqPairThreads = 3 * 64;

template <class LK, int MU, int NU>
__device__ __forceinline__ double plaq_rows(const cx<double> (*own)[6][64], int lane, const mat3<double>& B,
                                            const mat3<double>& C) {
  mat3<double> A, D, a, b;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    A.m[k] = own[MU][k][lane];
    D.m[k] = own[NU][k][lane];
  }
  mul_r01(A, B, a);  // rows 0, 1 of U_mu(x) U_nu(x+mu)
  mul_r01(D, C, b);  // rows 0, 1 of U_nu(x) U_mu(x+nu)
  cx<double> h[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cx<double> t = cmadd_conj(cx<double>{0, 0}, a.m[3 * i], b.m[3 * j]);
      t = cmadd_conj(t, a.m[3 * i + 1], b.m[3 * j + 1]);
      h[i][j] = cmadd_conj(t, a.m[3 * i + 2], b.m[3 * j + 2]);
    }
  const cx<double> d = h[0][0] * h[1][1] - h[0][1] * h[1][0];
  return h[0][0].re + h[1][1].re + d.re;
}

template <class LK, int M1, int N1, int M2, int N2>
__device__ __forceinline__ double plaq_pair(const Lat& g, const void* U, const Site& x, cx<double> (*own)[6][64],
                                            int w, int lane, int par, int s, bool on) {
  mat3<double> B1, C1, B2, C2;
  if (on) {
    B1 = link2<LK>(g, U, N1, shift<M1, +1>(g, x));
    C1 = link2<LK>(g, U, M1, shift<N1, +1>(g, x));
    B2 = link2<LK>(g, U, N2, shift<M2, +1>(g, x));
    C2 = link2<LK>(g, U, M2, shift<N2, +1>(g, x));
    {
      const mat3<double> u = LK::load2(U, g.stride, w + 1, par, s);
#pragma unroll
      for (int k = 0; k < 6; ++k) own[w + 1][k][lane] = u.m[k];
    }
    if (w == 0) {
      const mat3<double> u = LK::load2(U, g.stride, 0, par, s);
#pragma unroll
      for (int k = 0; k < 6; ++k) own[0][k][lane] = u.m[k];
    }
  }
  __syncthreads();
  if (!on) return 0.0;
  third_row(B1);
  third_row(C1);
  const double p1 = plaq_rows<LK, M1, N1>(own, lane, B1, C1);
  third_row(B2);
  third_row(C2);
  return p1 + plaq_rows<LK, M2, N2>(own, lane, B2, C2);
}

template <class LK>
__global__ void __launch_bounds__(kPlaqPairThreads) k_plaquette_pairs(Lat g, const void* U, double* part) {
  int par, s;
  walk_site(g, blockIdx.x & 7, walk_unit(g, 1), &par, &s);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const bool on = s < g.Vh;
  __shared__ cx<double> own[4][6][64];
  const Site x = cb_site(g, on ? par : 0, on ? s : 0);
  double v[1];
  // w is uniform over a wavefront; each case holds exactly one barrier,
  // which every wavefront (and every work-item, on or off the lattice)
  // reaches once
  switch (w) {
    case 0: v[0] = plaq_pair<LK, 0, 1, 2, 3>(g, U, x, own, w, lane, par, s, on); break;
    case 1: v[0] = plaq_pair<LK, 0, 2, 1, 3>(g, U, x, own, w, lane, par, s, on); break;
    default: v[0] = plaq_pair<LK, 0, 3, 1, 2>(g, U, x, own, w, lane, par, s, on); break;
  }
  block_sum<1, 3>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Rows 0 and 1 of the links U_mu(x) and U_mu(x-mu) of a block's 64 sites,
// parked in LDS by the site-blocked staple force: the wavefront of
// direction mu needs U_nu(x) of the other three directions in its upper
// staples (and its own link at the end) and U_nu(x-nu) in its lower ones,
// which the block has then read from memory once instead of three times.
struct OwnLinks {
  cx<double> m[4][6][64];     // U_mu(x)
  cx<double> back[4][6][64];  // U_mu(x - mu)
};

__device__ __forceinline__ mat3<double> own_link(const OwnLinks& o, int mu, int lane) {
  mat3<double> u;
#pragma unroll
  for (int k = 0; k < 6; ++k) u.m[k] = o.m[mu][k][lane];
  return u;
}
__device__ __forceinline__ mat3<double> back_link(const OwnLinks& o, int mu, int lane) {
  mat3<double> u;
#pragma unroll
  for (int k = 0; k < 6; ++k) u.m[k] = o.back[mu][k][lane];
  return u;
}

// A link of the site-blocked walk, whose sites of one parity make the
// parity of every neighbour uniform over the wavefront (scalar array
// bases, LK::load_u); the other forms take it from the site.
template <class LK, bool UNI>
__device__ __forceinline__ mat3<double> slink(const Lat& g, const void* U, int mu, const Site& st, int par) {
  if constexpr (UNI)
    return LK::load_u(U, g.stride, mu, par, st.lex >> 1);
  else
    return link<LK>(g, U, mu, st);
}
template <class LK, bool UNI>
__device__ __forceinline__ mat3<double> slink2(const Lat& g, const void* U, int mu, const Site& st, int par) {
  if constexpr (UNI)
    return LK::load2_u(U, g.stride, mu, par, st.lex >> 1);
  else
    return link2<LK>(g, U, mu, st);
}

// par: the parity of x (used where OWN: the site-blocked walk)
template <class LK, int MU, int NU, bool OWN>
__device__ __forceinline__ void add_staples_su3(const Lat& g, const void* U, Site x, Site xm, mat3<double>& A,
                                                const OwnLinks* own, int lane, int par) {
  const int po = par ^ 1;
  chain_sites(x, xm, A);
  {
    // upper: U_nu(x+mu) (U_nu(x) U_mu(x+nu))^dag
    Site xn = shift<NU, +1>(g, x);
    mat3<double> C;
    if constexpr (OWN)
      C = own_link(*own, NU, lane);
    else
      C = link2<LK>(g, U, NU, x);
    mat3<double> D;
    mul_r01(C, slink<LK, OWN>(g, U, MU, xn, po), D);
    third_row(D);
    chain_site(xm, D);
    mat3<double> S;
    mul_r01_nd(slink2<LK, OWN>(g, U, NU, xm, po), D, S);
#pragma unroll
    for (int k = 0; k < 6; ++k) A.m[k] = A.m[k] + S.m[k];
    A.m[6] = acc_conj_cross(A.m[6], S.m[1], S.m[5], S.m[2], S.m[4]);
    A.m[7] = acc_conj_cross(A.m[7], S.m[2], S.m[3], S.m[0], S.m[5]);
    A.m[8] = acc_conj_cross(A.m[8], S.m[0], S.m[4], S.m[1], S.m[3]);
  }
  chain_sites(x, xm, A);
  {
    // lower: (U_mu(x-nu) U_nu(x+mu-nu))^dag U_nu(x-nu)
    Site xmn = shift<NU, -1>(g, xm), xn = shift<NU, -1>(g, x);
    mat3<double> H;
    mul_r01(slink2<LK, OWN>(g, U, MU, xn, po), slink<LK, OWN>(g, U, NU, xmn, par), H);
    third_row(H);
    chain_site(xn, H);
    mat3<double> G;
    if constexpr (OWN)
      G = back_link(*own, NU, lane);
    else
      G = link2<LK>(g, U, NU, xn);
    G.m[6] = conj(G.m[1] * G.m[5] - G.m[2] * G.m[4]);  // row 2, columns 0 and 1
    G.m[7] = conj(G.m[2] * G.m[3] - G.m[0] * G.m[5]);
    mat3<double> S;
    mul_c01_dn(H, G, S);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      A.m[3 * i] = A.m[3 * i] + S.m[3 * i];
      A.m[3 * i + 1] = A.m[3 * i + 1] + S.m[3 * i + 1];
    }
    A.m[2] = acc_conj_cross(A.m[2], S.m[3], S.m[7], S.m[6], S.m[4]);
    A.m[5] = acc_conj_cross(A.m[5], S.m[6], S.m[1], S.m[0], S.m[7]);
    A.m[8] = acc_conj_cross(A.m[8], S.m[0], S.m[4], S.m[3], S.m[1]);
  }
}

template <class LK, int MU, int NU, bool OWN = false>
__device__ __forceinline__ void add_staples(const Lat& g, const void* U, Site x, Site xm, mat3<double>& A,
                                            const OwnLinks* own = nullptr, int lane = 0, int par = 0) {
  if constexpr (CompactLinks<LK>::value) {
    add_staples_su3<LK, MU, NU, OWN>(g, U, x, xm, A, own, lane, par);
    return;
  }
  chain_sites(x, xm, A);
  {
    Site xn = shift<NU, +1>(g, x);
    mat3<double> t = mmul_nd(link<LK>(g, U, NU, xm), link<LK>(g, U, MU, xn));
    chain_site(x, t);
    A = madd(A, mmul_nd(t, link<LK>(g, U, NU, x)));
  }
  chain_sites(x, xm, A);
  {
    Site xmn = shift<NU, -1>(g, xm), xn = shift<NU, -1>(g, x);
    // U_nu(x+mu-nu)^dag U_mu(x-nu)^dag = (U_mu(x-nu) U_nu(x+mu-nu))^dag
    mat3<double> ba = mmul(link<LK>(g, U, MU, xn), link<LK>(g, U, NU, xmn));
    chain_site(xn, ba);
    A = madd(A, mmul_dn(ba, link<LK>(g, U, NU, xn)));
  }
}

// P_mu(x) += (i coef beta / 12) TA(U_mu(x) A), A the staple sum: with
// F = -(i beta / 12) TA(W) this is P <- P - coef F.
template <class LK, int MU, bool OWN = false, bool NT = false>
__device__ __forceinline__ void gauge_force_finish(const Lat& g, const void* U, double* P, double coef_beta, int par,
                                                   int s, const mat3<double>& A, const OwnLinks* own = nullptr,
                                                   int lane = 0) {
  mat3<double> u;
  if constexpr (OWN) {
    u = own_link(*own, MU, lane);
    third_row(u);
  } else {
    u = LK::load(U, g.stride, MU, par, s);
  }
  mat3<double> W = mmul(u, A);
  double f[8], c[8];
  i_ta_compact(W, coef_beta / 12.0, f);
  // NT: non-temporal momentum accesses (each read and written once)
  double* pm = P + (size_t)(MU * 2 + par) * 8 * g.stride;
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] = gld_link<double, NT>(pm, k * g.stride + s);
#pragma unroll
  for (int k = 0; k < 8; ++k) gput<NT>(pm, k * g.stride + s, c[k] + f[k]);
}

template <class LK, int MU, bool OWN = false, bool NT = false>
__device__ __forceinline__ void gauge_force_link(const Lat& g, const void* U, double* P, double coef_beta, int par,
                                                 int s, const OwnLinks* own = nullptr, int lane = 0) {
  Site x = cb_site(g, par, s);
  Site xm = shift<MU, +1>(g, x);
  mat3<double> A;
#pragma unroll
  for (int k = 0; k < 9; ++k) A.m[k] = {0.0, 0.0};
  if (MU != 0) add_staples<LK, MU, 0, OWN>(g, U, x, xm, A, own, lane, par);
  if (MU != 1) add_staples<LK, MU, 1, OWN>(g, U, x, xm, A, own, lane, par);
  if (MU != 2) add_staples<LK, MU, 2, OWN>(g, U, x, xm, A, own, lane, par);
  if (MU != 3) add_staples<LK, MU, 3, OWN>(g, U, x, xm, A, own, lane, par);
  gauge_force_finish<LK, MU, OWN, NT>(g, U, P, coef_beta, par, s, A, own, lane);
}

template <class LK>
__global__ void __launch_bounds__(kBlock) k_gauge_force(Lat g, const void* U, double* P, double coef_beta) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= 2 * g.Vh) return;
  int par = j >= g.Vh, s = j - par * g.Vh;
  switch (blockIdx.y) {
    case 0: gauge_force_link<LK, 0>(g, U, P, coef_beta, par, s); break;
    case 1: gauge_force_link<LK, 1>(g, U, P, coef_beta, par, s); break;
    case 2: gauge_force_link<LK, 2>(g, U, P, coef_beta, par, s); break;
    default: gauge_force_link<LK, 3>(g, U, P, coef_beta, par, s); break;
  }
}

// Site-blocked form: a block of four wavefronts covers 64 sites of one
// parity, wavefront w the links U_w of those sites (walk_site with the
// block as the walk unit).  With compact (SU(3)) links the block first
// parks rows 0 and 1 of its 256 own links and of the 256 links U_mu(x-mu)
// in LDS (48 KB), which the wavefronts read for their staples and for the
// final product instead of loading each three times.
template <class LK, bool NT>
__global__ void __launch_bounds__(kBlock) k_gauge_force_sites(Lat g, const void* U, double* P, double coef_beta) {
  int par, s;
  walk_site(g, blockIdx.x & 7, walk_unit(g, 1), &par, &s);
  par = __builtin_amdgcn_readfirstlane(par);  // one parity per walk unit
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // the wavefront (direction), as a scalar
  if constexpr (CompactLinks<LK>::value) {
    // each wavefront parks rows 0 and 1 of its own links; every work-item
    // reaches the barrier
    __shared__ OwnLinks own;
    const int lane = threadIdx.x & 63;
    if (s < g.Vh) {
      const Site x = cb_site(g, par, s);
      const mat3<double> u = LK::load2_u(U, g.stride, w, par, s);
      Site xb;
      switch (w) {
        case 0: xb = shift<0, -1>(g, x); break;
        case 1: xb = shift<1, -1>(g, x); break;
        case 2: xb = shift<2, -1>(g, x); break;
        default: xb = shift<3, -1>(g, x); break;
      }
      const mat3<double> ub = LK::load2_u(U, g.stride, w, par ^ 1, xb.lex >> 1);
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        own.m[w][k][lane] = u.m[k];
        own.back[w][k][lane] = ub.m[k];
      }
    }
    __syncthreads();
    if (s >= g.Vh) return;
    switch (w) {
      case 0: gauge_force_link<LK, 0, true, NT>(g, U, P, coef_beta, par, s, &own, lane); break;
      case 1: gauge_force_link<LK, 1, true, NT>(g, U, P, coef_beta, par, s, &own, lane); break;
      case 2: gauge_force_link<LK, 2, true, NT>(g, U, P, coef_beta, par, s, &own, lane); break;
      default: gauge_force_link<LK, 3, true, NT>(g, U, P, coef_beta, par, s, &own, lane); break;
    }
    return;
  }
  if (s >= g.Vh) return;
  switch (w) {
    case 0: gauge_force_link<LK, 0>(g, U, P, coef_beta, par, s); break;
    case 1: gauge_force_link<LK, 1>(g, U, P, coef_beta, par, s); break;
    case 2: gauge_force_link<LK, 2>(g, U, P, coef_beta, par, s); break;
    default: gauge_force_link<LK, 3>(g, U, P, coef_beta, par, s); break;
  }
}

// Plane-split form: a block of three wavefronts covers 64 links of one
// direction MU; wavefront w sums the two staples of the w-th plane (MU, NU)
// and parks them in LDS; after a barrier the first wavefront adds the three
// planes in a fixed order and finishes the 64 links.  Three times the
// wavefronts of the one-link-per-work-item kernel with a third of its
// serial load chain.
constexpr int kGfSites = 64;

template <class LK, int MU, int W>
__device__ __forceinline__ void plane_staples(const Lat& g, const void* U, const Site& x, const Site& xm,
                                              mat3<double>& A) {
  constexpr int NU = W < MU ? W : W + 1;  // the W-th direction other than MU
  add_staples<LK, MU, NU>(g, U, x, xm, A);
}

template <class LK, int MU>
__device__ __forceinline__ void gauge_force_planes(const Lat& g, const void* U, double* P, double coef_beta,
                                                   cx<double> (*part)[9][kGfSites]) {
  const int w = threadIdx.x >> 6, ls = threadIdx.x & 63;
  const int j = blockIdx.x * kGfSites + ls;
  const bool active = j < 2 * g.Vh;
  const int par = j >= g.Vh, s = j - par * g.Vh;
  {
    mat3<double> A;
#pragma unroll
    for (int k = 0; k < 9; ++k) A.m[k] = {0.0, 0.0};
    if (active) {
      const Site x = cb_site(g, par, s);
      const Site xm = shift<MU, +1>(g, x);
      switch (w) {
        case 0: plane_staples<LK, MU, 0>(g, U, x, xm, A); break;
        case 1: plane_staples<LK, MU, 1>(g, U, x, xm, A); break;
        default: plane_staples<LK, MU, 2>(g, U, x, xm, A); break;
      }
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) part[w][k][ls] = A.m[k];
  }
  __syncthreads();
  if (w != 0 || !active) return;
  mat3<double> A;
#pragma unroll
  for (int k = 0; k < 9; ++k) A.m[k] = part[0][k][ls] + part[1][k][ls] + part[2][k][ls];
  gauge_force_finish<LK, MU>(g, U, P, coef_beta, par, s, A);
}

template <class LK>
__global__ void __launch_bounds__(3 * kGfSites) k_gauge_force_planes(Lat g, const void* U, double* P,
                                                                     double coef_beta) {
  __shared__ cx<double> part[3][9][kGfSites];
  switch (blockIdx.y) {
    case 0: gauge_force_planes<LK, 0>(g, U, P, coef_beta, part); break;
    case 1: gauge_force_planes<LK, 1>(g, U, P, coef_beta, part); break;
    case 2: gauge_force_planes<LK, 2>(g, U, P, coef_beta, part); break;
    default: gauge_force_planes<LK, 3>(g, U, P, coef_beta, part); break;
  }
}

// U <- reunit(exp(i eps P) U), one link per work-item.  The reunitarisation
// uses rows 0 and 1 of the product only, so on SU(3) links LK reads rows 0
// and 1 of U and rebuilds row 2 (which the product needs) from them; the
// full link is written.  NT: non-temporal loads of P and U and stores of U
// (each touched once; on large lattices they would only displace other
// data from the caches).
template <class LK, bool NT>
__global__ void __launch_bounds__(kBlock) k_exp_update(Lat g, void* U, const double* P, double eps) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= 2 * g.Vh) return;
  int par = j >= g.Vh, s = j - par * g.Vh;
  int mu = blockIdx.y;
  double c[8];
  {
    const double* p = P + (size_t)(mu * 2 + par) * 8 * g.stride;
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = gld_link<double, NT>(p, k * g.stride + s);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] *= eps;
  mat3<double> E = exp_iQ(herm_from_compact(c));
  mat3<double> u = mmul(E, LK::load(U, g.stride, mu, par, s));
  reunitarise(u);
  void* q = (char*)U + (size_t)(mu * 2 + par) * 9 * g.stride * sizeof(v2d);
#pragma unroll
  for (int k = 0; k < 9; ++k) gput<NT>(q, k * g.stride + s, v2d{u.m[k].re, u.m[k].im});
}

int plaquette_blocks(const LatArg& g, bool su3) {
  if (su3 && plaquette_shape(g) == 1) return 2 * ceil_div(g.Vh, 64);
  return tiled_order_valid(g) ? g.Vh / 128 : ceil_div(2 * ceil_div(g.Vh, 64), 4);
}

hipError_t launch_plaquette_partials(const LatArg& g, const void* U, double* part, hipStream_t st, bool su3) {
  const int form = link_form_for(su3, plaquette_link_form(g));
  const int lb = form == LINK_ROWCOL ? LkRowCol<LkF64>::kBytes : form == LINK_ROWS2 ? LkRows2<LkF64>::kBytes
                                                                                     : LkF64::kBytes;
  TimedScope ts(TK_PLAQUETTE, st, 2.0 * g.Vh * 4 * LkF64::kBytes, 2.0 * g.Vh * 4 * lb);
  const dim3 grid(plaquette_blocks(g, su3)), block(kBlock);
  const Lat lat = walk_lat(g);
  if (su3 && plaquette_shape(g) == 1) {
    if (form == LINK_ROWCOL)
      hipLaunchKernelGGL(k_plaquette_pairs<LkRowCol<LkF64>>, grid, dim3(kPlaqPairThreads), 0, st, lat, U, part);
    else
      hipLaunchKernelGGL(k_plaquette_pairs<LkRows2<LkF64>>, grid, dim3(kPlaqPairThreads), 0, st, lat, U, part);
  } else if (form == LINK_ROWCOL)
    hipLaunchKernelGGL(k_plaquette_partials<LkRowCol<LkF64>>, grid, block, 0, st, lat, U, part);
  else if (form == LINK_ROWS2)
    hipLaunchKernelGGL(k_plaquette_partials<LkRows2<LkF64>>, grid, block, 0, st, lat, U, part);
  else
    hipLaunchKernelGGL(k_plaquette_partials<LkF64>, grid, block, 0, st, lat, U, part);
  return hipGetLastError();
}

hipError_t launch_kinetic_partials(const LatArg& g, const double* P, double* part, int nb, hipStream_t st) {
  TimedScope ts(TK_REDUCE, st, 2.0 * g.Vh * 4 * 64);
  hipLaunchKernelGGL(k_kinetic_partials, dim3(nb), dim3(kBlock), 0, st, to_lat(g), P, part);
  return hipGetLastError();
}

template <class LK>
static void gauge_force_typed(const LatArg& g, const void* U, double* P, double coef_beta, hipStream_t st, int shape) {
  if (shape == 2) {
    if (gauge_force_stream(g))
      hipLaunchKernelGGL((k_gauge_force_sites<LK, true>), dim3(2 * ceil_div(g.Vh, 64)), dim3(kBlock), 0, st,
                         walk_lat(g), U, P, coef_beta);
    else
      hipLaunchKernelGGL((k_gauge_force_sites<LK, false>), dim3(2 * ceil_div(g.Vh, 64)), dim3(kBlock), 0, st,
                         walk_lat(g), U, P, coef_beta);
  } else if (shape == 1)
    hipLaunchKernelGGL(k_gauge_force_planes<LK>, dim3(ceil_div(2LL * g.Vh, kGfSites), 4), dim3(3 * kGfSites), 0, st,
                       to_lat(g), U, P, coef_beta);
  else
    hipLaunchKernelGGL(k_gauge_force<LK>, dim3(ceil_div(2LL * g.Vh, kBlock), 4), dim3(kBlock), 0, st, to_lat(g), U,
                       P, coef_beta);
}

hipError_t launch_gauge_force(const LatArg& g, const void* U, double* P, double coef_beta, hipStream_t st,
                              bool su3, int shape, int form) {
  if (shape < 0) shape = gauge_force_shape(g);
  form = link_form_for(su3, form ? form : staple_link_form(g));
  const int lb = form == LINK_ROWCOL ? LkRowCol<LkF64>::kBytes : form == LINK_ROWS2 ? LkRows2<LkF64>::kBytes
                                                                                     : LkF64::kBytes;
  // per site: 4 links read, momenta read + written
  TimedScope ts(TK_GAUGE_FORCE, st, 2.0 * g.Vh * (4 * LkF64::kBytes + 2 * 4 * 64), 2.0 * g.Vh * (4 * lb + 2 * 4 * 64));
  if (form == LINK_ROWCOL)
    gauge_force_typed<LkRowCol<LkF64>>(g, U, P, coef_beta, st, shape);
  else if (form == LINK_ROWS2)
    gauge_force_typed<LkRows2<LkF64>>(g, U, P, coef_beta, st, shape);
  else
    gauge_force_typed<LkF64>(g, U, P, coef_beta, st, shape);
  return hipGetLastError();
}

hipError_t launch_exp_update(const LatArg& g, void* U, const double* P, double eps, hipStream_t st, bool su3) {
  // per link: read (two rows on SU(3) links) and written, momenta read
  const int rb = su3 ? LkRows2<LkF64>::kBytes : LkF64::kBytes;
  TimedScope ts(TK_EXP_UPDATE, st, 2.0 * g.Vh * 4 * (2 * LkF64::kBytes + 64), 2.0 * g.Vh * 4 * (rb + LkF64::kBytes + 64));
  const dim3 grid(ceil_div(2LL * g.Vh, kBlock), 4), block(kBlock);
  const bool nt = exp_update_stream(g);
  if (su3 && nt)
    hipLaunchKernelGGL((k_exp_update<LkRows2<LkF64, true>, true>), grid, block, 0, st, to_lat(g), U, P, eps);
  else if (su3)
    hipLaunchKernelGGL((k_exp_update<LkRows2<LkF64>, false>), grid, block, 0, st, to_lat(g), U, P, eps);
  else
    hipLaunchKernelGGL((k_exp_update<LkF64, false>), grid, block, 0, st, to_lat(g), U, P, eps);
  return hipGetLastError();
}

}  // namespace hmc
