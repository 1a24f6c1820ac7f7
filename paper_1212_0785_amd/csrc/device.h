// Device-side building blocks of the gfx950 Wilson-HMC library: complex and
// SU(3) arithmetic, the structure-of-arrays storage formats, checkerboard
// geometry, Philox4x64-10 and deterministic block reductions.
//
// Site mapping follows the one-thread-per-site parallelisation of the
// paper's Sec. 3 (outer level of the QDP++ tensor structure on threads):
// a work-item owns one checkerboard site, its spin/colour/complex levels
// stay in registers.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace hmc {

// Global-memory pointer qualifier: field pointers read from argument structs
// are otherwise generic, which costs flat loads and 64-bit vector addressing.
#define HMC_GLOBAL __attribute__((address_space(1)))

// Native clang vectors (usable in an explicit address space, unlike HIP's
// class vector types).
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef _Float16 v2h __attribute__((ext_vector_type(2)));

constexpr int kBlock = 256;  // work-items per block (4 wave64)

// Element `idx` of a global array of T addressed as base + 32-bit byte
// offset (the scalar-base + vector-offset form of global loads).  Every
// field component array here is below 4 GiB.
template <typename T>
__device__ __forceinline__ const HMC_GLOBAL T& gld(const void* base, unsigned idx) {
  return *(const HMC_GLOBAL T*)((const HMC_GLOBAL char*)base + idx * (unsigned)sizeof(T));
}
// Same, with the non-temporal hint when NT (data used once per sweep, which
// then leaves the caches to data that is reused).
template <typename T, bool NT = false>
__device__ __forceinline__ T gld_link(const void* base, unsigned idx) {
  if constexpr (NT)
    return __builtin_nontemporal_load((const HMC_GLOBAL T*)((const HMC_GLOBAL char*)base + idx * (unsigned)sizeof(T)));
  else
    return gld<T>(base, idx);
}
template <typename T>
__device__ __forceinline__ HMC_GLOBAL T& gst(void* base, unsigned idx) {
  return *(HMC_GLOBAL T*)((HMC_GLOBAL char*)base + idx * (unsigned)sizeof(T));
}
// A store, with the non-temporal hint when NT.
template <bool NT, typename T>
__device__ __forceinline__ void gput(void* base, unsigned idx, T v) {
  HMC_GLOBAL T* p = (HMC_GLOBAL T*)((HMC_GLOBAL char*)base + idx * (unsigned)sizeof(T));
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// ------------------------------------------------------------ complex

template <typename R>
struct cx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cmake(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> mul_i(cx<R> a) { return {-a.im, a.re}; }  // i*a
template <typename R>
__device__ __forceinline__ cx<R> mul_mi(cx<R> a) { return {a.im, -a.re}; }  // -i*a
// acc + a*b
template <typename R>
__device__ __forceinline__ cx<R> cmadd(cx<R> acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
// acc + conj(a)*b
template <typename R>
__device__ __forceinline__ cx<R> cmadd_conj(cx<R> acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
  return acc;
}
template <typename R>
__device__ __forceinline__ R norm2(cx<R> a) { return a.re * a.re + a.im * a.im; }

// 3x3 complex matrices, row-major m[3*row + col].
template <typename R>
struct mat3 {
  cx<R> m[9];
};

template <typename R>
__device__ __forceinline__ mat3<R> mmul(const mat3<R>& a, const mat3<R>& b) {
  mat3<R> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<R> s = a.m[3 * i] * b.m[j];
      s = cmadd(s, a.m[3 * i + 1], b.m[3 + j]);
      s = cmadd(s, a.m[3 * i + 2], b.m[6 + j]);
      r.m[3 * i + j] = s;
    }
  return r;
}
// a * b^dagger
template <typename R>
__device__ __forceinline__ mat3<R> mmul_nd(const mat3<R>& a, const mat3<R>& b) {
  mat3<R> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<R> s = a.m[3 * i] * conj(b.m[3 * j]);
      s = cmadd(s, a.m[3 * i + 1], conj(b.m[3 * j + 1]));
      s = cmadd(s, a.m[3 * i + 2], conj(b.m[3 * j + 2]));
      r.m[3 * i + j] = s;
    }
  return r;
}
// a^dagger * b
template <typename R>
__device__ __forceinline__ mat3<R> mmul_dn(const mat3<R>& a, const mat3<R>& b) {
  mat3<R> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<R> s = cmadd_conj(cx<R>{0, 0}, a.m[i], b.m[j]);
      s = cmadd_conj(s, a.m[3 + i], b.m[3 + j]);
      s = cmadd_conj(s, a.m[6 + i], b.m[6 + j]);
      r.m[3 * i + j] = s;
    }
  return r;
}
template <typename R>
__device__ __forceinline__ mat3<R> madd(const mat3<R>& a, const mat3<R>& b) {
  mat3<R> r;
#pragma unroll
  for (int k = 0; k < 9; ++k) r.m[k] = a.m[k] + b.m[k];
  return r;
}
template <typename R>
__device__ __forceinline__ mat3<R> msub(const mat3<R>& a, const mat3<R>& b) {
  mat3<R> r;
#pragma unroll
  for (int k = 0; k < 9; ++k) r.m[k] = a.m[k] - b.m[k];
  return r;
}
// U * v (colour vector)
template <typename R>
__device__ __forceinline__ void mv(const mat3<R>& u, const cx<R>* v, cx<R>* out) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    cx<R> s = u.m[3 * i] * v[0];
    s = cmadd(s, u.m[3 * i + 1], v[1]);
    out[i] = cmadd(s, u.m[3 * i + 2], v[2]);
  }
}
// U^dagger * v
template <typename R>
__device__ __forceinline__ void mdv(const mat3<R>& u, const cx<R>* v, cx<R>* out) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    cx<R> s = cmadd_conj(cx<R>{0, 0}, u.m[i], v[0]);
    s = cmadd_conj(s, u.m[3 + i], v[1]);
    out[i] = cmadd_conj(s, u.m[6 + i], v[2]);
  }
}

// Compact traceless Hermitian storage (8 reals):
// (H00, H11, Re H01, Im H01, Re H02, Im H02, Re H12, Im H12), H22 = -H00-H11.
template <typename R>
__device__ __forceinline__ mat3<R> herm_from_compact(const R* c) {
  mat3<R> h;
  h.m[0] = {c[0], 0};
  h.m[4] = {c[1], 0};
  h.m[8] = {-c[0] - c[1], 0};
  h.m[1] = {c[2], c[3]};
  h.m[3] = {c[2], -c[3]};
  h.m[2] = {c[4], c[5]};
  h.m[6] = {c[4], -c[5]};
  h.m[5] = {c[6], c[7]};
  h.m[7] = {c[6], -c[7]};
  return h;
}

// Traceless anti-Hermitian projection Z = (W - W^dag) - Tr(W - W^dag)/3 of a
// matrix W, multiplied by (i*c), returned in compact Hermitian form.  (i*Z
// is Hermitian because Z is anti-Hermitian.)
template <typename R>
__device__ __forceinline__ void i_ta_compact(const mat3<R>& W, R c, R* out) {
  // diagonal of Z is 2i Im W_kk; trace removal on the imaginary parts
  R d0 = 2 * W.m[0].im, d1 = 2 * W.m[4].im, d2 = 2 * W.m[8].im;
  R tr = (d0 + d1 + d2) / 3;
  // (i c) * (i d) = -c d on the diagonal
  out[0] = -c * (d0 - tr);
  out[1] = -c * (d1 - tr);
  // Z01 = W01 - conj(W10);  (i c) Z01
  cx<R> z01 = W.m[1] - conj(W.m[3]);
  cx<R> z02 = W.m[2] - conj(W.m[6]);
  cx<R> z12 = W.m[5] - conj(W.m[7]);
  out[2] = -c * z01.im;
  out[3] = c * z01.re;
  out[4] = -c * z02.im;
  out[5] = c * z02.re;
  out[6] = -c * z12.im;
  out[7] = c * z12.re;
}

// Gram-Schmidt projection to SU(3) of rows: normalise row 0, orthogonalise
// row 1 against it and normalise, row 2 = conj(row0 x row1).
// Third row of an SU(3) matrix from the first two: conj(row0 x row1)
// (unitarity with det = 1).  Shared by the reunitarisation and by the
// two-row link loads, so a reunitarised link is rebuilt bit for bit.
template <typename R>
__device__ __forceinline__ void third_row(mat3<R>& u) {
  u.m[6] = conj(u.m[1] * u.m[5] - u.m[2] * u.m[4]);
  u.m[7] = conj(u.m[2] * u.m[3] - u.m[0] * u.m[5]);
  u.m[8] = conj(u.m[0] * u.m[4] - u.m[1] * u.m[3]);
}

template <typename R>
__device__ __forceinline__ void reunitarise(mat3<R>& u) {
  R n0 = norm2(u.m[0]) + norm2(u.m[1]) + norm2(u.m[2]);
  n0 = R(1) / sqrt(n0);
#pragma unroll
  for (int k = 0; k < 3; ++k) u.m[k] = n0 * u.m[k];
  cx<R> ov = cmadd_conj(cx<R>{0, 0}, u.m[0], u.m[3]);
  ov = cmadd_conj(ov, u.m[1], u.m[4]);
  ov = cmadd_conj(ov, u.m[2], u.m[5]);
#pragma unroll
  for (int k = 0; k < 3; ++k) u.m[3 + k] = u.m[3 + k] - ov * u.m[k];
  R n1 = norm2(u.m[3]) + norm2(u.m[4]) + norm2(u.m[5]);
  n1 = R(1) / sqrt(n1);
#pragma unroll
  for (int k = 0; k < 3; ++k) u.m[3 + k] = n1 * u.m[3 + k];
  third_row(u);
}

// exp(i Q) for traceless Hermitian Q.  With A = iQ traceless, the
// Cayley-Hamilton relation A^3 = s A + d 1 (s = Tr(A^2)/2, d = det A)
// folds every power into A^n = p_n 1 + q_n A + r_n A^2, so the exponential
// series reduces to three scalar series f0 + f1 A + f2 A^2.  The series
// runs until the bound |Q|_F^n / n! falls below 1e-18 (at most 48 terms).
__device__ __forceinline__ mat3<double> exp_iQ(const mat3<double>& Q) {
  using C = cx<double>;
  // A = iQ, A^2 = -Q^2
  mat3<double> Q2 = mmul(Q, Q);
  double trQ2 = Q2.m[0].re + Q2.m[4].re + Q2.m[8].re;  // = |Q|_F^2
  double s = -0.5 * trQ2;                               // Tr(A^2)/2
  // det(A) = i^3 det(Q) = -i det(Q); det Q is real for Hermitian Q
  C dq = Q.m[0] * (Q.m[4] * Q.m[8] - Q.m[5] * Q.m[7]) - Q.m[1] * (Q.m[3] * Q.m[8] - Q.m[5] * Q.m[6]) +
         Q.m[2] * (Q.m[3] * Q.m[7] - Q.m[4] * Q.m[6]);
  C d = mul_mi(dq);
  C p = {1, 0}, q = {0, 0}, r = {0, 0};  // coefficients of A^n / n!
  C f0 = p, f1 = q, f2 = r;
  double nrm = sqrt(trQ2), bound = 1.0;
  for (int n = 1; n <= 48; ++n) {
    double inv = 1.0 / n;
    C pn = inv * (r * d);
    C qn = inv * (p + s * r);
    C rn = inv * q;
    p = pn;
    q = qn;
    r = rn;
    f0 = f0 + p;
    f1 = f1 + q;
    f2 = f2 + r;
    bound *= nrm * inv;
    if (bound < 1e-18 && n >= 3) break;
  }
  // E = f0 + f1 (iQ) - f2 Q^2
  mat3<double> E;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    C iq = mul_i(Q.m[k]);
    E.m[k] = f1 * iq - f2 * Q2.m[k];
  }
  E.m[0] = E.m[0] + f0;
  E.m[4] = E.m[4] + f0;
  E.m[8] = E.m[8] + f0;
  return E;
}

// ------------------------------------------------------ spin projection

// (1 + SIG*gamma_mu) psi in the DeGrand-Rossi basis is fixed by its first
// two spin components h0, h1; components 2 and 3 are +-h or +-i h.
template <int MU, int SIG, typename R>
__device__ __forceinline__ void spin_project(const cx<R>* psi, cx<R>* h) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R> p0 = psi[c], p1 = psi[3 + c], p2 = psi[6 + c], p3 = psi[9 + c];
    if (MU == 0) {  // gamma_1 psi = ( i p3,  i p2, -i p1, -i p0)
      h[c] = SIG > 0 ? p0 + mul_i(p3) : p0 - mul_i(p3);
      h[3 + c] = SIG > 0 ? p1 + mul_i(p2) : p1 - mul_i(p2);
    } else if (MU == 1) {  // gamma_2 psi = (-p3,  p2,  p1, -p0)
      h[c] = SIG > 0 ? p0 - p3 : p0 + p3;
      h[3 + c] = SIG > 0 ? p1 + p2 : p1 - p2;
    } else if (MU == 2) {  // gamma_3 psi = ( i p2, -i p3, -i p0,  i p1)
      h[c] = SIG > 0 ? p0 + mul_i(p2) : p0 - mul_i(p2);
      h[3 + c] = SIG > 0 ? p1 - mul_i(p3) : p1 + mul_i(p3);
    } else {  // gamma_4 psi = (p2, p3, p0, p1)
      h[c] = SIG > 0 ? p0 + p2 : p0 - p2;
      h[3 + c] = SIG > 0 ? p1 + p3 : p1 - p3;
    }
  }
}

// acc += (1 + SIG*gamma_mu)-reconstruction of the projected, link-multiplied
// half spinor uh (components 2, 3 rebuilt from components 0, 1).
template <int MU, int SIG, typename R>
__device__ __forceinline__ void spin_accum(cx<R>* acc, const cx<R>* uh) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R> h0 = uh[c], h1 = uh[3 + c];
    acc[c] = acc[c] + h0;
    acc[3 + c] = acc[3 + c] + h1;
    if (MU == 0) {  // r2 = -SIG i h1, r3 = -SIG i h0
      acc[6 + c] = acc[6 + c] + (SIG > 0 ? mul_mi(h1) : mul_i(h1));
      acc[9 + c] = acc[9 + c] + (SIG > 0 ? mul_mi(h0) : mul_i(h0));
    } else if (MU == 1) {  // r2 = SIG h1, r3 = -SIG h0
      acc[6 + c] = SIG > 0 ? acc[6 + c] + h1 : acc[6 + c] - h1;
      acc[9 + c] = SIG > 0 ? acc[9 + c] - h0 : acc[9 + c] + h0;
    } else if (MU == 2) {  // r2 = -SIG i h0, r3 = SIG i h1
      acc[6 + c] = acc[6 + c] + (SIG > 0 ? mul_mi(h0) : mul_i(h0));
      acc[9 + c] = acc[9 + c] + (SIG > 0 ? mul_i(h1) : mul_mi(h1));
    } else {  // r2 = SIG h0, r3 = SIG h1
      acc[6 + c] = SIG > 0 ? acc[6 + c] + h0 : acc[6 + c] - h0;
      acc[9 + c] = SIG > 0 ? acc[9 + c] + h1 : acc[9 + c] - h1;
    }
  }
}

// ------------------------------------------------------------ geometry

// Lattice extents and checkerboard sizes.  Lx and every other extent are
// even; the checkerboard index of lexicographic site i is i >> 1.
struct Lat {
  int L[4];
  int Vh;      // sites per parity
  int stride;  // elements between successive components of a field (= Vh)
  // Tiled site order of the one-site-per-work-item Dslash (tiled = 0: the
  // linear order with XCD-contiguous ranges): checkerboard sites per z-plane
  // and per t-slice, 64-site chunks per z-plane, t-slices per XCD, chunks
  // per y-block (tile_y = tile_r: the whole plane is one block; tile_y = 0:
  // the z-planes are not whole chunks and the walk takes the chunks of the
  // t-slices instead).
  int tiled, plane, slice, tile_r, tile_t, tile_y;
};

inline Lat to_lat(const LatArg& a) {
  Lat g;
  for (int k = 0; k < 4; ++k) g.L[k] = a.L[k];
  g.Vh = a.Vh;
  g.stride = a.stride;
  g.tiled = g.plane = g.slice = g.tile_r = g.tile_t = g.tile_y = 0;
  return g;
}

struct Site {
  int c[4];
  int lex;
};

__device__ __forceinline__ Site cb_site(const Lat& g, int par, int s) {
  Site st;
  int i0 = 2 * s;
  int x0 = i0 % g.L[0];
  int r = i0 / g.L[0];
  st.c[1] = r % g.L[1];
  r /= g.L[1];
  st.c[2] = r % g.L[2];
  st.c[3] = r / g.L[2];
  int odd = (par ^ st.c[1] ^ st.c[2] ^ st.c[3]) & 1;
  st.c[0] = x0 + odd;
  st.lex = i0 + odd;
  return st;
}

// Lexicographic index of the neighbour of `st` one step along +mu (DIR=+1)
// or -mu (DIR=-1); *wrapped is set when the step crosses the boundary.
template <int MU, int DIR>
__device__ __forceinline__ int neighbour_lex(const Lat& g, const Site& st, bool* wrapped) {
  int step = 1;
#pragma unroll
  for (int k = 0; k < MU; ++k) step *= g.L[k];
  int c = st.c[MU];
  if (DIR > 0) {
    bool w = (c == g.L[MU] - 1);
    *wrapped = w;
    return w ? st.lex - (g.L[MU] - 1) * step : st.lex + step;
  } else {
    bool w = (c == 0);
    *wrapped = w;
    return w ? st.lex + (g.L[MU] - 1) * step : st.lex - step;
  }
}

__device__ __forceinline__ int parity_of_lex(const Lat& g, int lex) {
  int x = lex % g.L[0];
  int r = lex / g.L[0];
  int y = r % g.L[1];
  r /= g.L[1];
  int z = r % g.L[2];
  int t = r / g.L[2];
  return (x + y + z + t) & 1;
}

// The 8 XCDs of an MI355X take workgroups round-robin.  This remaps the
// hardware block id so that each XCD walks one contiguous range of logical
// blocks (sites), keeping neighbour reuse inside one XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  constexpr int X = 8;
  int q = nb / X, r = nb % X;
  int xcd = b % X, k = b / X;
  return xcd * q + min(xcd, r) + k;
}

// Output site of this work-item in a one-site-per-work-item launch of
// 256-site blocks; *part gets the block's partial-sum slot.  Linear order:
// block b covers sites 256 b .. 256 b + 255, XCD-contiguous (xcd_remap).
// Tiled order: XCD x (blocks with blockIdx.x % 8 == x) owns the t-slices
// [x tile_t, (x + 1) tile_t).  Each z-plane of a t-slice is cut into
// y-blocks of tile_y 64-site chunks (consecutive checkerboard sites, so a
// block spans whole rows of constant y but for its ends); the XCD walks its
// wavefronts y-block by y-block, within a y-block z-plane by z-plane, then
// t-slice by t-slice, then chunk by chunk.  The +-t neighbours of a site are
// then tile_y wavefronts away in the walk and the +-z neighbours
// tile_t tile_y away: with small y-blocks several z-planes are in flight at
// once and the neighbours they share are still in the XCD's L2, where the
// linear order has the t neighbours a whole t-slice (tens of MB of traffic)
// away.  Only the +-y neighbours of the two edge rows of a y-block and the
// +-t neighbours across XCDs are read a second time from beyond L2.  Where
// a z-plane is not a whole number of chunks (tile_y = 0) the XCD walks the
// 64-site chunks of its t-slices, t-slice fastest: the +-t neighbours are
// then one wavefront away and the +-z neighbours tile_t plane / 64.
__device__ __forceinline__ int dslash_site(const Lat& g, int* part) {
  if (g.tiled) {
    const int xcd = blockIdx.x & 7, k = blockIdx.x >> 3;
    const int w = k * 4 + (threadIdx.x >> 6);  // wavefront of this XCD, in walk order
    *part = blockIdx.x;
    if (g.tile_y == 0) return (xcd * g.tile_t + w % g.tile_t) * g.slice + (w / g.tile_t) * 64 + (threadIdx.x & 63);
    const int c = w % g.tile_y, q = w / g.tile_y;
    const int t = xcd * g.tile_t + q % g.tile_t, q2 = q / g.tile_t;
    const int z = q2 % g.L[2], yb = q2 / g.L[2];
    return t * g.slice + z * g.plane + (yb * g.tile_y + c) * 64 + (threadIdx.x & 63);
  }
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  *part = b;
  return b * kBlock + threadIdx.x;
}

// ------------------------------------------------------ storage formats
//
// Spinor half-fields are 12 complex components (spin-major, colour minor)
// stored component-major: element (k, s) at k*stride + s.  Consecutive
// work-items therefore read consecutive addresses for every component.
//   SpF64  double2                      (192 B / site)
//   SpF32  float2                       ( 96 B / site)
//   SpF16  __half2, then one float scale per site (52 B / site); the stored
//          halves are the components divided by the site's max |re|,|im|
//   SpBF16 two bfloat16 in a uint32     ( 48 B / site)
// Gauge fields: [mu][parity][9][stride] of the same element types (links
// need no scale: every |U_ij| <= 1).

__device__ __forceinline__ float bf16_to_f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ uint32_t f_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return u >> 16;
}

// Loads and stores take a base pointer (uniform across the wave) and a
// 32-bit element index, so the compiler emits global loads with a scalar
// base and a 32-bit vector offset.
struct SpF64 {
  static constexpr bool kScaled = false;
  using R = double;
  static constexpr int kBytes = 192;
  __device__ static void load(const void* base, int stride, int s, cx<R>* v) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      v2d t = gld<v2d>(base, k * stride + s);
      v[k] = {t.x, t.y};
    }
  }
  template <bool NT = false>
  __device__ static void store(void* base, int stride, int s, const cx<R>* v) {
#pragma unroll
    for (int k = 0; k < 12; ++k) gput<NT>(base, k * stride + s, v2d{v[k].re, v[k].im});
  }
  // component k of site s
  __device__ static cx<R> load_one(const void* base, int stride, int s, int k) {
    v2d t = gld<v2d>(base, k * stride + s);
    return {t.x, t.y};
  }
  // components 3*part .. 3*part+2 of site s
  template <bool NT = false>
  __device__ static void store_part(void* base, int stride, int s, int part, const cx<R>* v) {
#pragma unroll
    for (int c = 0; c < 3; ++c) gput<NT>(base, (3 * part + c) * stride + s, v2d{v[c].re, v[c].im});
  }
};

struct SpF32 {
  static constexpr bool kScaled = false;
  using R = float;
  static constexpr int kBytes = 96;
  __device__ static void load(const void* base, int stride, int s, cx<R>* v) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      v2f t = gld<v2f>(base, k * stride + s);
      v[k] = {t.x, t.y};
    }
  }
  template <bool NT = false>
  __device__ static void store(void* base, int stride, int s, const cx<R>* v) {
#pragma unroll
    for (int k = 0; k < 12; ++k) gput<NT>(base, k * stride + s, v2f{v[k].re, v[k].im});
  }
  __device__ static cx<R> load_one(const void* base, int stride, int s, int k) {
    v2f t = gld<v2f>(base, k * stride + s);
    return {t.x, t.y};
  }
  template <bool NT = false>
  __device__ static void store_part(void* base, int stride, int s, int part, const cx<R>* v) {
#pragma unroll
    for (int c = 0; c < 3; ++c) gput<NT>(base, (3 * part + c) * stride + s, v2f{v[c].re, v[c].im});
  }
};

struct SpF16 {
  static constexpr bool kScaled = true;
  using R = float;
  static constexpr int kBytes = 52;
  __device__ static void load(const void* base, int stride, int s, cx<R>* v) {
    const float f = gld<float>(base, 12 * stride + s);  // scales follow the 12 components
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      v2f t = __builtin_convertvector(gld<v2h>(base, k * stride + s), v2f);
      v[k] = {t.x * f, t.y * f};
    }
  }
  // A site whose largest component is below the smallest normal float is
  // stored as zero: 1/m would overflow to infinity.  Such sites arise where
  // a field spreads from a point: each hop onto a new site carries the
  // half-precision remainders of its neighbours, so the scales of the front
  // shrink by ~1e-8 per hop and reach the float denormals within a few
  // applications of the operator; they are ~1e-38 of the field's norm.
  // (A NaN or infinite m passes, so a non-finite site stays non-finite.)
  __device__ static float live_scale(float m) { return m < __FLT_MIN__ ? 0.f : m; }
  template <bool NT = false>
  __device__ static void store(void* base, int stride, int s, const cx<R>* v) {
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
    m = live_scale(m);
    float inv = m > 0.f ? 1.f / m : 0.f;
    gput<NT>(base, 12 * stride + s, m);
#pragma unroll
    for (int k = 0; k < 12; ++k)
      gput<NT>(base, k * stride + s, __builtin_convertvector((v2f{v[k].re * inv, v[k].im * inv}), v2h));
  }
  __device__ static cx<R> load_one(const void* base, int stride, int s, int k) {
    const float f = gld<float>(base, 12 * stride + s);
    v2f t = __builtin_convertvector(gld<v2h>(base, k * stride + s), v2f);
    return {t.x * f, t.y * f};
  }
  // components 3*part .. 3*part+2 of site s, with the site's max |re|,|im|
  // m computed by the caller over all 12 components (part 0 writes it)
  template <bool NT = false>
  __device__ static void store_part_scaled(void* base, int stride, int s, int part, const cx<R>* v, float m) {
    m = live_scale(m);
    const float inv = m > 0.f ? 1.f / m : 0.f;
    if (part == 0) gput<NT>(base, 12 * stride + s, m);
#pragma unroll
    for (int c = 0; c < 3; ++c)
      gput<NT>(base, (3 * part + c) * stride + s, __builtin_convertvector((v2f{v[c].re * inv, v[c].im * inv}), v2h));
  }
};

struct SpBF16 {
  static constexpr bool kScaled = false;
  using R = float;
  static constexpr int kBytes = 48;
  __device__ static void load(const void* base, int stride, int s, cx<R>* v) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      uint32_t w = gld<uint32_t>(base, k * stride + s);
      v[k] = {bf16_to_f(w & 0xffffu), bf16_to_f(w >> 16)};
    }
  }
  template <bool NT = false>
  __device__ static void store(void* base, int stride, int s, const cx<R>* v) {
#pragma unroll
    for (int k = 0; k < 12; ++k) gput<NT>(base, k * stride + s, f_to_bf16(v[k].re) | (f_to_bf16(v[k].im) << 16));
  }
  __device__ static cx<R> load_one(const void* base, int stride, int s, int k) {
    uint32_t w = gld<uint32_t>(base, k * stride + s);
    return {bf16_to_f(w & 0xffffu), bf16_to_f(w >> 16)};
  }
  template <bool NT = false>
  __device__ static void store_part(void* base, int stride, int s, int part, const cx<R>* v) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      gput<NT>(base, (3 * part + c) * stride + s, f_to_bf16(v[c].re) | (f_to_bf16(v[c].im) << 16));
  }
};

// Links: element (mu, parity, k, s) at ((mu*2 + parity)*9 + k)*stride + s.
struct LkF64 {
  static constexpr bool kStream = false;
  using R = double;
  static constexpr int kBytes = 144;
  // component K (row K / 3, column K % 3) alone
  template <int K, bool NT = false>
  __device__ static cx<R> one(const void* base, int stride, int mu, int par, int s) {
    const void* p = (const char*)base + (size_t)(mu * 2 + par) * 9 * stride * sizeof(v2d);
    v2d t = gld_link<v2d, NT>(p, K * stride + s);
    return {t.x, t.y};
  }
  template <int K = 9, bool NT = false>
  __device__ static mat3<R> load(const void* base, int stride, int mu, int par, int s) {
    const void* p = (const char*)base + (size_t)(mu * 2 + par) * 9 * stride * sizeof(v2d);
    mat3<R> u;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      v2d t = gld_link<v2d, NT>(p, k * stride + s);
      u.m[k] = {t.x, t.y};
    }
    return u;
  }
  // Component K of the link at checkerboard site s of parity par, where mu
  // and par are uniform over the wavefront: the array's base is then a
  // scalar and the lane's byte offset voff = 16 s is shared by all
  // components, so a load costs no vector address arithmetic.
  template <int K>
  __device__ static cx<R> one_u(const void* base, int stride, int mu, int par, unsigned voff) {
    const HMC_GLOBAL char* p =
        (const HMC_GLOBAL char*)base + ((size_t)((mu * 2 + par) * 9 + K) * (size_t)stride) * sizeof(v2d);
    v2d t = *(const HMC_GLOBAL v2d*)(p + voff);
    return {t.x, t.y};
  }
  __device__ static void store(void* base, int stride, int mu, int par, int s, const mat3<R>& u) {
    void* p = (char*)base + (size_t)(mu * 2 + par) * 9 * stride * sizeof(v2d);
#pragma unroll
    for (int k = 0; k < 9; ++k) gst<v2d>(p, k * stride + s) = v2d{u.m[k].re, u.m[k].im};
  }
};

struct LkF32 {
  static constexpr bool kStream = false;
  using R = float;
  static constexpr int kBytes = 72;
  // component K (row K / 3, column K % 3) alone
  template <int K, bool NT = false>
  __device__ static cx<R> one(const void* base, int stride, int mu, int par, int s) {
    const void* p = (const char*)base + (size_t)(mu * 2 + par) * 9 * stride * sizeof(v2f);
    v2f t = gld_link<v2f, NT>(p, K * stride + s);
    return {t.x, t.y};
  }
  template <int K = 9, bool NT = false>
  __device__ static mat3<R> load(const void* base, int stride, int mu, int par, int s) {
    const void* p = (const char*)base + (size_t)(mu * 2 + par) * 9 * stride * sizeof(v2f);
    mat3<R> u;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      v2f t = gld_link<v2f, NT>(p, k * stride + s);
      u.m[k] = {t.x, t.y};
    }
    return u;
  }
  __device__ static void store(void* base, int stride, int mu, int par, int s, const mat3<double>& u) {
    void* p = (char*)base + (size_t)(mu * 2 + par) * 9 * stride * sizeof(v2f);
#pragma unroll
    for (int k = 0; k < 9; ++k) gst<v2f>(p, k * stride + s) = v2f{(float)u.m[k].re, (float)u.m[k].im};
  }
};

struct LkF16 {
  static constexpr bool kStream = false;
  using R = float;
  static constexpr int kBytes = 36;
  // component K (row K / 3, column K % 3) alone
  template <int K, bool NT = false>
  __device__ static cx<R> one(const void* base, int stride, int mu, int par, int s) {
    const void* p = (const char*)base + (size_t)(mu * 2 + par) * 9 * stride * sizeof(v2h);
    v2f t = __builtin_convertvector(gld_link<v2h, NT>(p, K * stride + s), v2f);
    return {t.x, t.y};
  }
  template <int K = 9, bool NT = false>
  __device__ static mat3<R> load(const void* base, int stride, int mu, int par, int s) {
    const void* p = (const char*)base + (size_t)(mu * 2 + par) * 9 * stride * sizeof(v2h);
    mat3<R> u;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      v2f t = __builtin_convertvector(gld_link<v2h, NT>(p, k * stride + s), v2f);
      u.m[k] = {t.x, t.y};
    }
    return u;
  }
  __device__ static void store(void* base, int stride, int mu, int par, int s, const mat3<double>& u) {
    void* p = (char*)base + (size_t)(mu * 2 + par) * 9 * stride * sizeof(v2h);
#pragma unroll
    for (int k = 0; k < 9; ++k)
      gst<v2h>(p, k * stride + s) = __builtin_convertvector((v2f{(float)u.m[k].re, (float)u.m[k].im}), v2h);
  }
};

struct LkBF16 {
  static constexpr bool kStream = false;
  using R = float;
  static constexpr int kBytes = 36;
  // component K (row K / 3, column K % 3) alone
  template <int K, bool NT = false>
  __device__ static cx<R> one(const void* base, int stride, int mu, int par, int s) {
    const void* p = (const char*)base + (size_t)(mu * 2 + par) * 9 * stride * sizeof(uint32_t);
    uint32_t w = gld_link<uint32_t, NT>(p, K * stride + s);
    return {bf16_to_f(w & 0xffffu), bf16_to_f(w >> 16)};
  }
  template <int K = 9, bool NT = false>
  __device__ static mat3<R> load(const void* base, int stride, int mu, int par, int s) {
    const void* p = (const char*)base + (size_t)(mu * 2 + par) * 9 * stride * sizeof(uint32_t);
    mat3<R> u;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      uint32_t w = gld_link<uint32_t, NT>(p, k * stride + s);
      u.m[k] = {bf16_to_f(w & 0xffffu), bf16_to_f(w >> 16)};
    }
    return u;
  }
  __device__ static void store(void* base, int stride, int mu, int par, int s, const mat3<double>& u) {
    void* p = (char*)base + (size_t)(mu * 2 + par) * 9 * stride * sizeof(uint32_t);
#pragma unroll
    for (int k = 0; k < 9; ++k)
      gst<uint32_t>(p, k * stride + s) = f_to_bf16((float)u.m[k].re) | (f_to_bf16((float)u.m[k].im) << 16);
  }
};

// Two-row form of any of the link formats above: reads components 0..5
// (rows 0 and 1) and rebuilds row 2, for fields that are SU(3) to rounding.
// Two thirds of the link bytes of a hop.
template <class LK, bool NT = false>
struct LkRows2 {
  using R = typename LK::R;
  static constexpr int kBytes = LK::kBytes / 9 * 6;
  static constexpr bool kStream = NT;  // non-temporal link loads (and output stores)
  __device__ static mat3<R> load(const void* base, int stride, int mu, int par, int s) {
    mat3<R> u = LK::template load<6, NT>(base, stride, mu, par, s);
    third_row(u);
    return u;
  }
  // rows 0 and 1 only (row 2 not set)
  __device__ static mat3<R> load2(const void* base, int stride, int mu, int par, int s) {
    return LK::template load<6, NT>(base, stride, mu, par, s);
  }
  // the same with mu and par uniform over the wavefront (LK::one_u)
  __device__ static mat3<R> load2_u(const void* base, int stride, int mu, int par, int s) {
    static_assert(!NT, "uniform-parity loads are not streamed");
    const unsigned v = (unsigned)s * 16u;
    mat3<R> u;
    u.m[0] = LK::template one_u<0>(base, stride, mu, par, v);
    u.m[1] = LK::template one_u<1>(base, stride, mu, par, v);
    u.m[2] = LK::template one_u<2>(base, stride, mu, par, v);
    u.m[3] = LK::template one_u<3>(base, stride, mu, par, v);
    u.m[4] = LK::template one_u<4>(base, stride, mu, par, v);
    u.m[5] = LK::template one_u<5>(base, stride, mu, par, v);
    return u;
  }
  __device__ static mat3<R> load_u(const void* base, int stride, int mu, int par, int s) {
    mat3<R> u = load2_u(base, stride, mu, par, s);
    third_row(u);
    return u;
  }
};

// Row 0 and column 2 of any of the link formats above (components 0, 1, 2,
// 5, 8: 5/9 of the link bytes), for fields that are SU(3) to rounding.
// Row 1's first two entries solve the 2x2 system of orthogonality to row 0
// and det U = 1 (through row 2 = conj(row0 x row1)), whose determinant is
// D = |u00|^2 + |u01|^2 = 1 - |u02|^2; row 2 is then rebuilt as in the
// two-row form.  The solve amplifies rounding by 1/D, so a link with
// D < 1/16 reads u10 and u11 instead (exact; on smooth fields no work-item
// takes that branch).
template <class LK, bool NT = false>
struct LkRowCol {
  using R = typename LK::R;
  static constexpr int kBytes = LK::kBytes / 9 * 5;
  static constexpr bool kStream = NT;  // non-temporal link loads (and output stores)
  __device__ static mat3<R> load(const void* base, int stride, int mu, int par, int s) {
    mat3<R> u = load2(base, stride, mu, par, s);
    third_row(u);
    return u;
  }
  // rows 0 and 1 only (row 2 not set)
  __device__ static mat3<R> load2(const void* base, int stride, int mu, int par, int s) {
    mat3<R> u;
    u.m[0] = LK::template one<0, NT>(base, stride, mu, par, s);
    u.m[1] = LK::template one<1, NT>(base, stride, mu, par, s);
    u.m[2] = LK::template one<2, NT>(base, stride, mu, par, s);
    u.m[5] = LK::template one<5, NT>(base, stride, mu, par, s);
    u.m[8] = LK::template one<8, NT>(base, stride, mu, par, s);
    const R d = norm2(u.m[0]) + norm2(u.m[1]);
    if (d < R(0.0625)) {
      u.m[3] = LK::template one<3, NT>(base, stride, mu, par, s);
      u.m[4] = LK::template one<4, NT>(base, stride, mu, par, s);
    } else {
      solve_row1(u, d);
    }
    return u;
  }
  // the same with mu and par uniform over the wavefront (LK::one_u)
  __device__ static mat3<R> load2_u(const void* base, int stride, int mu, int par, int s) {
    static_assert(!NT, "uniform-parity loads are not streamed");
    const unsigned v = (unsigned)s * 16u;
    mat3<R> u;
    u.m[0] = LK::template one_u<0>(base, stride, mu, par, v);
    u.m[1] = LK::template one_u<1>(base, stride, mu, par, v);
    u.m[2] = LK::template one_u<2>(base, stride, mu, par, v);
    u.m[5] = LK::template one_u<5>(base, stride, mu, par, v);
    u.m[8] = LK::template one_u<8>(base, stride, mu, par, v);
    const R d = norm2(u.m[0]) + norm2(u.m[1]);
    if (d < R(0.0625)) {
      u.m[3] = LK::template one_u<3>(base, stride, mu, par, v);
      u.m[4] = LK::template one_u<4>(base, stride, mu, par, v);
    } else {
      solve_row1(u, d);
    }
    return u;
  }
  __device__ static mat3<R> load_u(const void* base, int stride, int mu, int par, int s) {
    mat3<R> u = load2_u(base, stride, mu, par, s);
    third_row(u);
    return u;
  }
  // u10 = -(u00 conj(u02) u12 + conj(u01) conj(u22)) / D
  // u11 = (conj(u00) conj(u22) - u01 conj(u02) u12) / D
  __device__ static void solve_row1(mat3<R>& u, R d) {
    const R inv = R(1) / d;
    const cx<R> w = conj(u.m[2]) * u.m[5];
    u.m[3] = (-inv) * (u.m[0] * w + conj(u.m[1]) * conj(u.m[8]));
    u.m[4] = inv * (conj(u.m[0]) * conj(u.m[8]) - u.m[1] * w);
  }
};

// Link forms that hold only SU(3) fields and can hand out rows 0 and 1
// alone (load2): products of such links can skip what SU(3) fixes.
template <class LK>
struct CompactLinks {
  static constexpr bool value = false;
};
template <class LK, bool NT>
struct CompactLinks<LkRows2<LK, NT>> {
  static constexpr bool value = true;
};
template <class LK, bool NT>
struct CompactLinks<LkRowCol<LK, NT>> {
  static constexpr bool value = true;
};

// Compact momenta / forces: double [mu][parity][8][stride].
__device__ __forceinline__ void load_compact(const double* P, int stride, int mu, int par, int s, double* c) {
  const double* p = P + (size_t)(mu * 2 + par) * 8 * stride;
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] = gld<double>(p, k * stride + s);
}
__device__ __forceinline__ void store_compact(double* P, int stride, int mu, int par, int s, const double* c) {
  double* p = P + (size_t)(mu * 2 + par) * 8 * stride;
#pragma unroll
  for (int k = 0; k < 8; ++k) gst<double>(p, k * stride + s) = c[k];
}

// ------------------------------------------------------------ Philox

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 64x64->128 multiplications with the Weyl key schedule.
__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                              uint64_t k1, uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// Uniform on (0,1): top 53 bits plus one half, scaled by 2^-53 (exact).
__device__ __forceinline__ double u53(uint64_t w) { return ((double)(w >> 11) + 0.5) * 0x1p-53; }

// Box-Muller pair from two words.
__device__ __forceinline__ void box_muller(uint64_t w0, uint64_t w1, double* g0, double* g1) {
  double r = sqrt(-2.0 * log(u53(w0)));
  double th = 6.283185307179586476925286766559 * u53(w1);
  double sn, cs;
  sincos(th, &sn, &cs);
  *g0 = r * cs;
  *g1 = r * sn;
}

// ------------------------------------------------------------ reductions

// Deterministic sum over the block: wave64 butterfly (fixed xor order),
// then wave partials combined by thread 0 in wave order.  Result valid in
// thread 0 only.  `N` values reduced at once; W wavefronts per block.
template <int N, int W = kBlock / 64>
__device__ __forceinline__ void block_sum(double* v) {
  __shared__ double red[N][W];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += __shfl_xor(v[k], off, 64);
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) red[k][wave] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double s = red[k][0];
#pragma unroll
      for (int w = 1; w < W; ++w) s += red[k][w];
      v[k] = s;
    }
}

// Every block (of W wavefronts) sums the same n partials in the same order
// and gets the same bit pattern; the result is broadcast to all threads of
// the block.  Work-item t adds elements t, t + 64 W, t + 128 W, ... in that
// order; their loads are issued eight at a time, so the sum waits for one
// memory round trip per eight elements instead of one per element.
template <int W = kBlock / 64, int N = 1>
__device__ __forceinline__ void sum_partials_n(const double* const* part, const int* n, double* out) {
  constexpr int S = 64 * W, U = 8;
  __shared__ double bc[N];
  double v[N];
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = 0.0;
  int nmax = 0;
#pragma unroll
  for (int q = 0; q < N; ++q) nmax = max(nmax, n[q]);
  for (int base = threadIdx.x; base < nmax; base += U * S) {
    double t[N][U];
#pragma unroll
    for (int q = 0; q < N; ++q)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = base + u * S;
        t[q][u] = k < n[q] ? part[q][k] : 0.0;
      }
#pragma unroll
    for (int q = 0; q < N; ++q)
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (base + u * S < n[q]) v[q] += t[q][u];
  }
  block_sum<N, W>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < N; ++q) bc[q] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < N; ++q) out[q] = bc[q];
  __syncthreads();
}

template <int W = kBlock / 64>
__device__ __forceinline__ double sum_partials(const double* part, int n) {
  double r;
  sum_partials_n<W, 1>(&part, &n, &r);
  return r;
}

}  // namespace hmc
