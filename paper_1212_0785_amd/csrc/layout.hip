// Conversion between the canonical array-of-structures layout (complex128,
// site-major, the form fields are imported and exported in) and the
// structure-of-arrays device layouts of device.h, plus precision
// conversion for the mixed-precision solver.  Sec. 3's tensor structure
// (Outer x Spin x Color x Reality) is kept: the outer (site) level becomes
// the fastest-varying index so that each spin/colour/reality component of
// a field is one contiguous array.
#include "device.h"
#include "internal.h"

namespace hmc {


__global__ void k_pack_gauge(Lat g, const double2* canon, double2* U) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= 2 * g.Vh) return;
  int par = parity_of_lex(g, i), s = i >> 1;
  for (int mu = 0; mu < 4; ++mu)
#pragma unroll
    for (int k = 0; k < 9; ++k) U[((size_t)(mu * 2 + par) * 9 + k) * g.stride + s] = canon[((size_t)i * 4 + mu) * 9 + k];
}

__global__ void k_unpack_gauge(Lat g, const double2* U, double2* canon) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= 2 * g.Vh) return;
  int par = parity_of_lex(g, i), s = i >> 1;
  for (int mu = 0; mu < 4; ++mu)
#pragma unroll
    for (int k = 0; k < 9; ++k) canon[((size_t)i * 4 + mu) * 9 + k] = U[((size_t)(mu * 2 + par) * 9 + k) * g.stride + s];
}

// canonical full spinor -> half spinor of parity par (blockIdx.y selects
// the parity when both halves are packed).
__global__ void k_pack_spinor(Lat g, const double2* canon, double2* half, int par0) {
  int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.Vh) return;
  int par = par0 < 0 ? (int)blockIdx.y : par0;
  double2* dst = half + (par0 < 0 ? (size_t)par * 12 * g.stride : 0);
  Site st = cb_site(g, par, s);
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[(size_t)k * g.stride + s] = canon[(size_t)st.lex * 12 + k];
}

__global__ void k_unpack_spinor(Lat g, const double2* half, double2* canon, int par0) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= 2 * g.Vh) return;
  int par = parity_of_lex(g, i), s = i >> 1;
  if (par0 >= 0 && par != par0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) canon[(size_t)i * 12 + k] = make_double2(0.0, 0.0);
    return;
  }
  const double2* src = half + (par0 < 0 ? (size_t)par * 12 * g.stride : 0);
#pragma unroll
  for (int k = 0; k < 12; ++k) canon[(size_t)i * 12 + k] = src[(size_t)k * g.stride + s];
}

__global__ void k_pack_momenta(Lat g, const double2* canon, double* P) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= 2 * g.Vh) return;
  int par = parity_of_lex(g, i), s = i >> 1;
  for (int mu = 0; mu < 4; ++mu) {
    const double2* m = canon + ((size_t)i * 4 + mu) * 9;
    double c[8] = {m[0].x, m[4].x, m[1].x, m[1].y, m[2].x, m[2].y, m[5].x, m[5].y};
    store_compact(P, g.stride, mu, par, s, c);
  }
}

__global__ void k_unpack_momenta(Lat g, const double* P, double2* canon) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= 2 * g.Vh) return;
  int par = parity_of_lex(g, i), s = i >> 1;
  for (int mu = 0; mu < 4; ++mu) {
    double c[8];
    load_compact(P, g.stride, mu, par, s, c);
    mat3<double> h = herm_from_compact(c);
    double2* m = canon + ((size_t)i * 4 + mu) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = make_double2(h.m[k].re, h.m[k].im);
  }
}

template <class LK>
__global__ void k_convert_gauge(Lat g, const void* U64, void* Ulow) {
  int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.Vh) return;
  int mu = blockIdx.y >> 1, par = blockIdx.y & 1;
  mat3<double> u = LkF64::load(U64, g.stride, mu, par, s);
  LK::store(Ulow, g.stride, mu, par, s, u);
}

// Counts the links that are not SU(3) to within `tol`: rows 0 and 1 not
// orthonormal (|row|^2 - 1, <row0, row1>), or the stored third row not
// conj(row0 x row1) (which then makes det U = 1), in any real component
// (per-block partial counts).  The compact link forms rebuild entries from
// exactly these relations.
__global__ void __launch_bounds__(kBlock) k_su3_check(Lat g, const void* U, double tol, double* part) {
  double v[1] = {0.0};
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < 2 * g.Vh; j += gridDim.x * kBlock) {
    const int par = j >= g.Vh, s = j - par * g.Vh;
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      const mat3<double> u = LkF64::load(U, g.stride, mu, par, s);
      mat3<double> r = u;
      third_row(r);
      bool bad = false;
#pragma unroll
      for (int k = 6; k < 9; ++k)
        bad |= !(fabs(u.m[k].re - r.m[k].re) <= tol) || !(fabs(u.m[k].im - r.m[k].im) <= tol);
      const double n0 = norm2(u.m[0]) + norm2(u.m[1]) + norm2(u.m[2]);
      const double n1 = norm2(u.m[3]) + norm2(u.m[4]) + norm2(u.m[5]);
      cx<double> o = cmadd_conj(cx<double>{0, 0}, u.m[0], u.m[3]);
      o = cmadd_conj(o, u.m[1], u.m[4]);
      o = cmadd_conj(o, u.m[2], u.m[5]);
      bad |= !(fabs(n0 - 1.0) <= tol) || !(fabs(n1 - 1.0) <= tol) || !(fabs(o.re) <= tol) || !(fabs(o.im) <= tol);
      v[0] += bad ? 1.0 : 0.0;
    }
  }
  block_sum<1>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

template <class SI, class SO>
__global__ void k_convert_spinor(Lat g, const void* in, void* out, const void* const* tin, void* const* tout,
                                 const int* gate) {
  if (gate && *gate == 0) return;  // gated: a device-driven reliable update that was not requested
  int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.Vh) return;
  const void* src = tin ? tin[blockIdx.y] : in;
  void* dst = tout ? tout[blockIdx.y] : out;
  cx<typename SI::R> a[12];
  cx<typename SO::R> b[12];
  SI::load(src, g.stride, s, a);
#pragma unroll
  for (int k = 0; k < 12; ++k) b[k] = {(typename SO::R)a[k].re, (typename SO::R)a[k].im};
  SO::store(dst, g.stride, s, b);
}

hipError_t launch_pack_gauge(const LatArg& g, const void* canon, void* U, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_gauge, dim3(ceil_div(2LL * g.Vh, kBlock)), dim3(kBlock), 0, st, to_lat(g),
                     (const double2*)canon, (double2*)U);
  return hipGetLastError();
}
hipError_t launch_unpack_gauge(const LatArg& g, const void* U, void* canon, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack_gauge, dim3(ceil_div(2LL * g.Vh, kBlock)), dim3(kBlock), 0, st, to_lat(g),
                     (const double2*)U, (double2*)canon);
  return hipGetLastError();
}
hipError_t launch_pack_spinor(const LatArg& g, const void* canon, void* half, int par, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_spinor, dim3(site_blocks(g.Vh), par < 0 ? 2 : 1), dim3(kBlock), 0, st, to_lat(g),
                     (const double2*)canon, (double2*)half, par);
  return hipGetLastError();
}
hipError_t launch_unpack_spinor(const LatArg& g, const void* half, void* canon, int par, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack_spinor, dim3(ceil_div(2LL * g.Vh, kBlock)), dim3(kBlock), 0, st, to_lat(g),
                     (const double2*)half, (double2*)canon, par);
  return hipGetLastError();
}
hipError_t launch_pack_momenta(const LatArg& g, const void* canon, double* P, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_momenta, dim3(ceil_div(2LL * g.Vh, kBlock)), dim3(kBlock), 0, st, to_lat(g),
                     (const double2*)canon, P);
  return hipGetLastError();
}
hipError_t launch_unpack_momenta(const LatArg& g, const double* P, void* canon, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack_momenta, dim3(ceil_div(2LL * g.Vh, kBlock)), dim3(kBlock), 0, st, to_lat(g), P,
                     (double2*)canon);
  return hipGetLastError();
}

hipError_t launch_su3_check(const LatArg& g, const void* U, double tol, double* part, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_su3_check, dim3(nb), dim3(kBlock), 0, st, to_lat(g), U, tol, part);
  return hipGetLastError();
}

hipError_t launch_convert_gauge(const LatArg& g, const void* U64, void* Ulow, hmc_prec prec, hipStream_t st) {
  dim3 grid(site_blocks(g.Vh), 8), block(kBlock);
  switch (prec) {
    case HMC_F32: hipLaunchKernelGGL(k_convert_gauge<LkF32>, grid, block, 0, st, to_lat(g), U64, Ulow); break;
    case HMC_F16: hipLaunchKernelGGL(k_convert_gauge<LkF16>, grid, block, 0, st, to_lat(g), U64, Ulow); break;
    case HMC_BF16: hipLaunchKernelGGL(k_convert_gauge<LkBF16>, grid, block, 0, st, to_lat(g), U64, Ulow); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class SI>
static hipError_t conv_out(const LatArg& g, const void* in, void* out, hmc_prec pout, int nbatch,
                           const void* const* tin, void* const* tout, hipStream_t st, const int* gate) {
  dim3 grid(site_blocks(g.Vh), nbatch), block(kBlock);
  switch (pout) {
    case HMC_F64: hipLaunchKernelGGL((k_convert_spinor<SI, SpF64>), grid, block, 0, st, to_lat(g), in, out, tin, tout, gate); break;
    case HMC_F32: hipLaunchKernelGGL((k_convert_spinor<SI, SpF32>), grid, block, 0, st, to_lat(g), in, out, tin, tout, gate); break;
    case HMC_F16: hipLaunchKernelGGL((k_convert_spinor<SI, SpF16>), grid, block, 0, st, to_lat(g), in, out, tin, tout, gate); break;
    case HMC_BF16: hipLaunchKernelGGL((k_convert_spinor<SI, SpBF16>), grid, block, 0, st, to_lat(g), in, out, tin, tout, gate); break;
  }
  return hipGetLastError();
}

hipError_t launch_convert_spinor(const LatArg& g, const void* in, hmc_prec pin, void* out, hmc_prec pout,
                                 int nbatch, const void* const* tab_in, void* const* tab_out, hipStream_t st,
                                 const int* gate) {
  switch (pin) {
    case HMC_F64: return conv_out<SpF64>(g, in, out, pout, nbatch, tab_in, tab_out, st, gate);
    case HMC_F32: return conv_out<SpF32>(g, in, out, pout, nbatch, tab_in, tab_out, st, gate);
    case HMC_F16: return conv_out<SpF16>(g, in, out, pout, nbatch, tab_in, tab_out, st, gate);
    case HMC_BF16: return conv_out<SpBF16>(g, in, out, pout, nbatch, tab_in, tab_out, st, gate);
  }
  return hipErrorInvalidValue;
}

}  // namespace hmc
