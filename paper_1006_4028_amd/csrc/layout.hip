// Layout kernels: host-order (x0 slowest, complex128 interleaved) fields to the
// structure-of-arrays parity layout and back, precision conversion, the source
// redefinition eta' = beta eta, the restoration S = S'/beta and the per-
// timeslice correlator C_PP(y0) = -sum_y tr[S^+ S] (heavy-quark section,
// restoration eq. backcorrection in the form C = C'/alpha^2).  beta(y) =
// alpha(y0) a_1(y1) a_2(y2) a_3(y3): the time profile alpha of eq. redeft and
// the spatial factors of the light-quark factorisation (eqs. redefa, betaa),
// which must be divided out site by site before the contraction.
#include <algorithm>

#include "dp_device.h"

namespace dp {

namespace {

// a_1(x1) a_2(x2) a_3(x3), or 1 without spatial profiles
__device__ __forceinline__ double space_factor(const Geom& g, const double* sprof, int x1, int x2, int x3) {
  return sprof ? sprof[x1] * sprof[g.L1 + x2] * sprof[g.L1 + g.L2 + x3] : 1.0;
}

__device__ __forceinline__ void lex_coords(const Geom& g, long s, int& x0, int& x1, int& x2, int& x3) {
  x3 = (int)(s % g.L3);
  s /= g.L3;
  x2 = (int)(s % g.L2);
  s /= g.L2;
  x1 = (int)(s % g.L1);
  x0 = (int)(s / g.L1);
}

template <int P>
__global__ void gauge_reorder_kernel(Geom g, const double2* __restrict__ U, void* e, void* o) {
  const long V = 2L * g.Vh;
  const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= V) return;
  int x0, x1, x2, x3;
  lex_coords(g, s, x0, x1, x2, x3);
  const int p = (x0 + x1 + x2 + x3) & 1;
  const int i = (int)(s >> 1);
  void* dst = p ? o : e;
  for (int mu = 0; mu < 4; ++mu)
    for (int k = 0; k < 9; ++k) {
      const double2 v = U ? U[(s * 4 + mu) * 9 + k] : make_double2((k % 4 == 0) ? 1.0 : 0.0, 0.0);
      const long at = (long)(mu * 9 + k) * g.Vp + i;
      if constexpr (P == F64) {
        static_cast<double2*>(dst)[at] = v;
      } else if constexpr (P == F32) {
        static_cast<float2*>(dst)[at] = make_float2((float)v.x, (float)v.y);
      } else {
        static_cast<unsigned*>(dst)[at] = f2h((float)v.x, (float)v.y);
      }
    }
}

// host-order spinors -> FP64 parity field, optionally times beta(x)
__global__ void spinor_import_kernel(Geom g, const double2* __restrict__ aos, long aos_ss, int p, SpinorRef dst,
                                     const double* __restrict__ amul, const double* __restrict__ sprof) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int slot = blockIdx.y;
  if (i >= g.Vh) return;
  int x0, x1, x2, x3;
  eo_coords(g, p, i, x0, x1, x2, x3);
  const long s = ((long)(x0 * g.L1 + x1) * g.L2 + x2) * g.L3 + x3;
  const double f = (amul ? amul[(long)slot * g.T + x0] : 1.0) * space_factor(g, sprof, x1, x2, x3);
  const double2* src = aos + slot * aos_ss + s * 12;
  double2* d = static_cast<double2*>(dst.data) + slot * dst.slot_stride;
  for (int c = 0; c < 12; ++c) {
    const double2 v = src[c];
    d[(long)c * g.Vp + i] = make_double2(f * v.x, f * v.y);
  }
}

// FP64 parity fields -> host-order spinors, optionally divided by beta(x)
__global__ void spinor_export_kernel(Geom g, SpinorRef e, SpinorRef o, const double* __restrict__ adiv,
                                     const double* __restrict__ sprof, double2* __restrict__ aos, long aos_ss) {
  const long V = 2L * g.Vh;
  const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int slot = blockIdx.y;
  if (s >= V) return;
  int x0, x1, x2, x3;
  lex_coords(g, s, x0, x1, x2, x3);
  const int p = (x0 + x1 + x2 + x3) & 1;
  const int i = (int)(s >> 1);
  const SpinorRef& f = p ? o : e;
  const double2* src = static_cast<const double2*>(f.data) + slot * f.slot_stride;
  const double inv = 1.0 / ((adiv ? adiv[(long)slot * g.T + x0] : 1.0) * space_factor(g, sprof, x1, x2, x3));
  double2* d = aos + slot * aos_ss + s * 12;
  for (int c = 0; c < 12; ++c) {
    const double2 v = src[(long)c * g.Vp + i];
    d[c] = make_double2(v.x * inv, v.y * inv);
  }
}

// One block per (timeslice, slot): -sum over both parities of |psi|^2 / beta^2
// (the time factor alpha^2 after the sum, the spatial ones per site).
__global__ void __launch_bounds__(kBlock) cpp_kernel(Geom g, SpinorRef e, SpinorRef o,
                                                     const double* __restrict__ alpha, const double* __restrict__ sprof,
                                                     const int* __restrict__ x0src, double* __restrict__ cpp) {
  const int x0 = blockIdx.x, slot = blockIdx.y;
  __shared__ double lds[kBlock / 64];
  double acc = 0.0;
  for (int par = 0; par < 2; ++par) {
    const SpinorRef& f = par ? o : e;
    const double2* src = static_cast<const double2*>(f.data) + slot * f.slot_stride;
    for (int k = threadIdx.x; k < g.Vsh; k += kBlock) {
      const int i = x0 * g.Vsh + k;
      double site = 0.0;
      for (int c = 0; c < 12; ++c) {
        const double2 v = src[(long)c * g.Vp + i];
        site += v.x * v.x + v.y * v.y;
      }
      if (sprof) {
        int y0, y1, y2, y3;
        eo_coords(g, par, i, y0, y1, y2, y3);
        const double f = space_factor(g, sprof, y1, y2, y3);
        site /= f * f;
      }
      acc += site;
    }
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += lds[w];
    const double a = alpha ? alpha[(long)slot * g.T + x0] : 1.0;
    const int t = ((x0 - (x0src ? x0src[slot] : 0)) % g.T + g.T) % g.T;
    cpp[(long)slot * g.T + t] = -s / (a * a);
  }
}

// Fill of ncols point-source columns (every entry written: no memset, so the
// launch may sit in a captured graph).  Grid-stride over the 12 V ncols
// complex entries.
__global__ void __launch_bounds__(kBlock) point_source_kernel(long per_col, long at, int c0, int ncols,
                                                              double2* __restrict__ out) {
  const long total = per_col * ncols;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
    const long j = k / per_col, r = k - j * per_col;
    out[k] = make_double2(r == at + c0 + j ? 1.0 : 0.0, 0.0);
  }
}

// The boundary sources of the Schroedinger functional, column j for
// c = c0 + j: side 0, U_0(x0 = 0, xs)^+ P+ e_c on the first interior
// timeslice, P+ = (1 + gamma_0)/2 (the projector of the backward time hop,
// so that this is the hop from a boundary field P+ psi(0) = e_c); side 1,
// U_0(x0 = T, xs) P- e_c on the last interior timeslice, P- = (1 -
// gamma_0)/2 (the forward time hop into the boundary field at x0 = T + 1);
// 0 elsewhere.  In the chiral basis gamma_0 has -1 between spins s and
// s +- 2, so P+- is 1/2 on the diagonal and -+1/2 between those spins.
// Ut: the time links of the boundary-adjacent timeslice, host layout
// [xs][mu][3][3]; the source timeslice starts at element site0 * 12.
__global__ void __launch_bounds__(kBlock) sf_wall_source_kernel(long per_col, long Vs, long site0, int side, int c0,
                                                                int ncols, const double2* __restrict__ Ut,
                                                                double2* __restrict__ out) {
  const long total = per_col * ncols;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
    const long j = k / per_col, r = k - j * per_col;
    const long site = r / 12 - site0;
    const int comp = (int)(r % 12), s = comp / 3, a = comp % 3;
    double2 v = make_double2(0.0, 0.0);
    if (site >= 0 && site < Vs) {  // the source timeslice
      const int c = c0 + (int)j, sc = c / 3, ac = c % 3;
      const double off = side == 0 ? -0.5 : 0.5;
      const double pp = s == sc ? 0.5 : ((s & 1) == (sc & 1) ? off : 0.0);
      if (side == 0) {  // (U^+)[a][ac] = conj(U[ac][a])
        const double2 u = Ut[(site * 4 + 0) * 9 + ac * 3 + a];
        v = make_double2(pp * u.x, -pp * u.y);
      } else {  // U[a][ac]
        const double2 u = Ut[(site * 4 + 0) * 9 + a * 3 + ac];
        v = make_double2(pp * u.x, pp * u.y);
      }
    }
    out[k] = v;
  }
}

}  // namespace

hipError_t launch_sf_wall_sources(const Geom& g, const double2* Ut, int side, int c0, int ncols, double2* out,
                                  hipStream_t st) {
  if (ncols <= 0 || c0 < 0 || c0 + ncols > 12 || (side != 0 && side != 1)) return hipErrorInvalidValue;
  const long per_col = 2L * g.Vh * 12;
  const long Vs = 2L * g.Vsh;
  const long site0 = side == 0 ? 0 : (long)(g.T - 1) * Vs;
  const long total = per_col * ncols;
  const long blocks = std::min<long>((total + kBlock - 1) / kBlock, 8L * 1024);
  hipLaunchKernelGGL(sf_wall_source_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, per_col, Vs, site0, side, c0,
                     ncols, Ut, out);
  return hipGetLastError();
}

hipError_t launch_point_sources(const Geom& g, const int site[4], int c0, int ncols, double2* out, hipStream_t st) {
  if (ncols <= 0 || c0 < 0 || c0 + ncols > 12) return hipErrorInvalidValue;
  const long per_col = 2L * g.Vh * 12;
  const long at = ((((long)site[0] * g.L1 + site[1]) * g.L2 + site[2]) * g.L3 + site[3]) * 12;
  const long total = per_col * ncols;
  const long blocks = std::min<long>((total + kBlock - 1) / kBlock, 8L * 1024);
  hipLaunchKernelGGL(point_source_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, per_col, at, c0, ncols, out);
  return hipGetLastError();
}

hipError_t launch_gauge_reorder(const Geom& g, const double2* U_aos, void* U_eo[2], int prec, hipStream_t st) {
  const long V = 2L * g.Vh;
  const dim3 grid((unsigned)((V + kBlock - 1) / kBlock));
  switch (prec) {
    case F64: hipLaunchKernelGGL(gauge_reorder_kernel<F64>, grid, dim3(kBlock), 0, st, g, U_aos, U_eo[0], U_eo[1]); break;
    case F32: hipLaunchKernelGGL(gauge_reorder_kernel<F32>, grid, dim3(kBlock), 0, st, g, U_aos, U_eo[0], U_eo[1]); break;
    case F16: hipLaunchKernelGGL(gauge_reorder_kernel<F16>, grid, dim3(kBlock), 0, st, g, U_aos, U_eo[0], U_eo[1]); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_spinor_import(const Geom& g, const double2* aos, int nslots, long aos_ss, int p, SpinorRef dst,
                                const double* alpha_mul, const double* sprof, hipStream_t st) {
  if (dst.prec != F64 || nslots <= 0) return hipErrorInvalidValue;
  const dim3 grid((g.Vh + kBlock - 1) / kBlock, nslots);
  hipLaunchKernelGGL(spinor_import_kernel, grid, dim3(kBlock), 0, st, g, aos, aos_ss, p, dst, alpha_mul, sprof);
  return hipGetLastError();
}

hipError_t launch_spinor_export(const Geom& g, SpinorRef even, SpinorRef odd, int nslots, const double* alpha_div,
                                const double* sprof, double2* aos, long aos_ss, hipStream_t st) {
  if (even.prec != F64 || odd.prec != F64 || nslots <= 0) return hipErrorInvalidValue;
  const long V = 2L * g.Vh;
  const dim3 grid((unsigned)((V + kBlock - 1) / kBlock), nslots);
  hipLaunchKernelGGL(spinor_export_kernel, grid, dim3(kBlock), 0, st, g, even, odd, alpha_div, sprof, aos, aos_ss);
  return hipGetLastError();
}

hipError_t launch_cpp(const Geom& g, SpinorRef even, SpinorRef odd, int nslots, const double* alpha,
                      const double* sprof, const int* x0src, double* cpp, hipStream_t st) {
  if (even.prec != F64 || odd.prec != F64 || nslots <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cpp_kernel, dim3(g.T, nslots), dim3(kBlock), 0, st, g, even, odd, alpha, sprof, x0src, cpp);
  return hipGetLastError();
}

}  // namespace dp
