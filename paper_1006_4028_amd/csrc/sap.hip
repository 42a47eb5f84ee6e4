// SAP+GCR: the domain-decomposition solver of the paper's light-quark
// iteration counts (Table 1, the Schwarz alternating procedure of the
// reference the paper cites for it) on the distance-preconditioned operator
// D' (time profile and the spatial profiles of the light-quark factorisation).
//
// The lattice is cut into blocks (an even number per direction) coloured by
// the parity of their block coordinates.  One application of the
// preconditioner, psi = M r, runs ncy cycles; each cycle treats colour 0, then
// colour 1: rho = (r - D' psi) on the blocks of that colour (zero elsewhere),
// then nmr minimal-residual steps on every block of the colour at once:
// a = D' rho (with rho zero off the colour, a on the colour's sites is the
// direct sum of the Dirichlet block operators, since touching blocks differ
// in colour), w_B = <a, rho>_B / <a, a>_B per block, psi += w_B rho,
// rho -= w_B a.  The block solves run in FP32 (or FP64); flexible GCR in FP64
// (restart length nkv) solves D' x = eta' with M on the right.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <complex>
#include <vector>

#include "dp_device.h"
#include "runtime.h"

using namespace dp;
using namespace dp::rt;

namespace dp {

namespace {

struct Blocking {
  int bs[4];     // block extents
  int nb[4];     // blocks per direction
  int vol;       // sites per block
  int nhalf;     // blocks of one colour
};

// the site's block colour
__device__ __forceinline__ int colour_of(const Blocking& b, int x0, int x1, int x2, int x3) {
  return (x0 / b.bs[0] + x1 / b.bs[1] + x2 / b.bs[2] + x3 / b.bs[3]) & 1;
}

// rho = colour-c part of (r - a) (a = D' psi; a null means psi = 0), zero
// elsewhere; grid over (sites of one parity, 2 parities)
template <int P>
__global__ void __launch_bounds__(kBlock) sap_residual_kernel(Geom g, Blocking b, int colour, SpinorRef r,
                                                              SpinorRef a, SpinorRef rho, int have_a) {
  using R = typename Tr<P>::R;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (i >= g.Vh) return;
  int x0, x1, x2, x3;
  eo_coords(g, p, i, x0, x1, x2, x3);
  cx<R> v[12];
  if (colour_of(b, x0, x1, x2, x3) == colour) {
    SpinorIO<P>::load(r, p, i, g.Vp, v);
    if (have_a) {
      cx<R> w[12];
      SpinorIO<P>::load(a, p, i, g.Vp, w);
#pragma unroll
      for (int c = 0; c < 12; ++c) v[c] = v[c] - w[c];
    }
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = cx<R>{R(0), R(0)};
  }
  SpinorIO<P>::store(rho, p, i, g.Vp, v);
}

// One minimal-residual step on every block of one colour: one workgroup per
// block, the block sums in FP64 in a fixed order, then psi += w rho, rho -= w a.
template <int P>
__global__ void __launch_bounds__(kBlock) sap_mr_kernel(Geom g, Blocking b, int colour, SpinorRef a, SpinorRef rho,
                                                        SpinorRef psi) {
  using R = typename Tr<P>::R;
  // the k-th block of this colour: the last block coordinate takes the parity
  int k = blockIdx.x;
  const int h3 = b.nb[3] / 2;
  int c3 = k % h3;
  k /= h3;
  const int c2 = k % b.nb[2];
  k /= b.nb[2];
  const int c1 = k % b.nb[1];
  const int c0 = k / b.nb[1];
  c3 = 2 * c3 + ((colour + c0 + c1 + c2) & 1);
  const int o0 = c0 * b.bs[0], o1 = c1 * b.bs[1], o2 = c2 * b.bs[2], o3 = c3 * b.bs[3];
  __shared__ double lds[3][kBlock / 64];
  __shared__ double wsh[2];
  double num_re = 0.0, num_im = 0.0, den = 0.0;
  for (int s = threadIdx.x; s < b.vol; s += kBlock) {
    int t = s;
    const int l3 = t % b.bs[3];
    t /= b.bs[3];
    const int l2 = t % b.bs[2];
    t /= b.bs[2];
    const int l1 = t % b.bs[1];
    const int l0 = t / b.bs[1];
    const int x0 = o0 + l0, x1 = o1 + l1, x2 = o2 + l2, x3 = o3 + l3;
    const int p = (x0 + x1 + x2 + x3) & 1;
    const int i = eo_index(g, x0, x1, x2, x3);
    cx<R> va[12], vr[12];
    SpinorIO<P>::load(a, p, i, g.Vp, va);
    SpinorIO<P>::load(rho, p, i, g.Vp, vr);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      num_re += (double)va[c].x * (double)vr[c].x + (double)va[c].y * (double)vr[c].y;
      num_im += (double)va[c].x * (double)vr[c].y - (double)va[c].y * (double)vr[c].x;
      den += (double)va[c].x * (double)va[c].x + (double)va[c].y * (double)va[c].y;
    }
  }
  num_re = wave_sum(num_re);
  num_im = wave_sum(num_im);
  den = wave_sum(den);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    lds[0][wv] = num_re;
    lds[1][wv] = num_im;
    lds[2][wv] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double nr = 0.0, ni = 0.0, d = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) {
      nr += lds[0][q];
      ni += lds[1][q];
      d += lds[2][q];
    }
    wsh[0] = d > 0.0 ? nr / d : 0.0;
    wsh[1] = d > 0.0 ? ni / d : 0.0;
  }
  __syncthreads();
  const cx<R> w{(R)wsh[0], (R)wsh[1]};
  for (int s = threadIdx.x; s < b.vol; s += kBlock) {
    int t = s;
    const int l3 = t % b.bs[3];
    t /= b.bs[3];
    const int l2 = t % b.bs[2];
    t /= b.bs[2];
    const int l1 = t % b.bs[1];
    const int l0 = t / b.bs[1];
    const int x0 = o0 + l0, x1 = o1 + l1, x2 = o2 + l2, x3 = o3 + l3;
    const int p = (x0 + x1 + x2 + x3) & 1;
    const int i = eo_index(g, x0, x1, x2, x3);
    cx<R> va[12], vr[12], vp[12];
    SpinorIO<P>::load(a, p, i, g.Vp, va);
    SpinorIO<P>::load(rho, p, i, g.Vp, vr);
    SpinorIO<P>::load(psi, p, i, g.Vp, vp);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      vp[c] = vp[c] + cmul(w, vr[c]);
      vr[c] = vr[c] - cmul(w, va[c]);
    }
    SpinorIO<P>::store(psi, p, i, g.Vp, vp);
    SpinorIO<P>::store(rho, p, i, g.Vp, vr);
  }
}

// ------------------------------------------------------------ vector kernels
// Full-lattice vectors are two-slot fields: slot p holds the sites of parity p.

// y = x converted between precisions
template <int PI, int PO>
__global__ void __launch_bounds__(kBlock) vec_convert_kernel(Geom g, SpinorRef x, SpinorRef y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (i >= g.Vh) return;
  cx<double> v[12];
  SpinorIO<PI>::load(x, p, i, g.Vp, v);
  SpinorIO<PO>::store(y, p, i, g.Vp, v);
}

// op 0: y += a x (a complex);  op 1: y = x - y;  op 2: y = 0;  op 3: y = x
// (2 and 3 do not read y, so that whatever a failed solve left in it is
// overwritten, not carried: 0 * NaN is NaN)
__global__ void __launch_bounds__(kBlock) vec_update_kernel(Geom g, int op, double ar, double ai, SpinorRef x,
                                                            SpinorRef y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (i >= g.Vh) return;
  cx<double> vx[12], vy[12];
  if (op <= 1) SpinorIO<F64>::load(y, p, i, g.Vp, vy);
  if (op != 2) SpinorIO<F64>::load(x, p, i, g.Vp, vx);
  const cx<double> a{ar, ai};
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    if (op == 0) vy[c] = vy[c] + cmul(a, vx[c]);
    else if (op == 1) vy[c] = vx[c] - vy[c];
    else if (op == 2) vy[c] = cx<double>{0.0, 0.0};
    else vy[c] = vx[c];
  }
  SpinorIO<F64>::store(y, p, i, g.Vp, vy);
}

// block partials of <x, y> (complex) over both parities: partials[blockIdx][2]
__global__ void __launch_bounds__(kBlock) vec_dot_kernel(Geom g, SpinorRef x, SpinorRef y, double* partials) {
  __shared__ double lds[2][kBlock / 64];
  double re = 0.0, im = 0.0;
  const long n = 2L * g.Vh;
  for (long s = (long)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (long)gridDim.x * blockDim.x) {
    const int p = (int)(s / g.Vh), i = (int)(s - (long)p * g.Vh);
    cx<double> vx[12], vy[12];
    SpinorIO<F64>::load(x, p, i, g.Vp, vx);
    SpinorIO<F64>::load(y, p, i, g.Vp, vy);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      re += vx[c].x * vy[c].x + vx[c].y * vy[c].y;
      im += vx[c].x * vy[c].y - vx[c].y * vy[c].x;
    }
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if ((threadIdx.x & 63) == 0) {
    lds[0][threadIdx.x >> 6] = re;
    lds[1][threadIdx.x >> 6] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) {
      a += lds[0][q];
      b += lds[1][q];
    }
    partials[2 * blockIdx.x] = a;
    partials[2 * blockIdx.x + 1] = b;
  }
}

// ------------------------------------------------------- fused block solves
//
// For blocks of at most kSapThreads sites the whole pass over one colour (the
// block residual, then nmr minimal-residual steps) runs as one kernel: a
// workgroup per block and a thread per site.  Each thread keeps its site's
// four forward links and clover blocks in registers for the pass; the block
// residual rho lives in LDS.  Of the hops inside a block, the forward one at x
// reads rho(x + mu) from LDS and multiplies by the thread's own link; the
// backward one at x needs U_mu(x - mu)^+ applied to rho(x - mu), which the
// thread of x - mu forms with its own link and leaves in LDS for x.  Hops that
// leave the block drop (Dirichlet block boundaries).
//
// The fields of the pass are stored block by block ("block layout"): the
// blocks of colour 0 in the order of their index k, then those of colour 1;
// each block as component arrays over its sites s = ((l0 b1 + l1) b2 + l2) b3
// + l3 (l = coordinates within the block), so that the lanes of a wave, one
// site each, read consecutive addresses.  Spinors: float4 [6][vol] per block
// (components 2q, 2q + 1); links: float2 [4][9][vol]; clover: float4 [18][vol]
// (the packed blocks of the parity fields).

constexpr int kSapThreads = 256;

struct BLoc {
  int blk, s;
};

// block-layout position of site x
__device__ __forceinline__ BLoc bl_locate(const Blocking& b, int x0, int x1, int x2, int x3) {
  const int c0 = x0 / b.bs[0], c1 = x1 / b.bs[1], c2 = x2 / b.bs[2], c3 = x3 / b.bs[3];
  const int colour = (c0 + c1 + c2 + c3) & 1;
  const int k = ((c0 * b.nb[1] + c1) * b.nb[2] + c2) * (b.nb[3] / 2) + c3 / 2;
  const int s = (((x0 - c0 * b.bs[0]) * b.bs[1] + (x1 - c1 * b.bs[1])) * b.bs[2] + (x2 - c2 * b.bs[2])) * b.bs[3] +
                (x3 - c3 * b.bs[3]);
  return {colour * b.nhalf + k, s};
}

// FP32 links and clover of both parities -> block layout
__global__ void __launch_bounds__(kBlock) sap_gather_kernel(Geom g, Blocking b, const float2* __restrict__ U0,
                                                            const float2* __restrict__ U1,
                                                            const float4* __restrict__ C0,
                                                            const float4* __restrict__ C1, float2* __restrict__ ubl,
                                                            float4* __restrict__ cbl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (i >= g.Vh) return;
  int x0, x1, x2, x3;
  eo_coords(g, p, i, x0, x1, x2, x3);
  const BLoc q = bl_locate(b, x0, x1, x2, x3);
  const float2* U = p ? U1 : U0;
  const float4* C = p ? C1 : C0;
  for (int k = 0; k < 36; ++k) ubl[((long)q.blk * 36 + k) * b.vol + q.s] = U[(long)k * g.Vp + i];
  for (int k = 0; k < 18; ++k) cbl[((long)q.blk * 18 + k) * b.vol + q.s] = C[(long)k * g.Vp + i];
}

// FP64 parity fields -> FP32 block layout
__global__ void __launch_bounds__(kBlock) sap_to_block_kernel(Geom g, Blocking b, SpinorRef x,
                                                              float4* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (i >= g.Vh) return;
  int x0, x1, x2, x3;
  eo_coords(g, p, i, x0, x1, x2, x3);
  const BLoc q = bl_locate(b, x0, x1, x2, x3);
  cx<double> v[12];
  SpinorIO<F64>::load(x, p, i, g.Vp, v);
#pragma unroll
  for (int k = 0; k < 6; ++k)
    out[((long)q.blk * 6 + k) * b.vol + q.s] =
        make_float4((float)v[2 * k].x, (float)v[2 * k].y, (float)v[2 * k + 1].x, (float)v[2 * k + 1].y);
}

// FP32 block layout -> FP64 parity fields
__global__ void __launch_bounds__(kBlock) sap_from_block_kernel(Geom g, Blocking b, const float4* __restrict__ in,
                                                                SpinorRef y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (i >= g.Vh) return;
  int x0, x1, x2, x3;
  eo_coords(g, p, i, x0, x1, x2, x3);
  const BLoc q = bl_locate(b, x0, x1, x2, x3);
  cx<double> v[12];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float4 f = in[((long)q.blk * 6 + k) * b.vol + q.s];
    v[2 * k] = cx<double>{f.x, f.y};
    v[2 * k + 1] = cx<double>{f.z, f.w};
  }
  SpinorIO<F64>::store(y, p, i, g.Vp, v);
}

// Spin projection in the chiral basis (psi = (u0, u1, l0, l1) in spin, as in
// the hop kernels): (1 - sg gamma_mu) psi is determined by its upper half h;
// the lower half is a fixed spin rotation of h.
template <int MU, int SG>
__device__ __forceinline__ void bl_proj(const cx<float> (&v)[12], cx<float> (&h)[6]) {
  constexpr float sg = (float)SG;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cx<float> u0 = v[a], u1 = v[3 + a], l0 = v[6 + a], l1 = v[9 + a];
    if constexpr (MU == 0) {
      h[a] = u0 + sg * l0;
      h[3 + a] = u1 + sg * l1;
    } else if constexpr (MU == 1) {
      h[a] = u0 + sg * ti(l1);
      h[3 + a] = u1 + sg * ti(l0);
    } else if constexpr (MU == 2) {
      h[a] = u0 + sg * l1;
      h[3 + a] = u1 - sg * l0;
    } else {
      h[a] = u0 + sg * ti(l0);
      h[3 + a] = u1 - sg * ti(l1);
    }
  }
}

// acc += c * (the full spinor whose upper half is w, of projector (1 - sg gamma_mu))
template <int MU, int SG>
__device__ __forceinline__ void bl_recon(cx<float> (&acc)[12], const cx<float> (&w)[6], float c) {
  constexpr float sg = (float)SG;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cx<float> w0 = c * w[a], w1 = c * w[3 + a];
    acc[a] = acc[a] + w0;
    acc[3 + a] = acc[3 + a] + w1;
    if constexpr (MU == 0) {
      acc[6 + a] = acc[6 + a] + sg * w0;
      acc[9 + a] = acc[9 + a] + sg * w1;
    } else if constexpr (MU == 1) {
      acc[6 + a] = acc[6 + a] - sg * ti(w1);
      acc[9 + a] = acc[9 + a] - sg * ti(w0);
    } else if constexpr (MU == 2) {
      acc[6 + a] = acc[6 + a] - sg * w1;
      acc[9 + a] = acc[9 + a] + sg * w0;
    } else {
      acc[6 + a] = acc[6 + a] - sg * ti(w0);
      acc[9 + a] = acc[9 + a] + sg * ti(w1);
    }
  }
}

// o = U h (DAG: U^+ h) on both spin components of a half spinor
template <bool DAG>
__device__ __forceinline__ void bl_link(const cx<float> (&u)[9], const cx<float> (&h)[6], cx<float> (&o)[6]) {
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<float> t;
      if constexpr (DAG) {
        t = cjmul(u[a], h[3 * sp]);
        cjfma(t, u[3 + a], h[3 * sp + 1]);
        cjfma(t, u[6 + a], h[3 * sp + 2]);
      } else {
        t = cmul(u[3 * a], h[3 * sp]);
        cfma(t, u[3 * a + 1], h[3 * sp + 1]);
        cfma(t, u[3 * a + 2], h[3 * sp + 2]);
      }
      o[3 * sp + a] = t;
    }
}

// y = (C + m4) x with the site's clover blocks read from the block layout,
// one chirality at a time
__device__ __forceinline__ void bl_diag(const float4* C, int blk, int vol, int s, float m4, const cx<float> (&x)[12],
                                        cx<float> (&y)[12]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float raw[36];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const float4 v = C[((long)blk * 18 + 9 * h + q) * vol + s];
      raw[4 * q] = v.x;
      raw[4 * q + 1] = v.y;
      raw[4 * q + 2] = v.z;
      raw[4 * q + 3] = v.w;
    }
    HermBlock<float> B;
#pragma unroll
    for (int q = 0; q < 6; ++q) B.d[q] = raw[q];
#pragma unroll
    for (int q = 0; q < 15; ++q) B.o[q] = cx<float>{raw[6 + 2 * q], raw[7 + 2 * q]};
    herm_apply(B, m4, &x[6 * h], &y[6 * h]);
  }
}

__device__ __forceinline__ void bl_load_spinor(const float4* f, long base, int vol, int s, cx<float> (&v)[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float4 q = f[(base + k) * vol + s];
    v[2 * k] = cx<float>{q.x, q.y};
    v[2 * k + 1] = cx<float>{q.z, q.w};
  }
}

struct SapPass {
  Geom g;
  Blocking b;
  int colour;
  int nmr;
  int own_zero;  // psi of the pass's blocks is still zero (not read)
  const float4* r;
  float4* psi;
  const float2* U;
  const float4* C;
  float4* av;            // the large-block kernel's D'_B rho between its two phases (block layout)
  const double* rt;      // time hop ratios [4][T] (fwd, bwd, ...; boundary sign folded in)
  const double* sratio;  // spatial hop ratios of the light-quark factorisation, or null
  float m4;              // 4 + M
};

// the origin of the kidx-th block of a colour
__device__ __forceinline__ void bl_origin(const Blocking& b, int colour, int kidx, int (&o)[4]) {
  const int h3 = b.nb[3] / 2;
  int c3 = kidx % h3;
  kidx /= h3;
  const int c2 = kidx % b.nb[2];
  kidx /= b.nb[2];
  const int c1 = kidx % b.nb[1];
  const int c0 = kidx / b.nb[1];
  c3 = 2 * c3 + ((colour + c0 + c1 + c2) & 1);
  o[0] = c0 * b.bs[0];
  o[1] = c1 * b.bs[1];
  o[2] = c2 * b.bs[2];
  o[3] = c3 * b.bs[3];
}

// coordinates within its block of the block's site s
__device__ __forceinline__ void bl_local(const Blocking& b, int s, int (&l)[4]) {
  l[3] = s % b.bs[3];
  s /= b.bs[3];
  l[2] = s % b.bs[2];
  s /= b.bs[2];
  l[1] = s % b.bs[1];
  l[0] = s / b.bs[1];
}

// hop coefficients at x: time ratios, spatial ratios (or 1)
__device__ __forceinline__ void bl_coefs(const SapPass& a, const int (&x)[4], float (&cf)[4], float (&cb)[4]) {
  const Geom& g = a.g;
  const int Ls[4] = {g.T, g.L1, g.L2, g.L3};
  cf[0] = (float)a.rt[x[0]];
  cb[0] = (float)a.rt[g.T + x[0]];
  int off = 0;
#pragma unroll
  for (int mu = 1; mu < 4; ++mu) {
    cf[mu] = a.sratio ? (float)a.sratio[off + x[mu]] : 1.f;
    cb[mu] = a.sratio ? (float)a.sratio[off + Ls[mu] + x[mu]] : 1.f;
    off += 4 * Ls[mu];
  }
}

__device__ __forceinline__ void bl_load_link(const float2* U, int blk, int mu, int vol, int s, cx<float> (&u)[9]) {
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const float2 v = U[((long)blk * 36 + mu * 9 + q) * vol + s];
    u[q] = cx<float>{v.x, v.y};
  }
}

// out = D' psi at site x (site s of block blk), psi from memory, every
// neighbour inside or outside the block; with own_zero the psi of block blk is
// zero and not read.  REG: the site's forward links are Ureg.
template <bool REG, int MU>
__device__ __forceinline__ void bl_dprime_dir(const SapPass& a, int blk, const int (&x)[4], float cfm, float cbm,
                                              const cx<float> (&Ureg)[4][9], int s, cx<float> (&out)[12]) {
  const Geom& g = a.g;
  const Blocking& b = a.b;
  const int L = MU == 0 ? g.T : MU == 1 ? g.L1 : MU == 2 ? g.L2 : g.L3;
  cx<float> v[12], h[6], w[6], u[9];
  int y[4] = {x[0], x[1], x[2], x[3]};
  y[MU] = x[MU] + 1 == L ? 0 : x[MU] + 1;
  BLoc q = bl_locate(b, y[0], y[1], y[2], y[3]);
  if (!(a.own_zero && q.blk == blk)) {
    bl_load_spinor(a.psi, (long)q.blk * 6, b.vol, q.s, v);
    bl_proj<MU, 1>(v, h);
    if constexpr (REG) {
      bl_link<false>(Ureg[MU], h, w);
    } else {
      bl_load_link(a.U, blk, MU, b.vol, s, u);
      bl_link<false>(u, h, w);
    }
    bl_recon<MU, 1>(out, w, -0.5f * cfm);
  }
  y[MU] = x[MU] == 0 ? L - 1 : x[MU] - 1;
  q = bl_locate(b, y[0], y[1], y[2], y[3]);
  if (!(a.own_zero && q.blk == blk)) {
    bl_load_link(a.U, q.blk, MU, b.vol, q.s, u);
    bl_load_spinor(a.psi, (long)q.blk * 6, b.vol, q.s, v);
    bl_proj<MU, -1>(v, h);
    bl_link<true>(u, h, w);
    bl_recon<MU, -1>(out, w, -0.5f * cbm);
  }
}

template <bool REG>
__device__ __forceinline__ void bl_dprime(const SapPass& a, int blk, int s, const int (&x)[4], const float (&cf)[4],
                                          const float (&cb)[4], const cx<float> (&Ureg)[4][9],
                                          cx<float> (&out)[12]) {
  if (!a.own_zero) {
    cx<float> v[12];
    bl_load_spinor(a.psi, (long)blk * 6, a.b.vol, s, v);
    bl_diag(a.C, blk, a.b.vol, s, a.m4, v, out);
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) out[c] = cx<float>{0.f, 0.f};
  }
  bl_dprime_dir<REG, 0>(a, blk, x, cf[0], cb[0], Ureg, s, out);
  bl_dprime_dir<REG, 1>(a, blk, x, cf[1], cb[1], Ureg, s, out);
  bl_dprime_dir<REG, 2>(a, blk, x, cf[2], cb[2], Ureg, s, out);
  bl_dprime_dir<REG, 3>(a, blk, x, cf[3], cb[3], Ureg, s, out);
}

// the minimal-residual coefficient w = <a, rho>_B / |a|^2_B from per-thread
// FP64 partials: wave sums, then the waves in order (every thread calls it)
template <int NT>
__device__ __forceinline__ cx<float> bl_mr_coef(double nr, double ni, double dn, double (&red)[3][NT / 64],
                                                double (&wsh)[2]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  nr = wave_sum(nr);
  ni = wave_sum(ni);
  dn = wave_sum(dn);
  if (lane == 0) {
    red[0][wv] = nr;
    red[1][wv] = ni;
    red[2][wv] = dn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sr = 0.0, si = 0.0, sd = 0.0;
    for (int q = 0; q < NT / 64; ++q) {
      sr += red[0][q];
      si += red[1][q];
      sd += red[2][q];
    }
    wsh[0] = sd > 0.0 ? sr / sd : 0.0;
    wsh[1] = sd > 0.0 ? si / sd : 0.0;
  }
  __syncthreads();
  return cx<float>{(float)wsh[0], (float)wsh[1]};
}

__device__ __forceinline__ void bl_mr_sums(const cx<float> (&av)[12], const cx<float> (&rv)[12], double& nr,
                                           double& ni, double& dn) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    nr += (double)av[c].x * (double)rv[c].x + (double)av[c].y * (double)rv[c].y;
    ni += (double)av[c].x * (double)rv[c].y - (double)av[c].y * (double)rv[c].x;
    dn += (double)av[c].x * (double)av[c].x + (double)av[c].y * (double)av[c].y;
  }
}

__device__ __forceinline__ void bl_store_psi(const SapPass& a, int blk, int s, const cx<float> (&dpsi)[12]) {
  cx<float> v[12];
  if (a.own_zero) {
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = dpsi[c];
  } else {
    bl_load_spinor(a.psi, (long)blk * 6, a.b.vol, s, v);
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = v[c] + dpsi[c];
  }
#pragma unroll
  for (int q = 0; q < 6; ++q)
    a.psi[((long)blk * 6 + q) * a.b.vol + s] = make_float4(v[2 * q].x, v[2 * q].y, v[2 * q + 1].x, v[2 * q + 1].y);
}

// One pass of the Schwarz procedure over the blocks of one colour:
// rho = r - D' psi on the block (NB_ZERO: psi = 0 everywhere, rho = r), nmr
// minimal-residual steps with the Dirichlet block operator, psi += the
// accumulated correction.  Block sums in FP64, reduced in a fixed order.
// Blocks of at most kSapThreads sites, a thread per site.
template <bool NB_ZERO>
__global__ void __launch_bounds__(kSapThreads, 2) sap_block_kernel(SapPass a) {
  __shared__ float rho_l[24 * kSapThreads];
  __shared__ float hb[4 * 12 * kSapThreads];  // backward hops handed to x + mu
  __shared__ double red[3][kSapThreads / 64];
  __shared__ double wsh[2];
  const Blocking& b = a.b;
  const int s = threadIdx.x;
  const bool valid = s < b.vol;
  const int blk = a.colour * b.nhalf + blockIdx.x;
  const int st[4] = {b.bs[1] * b.bs[2] * b.bs[3], b.bs[2] * b.bs[3], b.bs[3], 1};
  int o[4], l[4];
  bl_origin(b, a.colour, blockIdx.x, o);
  bl_local(b, valid ? s : 0, l);
  const int x[4] = {o[0] + l[0], o[1] + l[1], o[2] + l[2], o[3] + l[3]};
  float cf[4], cb[4];
  bl_coefs(a, x, cf, cb);
  // the site's forward links, kept for the pass (the clover blocks are
  // read again at each use: holding them too would halve the waves per SIMD)
  cx<float> U[4][9];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) bl_load_link(a.U, blk, mu, b.vol, valid ? s : 0, U[mu]);
  // block residual
  if (valid) {
    cx<float> rv[12];
    bl_load_spinor(a.r, (long)blk * 6, b.vol, s, rv);
    if constexpr (!NB_ZERO) {
      cx<float> out[12];
      bl_dprime<true>(a, blk, s, x, cf, cb, U, out);
#pragma unroll
      for (int c = 0; c < 12; ++c) rv[c] = rv[c] - out[c];
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      rho_l[(2 * c) * kSapThreads + s] = rv[c].x;
      rho_l[(2 * c + 1) * kSapThreads + s] = rv[c].y;
    }
  }
  cx<float> dpsi[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) dpsi[c] = cx<float>{0.f, 0.f};
  for (int it = 0; it < a.nmr; ++it) {
    __syncthreads();  // rho complete
    cx<float> rv[12];
#pragma unroll
    for (int c = 0; c < 12; ++c)
      rv[c] = cx<float>{rho_l[(2 * c) * kSapThreads + s], rho_l[(2 * c + 1) * kSapThreads + s]};
    // hand the backward hops to the sites x + mu of the block
    if (valid) {
      cx<float> h[6], w[6];
#define DP_SAP_PUSH(MU)                                                \
  if (l[MU] + 1 < b.bs[MU]) {                                          \
    bl_proj<MU, -1>(rv, h);                                            \
    bl_link<true>(U[MU], h, w);                                        \
    for (int e = 0; e < 6; ++e) {                                      \
      hb[((MU * 12) + 2 * e) * kSapThreads + s + st[MU]] = w[e].x;     \
      hb[((MU * 12) + 2 * e + 1) * kSapThreads + s + st[MU]] = w[e].y; \
    }                                                                  \
  }
      DP_SAP_PUSH(0)
      DP_SAP_PUSH(1)
      DP_SAP_PUSH(2)
      DP_SAP_PUSH(3)
#undef DP_SAP_PUSH
    }
    __syncthreads();
    // av = D'_B rho at x: the diagonal term, then the hops with -1/2 folded
    // into their coefficients
    cx<float> av[12];
    double nr = 0.0, ni = 0.0, dn = 0.0;
    if (valid) {
      cx<float> v[12], h[6], w[6];
      bl_diag(a.C, blk, b.vol, s, a.m4, rv, av);
#define DP_SAP_PULL(MU)                                                                                 \
  if (l[MU] + 1 < b.bs[MU]) {                                                                           \
    const int n = s + st[MU];                                                                           \
    for (int c = 0; c < 12; ++c)                                                                        \
      v[c] = cx<float>{rho_l[(2 * c) * kSapThreads + n], rho_l[(2 * c + 1) * kSapThreads + n]};         \
    bl_proj<MU, 1>(v, h);                                                                               \
    bl_link<false>(U[MU], h, w);                                                                        \
    bl_recon<MU, 1>(av, w, -0.5f * cf[MU]);                                                             \
  }                                                                                                     \
  if (l[MU] > 0) {                                                                                      \
    for (int e = 0; e < 6; ++e)                                                                         \
      w[e] = cx<float>{hb[((MU * 12) + 2 * e) * kSapThreads + s], hb[((MU * 12) + 2 * e + 1) * kSapThreads + s]}; \
    bl_recon<MU, -1>(av, w, -0.5f * cb[MU]);                                                            \
  }
      DP_SAP_PULL(0)
      DP_SAP_PULL(1)
      DP_SAP_PULL(2)
      DP_SAP_PULL(3)
#undef DP_SAP_PULL
      bl_mr_sums(av, rv, nr, ni, dn);
    }
    const cx<float> w = bl_mr_coef<kSapThreads>(nr, ni, dn, red, wsh);
    if (valid) {
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        dpsi[c] = dpsi[c] + cmul(w, rv[c]);
        rv[c] = rv[c] - cmul(w, av[c]);
        rho_l[(2 * c) * kSapThreads + s] = rv[c].x;
        rho_l[(2 * c + 1) * kSapThreads + s] = rv[c].y;
      }
    }
  }
  if (valid) bl_store_psi(a, blk, s, dpsi);
}

// The same pass for blocks of kSapThreads + 1 .. kSapBigSites sites:
// kSapBigThreads threads with kSapBigPer sites each (site s = thread + q
// kSapBigThreads); the residual in LDS as before, but the links are read at
// each use, both hops of a site read rho from LDS (no hand-over buffer), and
// D'_B rho and psi stay in memory between the phases of a step, so that a
// block of up to 1536 sites fits.
constexpr int kSapBigThreads = 512;
constexpr int kSapBigPer = 3;
constexpr int kSapBigSites = kSapBigThreads * kSapBigPer;

template <bool NB_ZERO>
__global__ void __launch_bounds__(kSapBigThreads, 2) sap_block_big_kernel(SapPass a) {
  __shared__ float rho_l[24 * kSapBigSites];
  __shared__ double red[3][kSapBigThreads / 64];
  __shared__ double wsh[2];
  const Blocking& b = a.b;
  const int blk = a.colour * b.nhalf + blockIdx.x;
  const int st[4] = {b.bs[1] * b.bs[2] * b.bs[3], b.bs[2] * b.bs[3], b.bs[3], 1};
  int o[4];
  bl_origin(b, a.colour, blockIdx.x, o);
  const cx<float> Unone[4][9] = {};
  // block residual
#pragma unroll 1
  for (int q = 0; q < kSapBigPer; ++q) {
    const int s = threadIdx.x + q * kSapBigThreads;
    if (s < b.vol) {
      int l[4];
      bl_local(b, s, l);
      const int x[4] = {o[0] + l[0], o[1] + l[1], o[2] + l[2], o[3] + l[3]};
      cx<float> rv[12];
      bl_load_spinor(a.r, (long)blk * 6, b.vol, s, rv);
      if constexpr (!NB_ZERO) {
        float cf[4], cb[4];
        bl_coefs(a, x, cf, cb);
        cx<float> out[12];
        bl_dprime<false>(a, blk, s, x, cf, cb, Unone, out);
#pragma unroll
        for (int c = 0; c < 12; ++c) rv[c] = rv[c] - out[c];
      }
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        rho_l[(2 * c) * kSapBigSites + s] = rv[c].x;
        rho_l[(2 * c + 1) * kSapBigSites + s] = rv[c].y;
      }
    }
  }
  for (int it = 0; it < a.nmr; ++it) {
    __syncthreads();  // rho complete
    double nr = 0.0, ni = 0.0, dn = 0.0;
#pragma unroll 1
    for (int q = 0; q < kSapBigPer; ++q) {
      const int s = threadIdx.x + q * kSapBigThreads;
      if (s < b.vol) {
        int l[4];
        bl_local(b, s, l);
        const int x[4] = {o[0] + l[0], o[1] + l[1], o[2] + l[2], o[3] + l[3]};
        float cf[4], cb[4];
        bl_coefs(a, x, cf, cb);
        cx<float> rv[12], av[12], v[12], h[6], w[6], u[9];
#pragma unroll
        for (int c = 0; c < 12; ++c)
          rv[c] = cx<float>{rho_l[(2 * c) * kSapBigSites + s], rho_l[(2 * c + 1) * kSapBigSites + s]};
        bl_diag(a.C, blk, b.vol, s, a.m4, rv, av);
#define DP_SAP_BIG(MU)                                                                                   \
  if (l[MU] + 1 < b.bs[MU]) {                                                                            \
    const int n = s + st[MU];                                                                            \
    for (int c = 0; c < 12; ++c)                                                                         \
      v[c] = cx<float>{rho_l[(2 * c) * kSapBigSites + n], rho_l[(2 * c + 1) * kSapBigSites + n]};        \
    bl_proj<MU, 1>(v, h);                                                                                \
    bl_load_link(a.U, blk, MU, b.vol, s, u);                                                             \
    bl_link<false>(u, h, w);                                                                             \
    bl_recon<MU, 1>(av, w, -0.5f * cf[MU]);                                                              \
  }                                                                                                      \
  if (l[MU] > 0) {                                                                                       \
    const int n = s - st[MU];                                                                            \
    for (int c = 0; c < 12; ++c)                                                                         \
      v[c] = cx<float>{rho_l[(2 * c) * kSapBigSites + n], rho_l[(2 * c + 1) * kSapBigSites + n]};        \
    bl_proj<MU, -1>(v, h);                                                                               \
    bl_load_link(a.U, blk, MU, b.vol, n, u);                                                             \
    bl_link<true>(u, h, w);                                                                              \
    bl_recon<MU, -1>(av, w, -0.5f * cb[MU]);                                                             \
  }
        DP_SAP_BIG(0)
        DP_SAP_BIG(1)
        DP_SAP_BIG(2)
        DP_SAP_BIG(3)
#undef DP_SAP_BIG
        bl_mr_sums(av, rv, nr, ni, dn);
#pragma unroll
        for (int e = 0; e < 6; ++e)
          a.av[((long)blk * 6 + e) * b.vol + s] = make_float4(av[2 * e].x, av[2 * e].y, av[2 * e + 1].x, av[2 * e + 1].y);
      }
    }
    const cx<float> w = bl_mr_coef<kSapBigThreads>(nr, ni, dn, red, wsh);
#pragma unroll 1
    for (int q = 0; q < kSapBigPer; ++q) {
      const int s = threadIdx.x + q * kSapBigThreads;
      if (s < b.vol) {
        cx<float> rv[12], dp[12], av[12];
        bl_load_spinor(a.av, (long)blk * 6, b.vol, s, av);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          rv[c] = cx<float>{rho_l[(2 * c) * kSapBigSites + s], rho_l[(2 * c + 1) * kSapBigSites + s]};
          dp[c] = cmul(w, rv[c]);
          rv[c] = rv[c] - cmul(w, av[c]);
          rho_l[(2 * c) * kSapBigSites + s] = rv[c].x;
          rho_l[(2 * c + 1) * kSapBigSites + s] = rv[c].y;
        }
        // psi += w rho (psi of the block is read only by this workgroup)
        if (!(a.own_zero && it == 0)) {
          cx<float> pv[12];
          bl_load_spinor(a.psi, (long)blk * 6, b.vol, s, pv);
#pragma unroll
          for (int c = 0; c < 12; ++c) dp[c] = pv[c] + dp[c];
        }
#pragma unroll
        for (int e = 0; e < 6; ++e)
          a.psi[((long)blk * 6 + e) * b.vol + s] = make_float4(dp[2 * e].x, dp[2 * e].y, dp[2 * e + 1].x, dp[2 * e + 1].y);
      }
    }
  }
}

constexpr int kDotBlocks = 1024;

// The sum of the block partials of vec_dot_kernel in block order (the order
// the host used), on the device: out = <x, y> (mode 0), out = (|x|, 0)
// (mode 1), or <x, y> unless guard[0] (a norm) is zero or not finite, then 0
// (mode 2).
__global__ void __launch_bounds__(64) dot_finish_kernel(const double* __restrict__ partials, int mode,
                                                        const double* __restrict__ guard, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double re = 0.0, im = 0.0;
  for (int k = 0; k < kDotBlocks; ++k) {
    re += partials[2 * k];
    im += partials[2 * k + 1];
  }
  if (mode == 1) {
    re = sqrt(re);
    im = 0.0;
  } else if (mode == 2 && !(guard[0] > 0.0 && isfinite(guard[0]))) {
    re = im = 0.0;
  }
  out[0] = re;
  out[1] = im;
}

// One Gram-Schmidt step of GCR in one pass: the update of y with its
// coefficient on the device (op 0: y += sgn coef x, coef complex; op 1:
// y = y / coef[0], a norm, y left alone when it is zero or not finite), then
// the block partials of a dot product involving the updated y, as
// vec_dot_kernel forms them (same grid, order and arithmetic): dmode 0:
// <z, y>, 1: <y, z>, 2: <y, y>.
__global__ void __launch_bounds__(kBlock) vec_update_dot_kernel(Geom g, int op, const double* __restrict__ coef,
                                                                double sgn, SpinorRef x, SpinorRef y, int dmode,
                                                                SpinorRef z, double* __restrict__ partials) {
  __shared__ double lds[2][kBlock / 64];
  const double c0 = coef[0], c1 = coef[1];
  const bool skip = op == 1 && !(c0 > 0.0 && isfinite(c0));
  double re = 0.0, im = 0.0;
  const long n = 2L * g.Vh;
  for (long s = (long)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (long)gridDim.x * blockDim.x) {
    const int p = (int)(s / g.Vh), i = (int)(s - (long)p * g.Vh);
    cx<double> vx[12], vy[12];
    SpinorIO<F64>::load(y, p, i, g.Vp, vy);
    if (!skip) {
      if (op == 0) {
        SpinorIO<F64>::load(x, p, i, g.Vp, vx);
        const cx<double> a{sgn * c0, sgn * c1};
#pragma unroll
        for (int c = 0; c < 12; ++c) vy[c] = vy[c] + cmul(a, vx[c]);
      } else {
        const double ar = 1.0 / c0;
#pragma unroll
        for (int c = 0; c < 12; ++c) vy[c] = ar * vy[c];
      }
      SpinorIO<F64>::store(y, p, i, g.Vp, vy);
    }
    if (dmode == 2) {
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        re += vy[c].x * vy[c].x + vy[c].y * vy[c].y;
        im += vy[c].x * vy[c].y - vy[c].y * vy[c].x;
      }
    } else {
      SpinorIO<F64>::load(z, p, i, g.Vp, vx);
      if (dmode == 0) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          re += vx[c].x * vy[c].x + vx[c].y * vy[c].y;
          im += vx[c].x * vy[c].y - vx[c].y * vy[c].x;
        }
      } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          re += vy[c].x * vx[c].x + vy[c].y * vx[c].y;
          im += vy[c].x * vx[c].y - vy[c].y * vx[c].x;
        }
      }
    }
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if ((threadIdx.x & 63) == 0) {
    lds[0][threadIdx.x >> 6] = re;
    lds[1][threadIdx.x >> 6] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) {
      a += lds[0][q];
      b += lds[1][q];
    }
    partials[2 * blockIdx.x] = a;
    partials[2 * blockIdx.x + 1] = b;
  }
}


}  // namespace

// -------------------------------------------------------------- host driver

struct SapState {
  Geom g{};
  int nkv = 0;
  int prec = F32;
  Field eta, x, r, t;      // FP64 full-lattice vectors
  std::vector<Field> z, w;  // FP64, nkv each
  Field q_r, q_psi, q_rho, q_a;  // block-solve precision
  DevBuf ratio, m4, partials, alpha, cpp;
  // GCR coefficients on the device: c_jk [nkv][nkv], gamma_k [nkv], b_k
  // [nkv] (complex pairs), |r|^2; and their host copy
  DevBuf gcr;
  std::vector<double> h_gcr;
  // fused block solves: links, clover, r and psi in block layout (FP32)
  bool fused = false;
  DevBuf ubl, cbl, rbl, pbl, abl;
  std::vector<double> h_part;
};

namespace {

using zc = std::complex<double>;

size_t gcr_len(int nkv) { return (size_t)2 * nkv * nkv + 4 * nkv + 2; }
size_t gcr_cc(int nkv, int j, int k) { return (size_t)2 * (j * nkv + k); }
size_t gcr_gam(int nkv, int k) { return (size_t)2 * nkv * nkv + 2 * k; }
size_t gcr_bn(int nkv, int k) { return (size_t)2 * nkv * nkv + 2 * nkv + 2 * k; }
size_t gcr_rn(int nkv) { return (size_t)2 * nkv * nkv + 4 * nkv; }

int sap_alloc(dp_ctx* c, SapState& s, int nkv, int prec) {
  const Geom& g = c->g;
  Field* f64[] = {&s.eta, &s.x, &s.r, &s.t};
  for (Field* f : f64) DP_HIP(c, f->alloc(g, F64, 2));
  if ((int)s.z.size() < nkv) {
    s.z = std::vector<Field>(nkv);
    s.w = std::vector<Field>(nkv);
  }
  for (int k = 0; k < nkv; ++k) {
    DP_HIP(c, s.z[k].alloc(g, F64, 2));
    DP_HIP(c, s.w[k].alloc(g, F64, 2));
  }
  Field* fq[] = {&s.q_r, &s.q_psi, &s.q_rho, &s.q_a};
  for (Field* f : fq) DP_HIP(c, f->alloc(g, prec, 2));
  DP_HIP(c, s.ratio.reserve(sizeof(double) * 4 * g.T));
  DP_HIP(c, s.m4.reserve(sizeof(double)));
  DP_HIP(c, s.alpha.reserve(sizeof(double) * g.T));
  DP_HIP(c, s.partials.reserve(sizeof(double) * 2 * kDotBlocks));
  s.h_gcr.resize(gcr_len(nkv));
  DP_HIP(c, s.gcr.reserve(sizeof(double) * s.h_gcr.size()));
  s.h_part.resize(2 * kDotBlocks);
  s.g = g;
  s.nkv = nkv;
  s.prec = prec;
  return DP_OK;
}

// out = D' in on the whole lattice, both parities (full operator, not Schur)
int apply_full(dp_ctx* c, SapState& s, int prec, const Field& in, const Field& out) {
  for (int p = 0; p < 2; ++p) {
    HopArgs a;
    a.g = c->g;
    a.p = p;
    a.dag = 0;
    a.epi = EPI_DIAG;
    a.sign = 1.0;
    a.U_out = c->U[prec][p].p;
    a.U_in = c->U[prec][1 - p].p;
    a.link_prec = prec;
    a.in = in.ref(1 - p);
    a.out = out.ref(p);
    a.xin = in.ref(p);
    a.clov.prec = prec;
    a.clov.data = prec == F64 ? c->C64[p].p : prec == F32 ? c->C32[p].p : c->C16[p].p;
    a.clov.scale = prec == F16 ? c->C16s[p].as<float>() : nullptr;
    a.slots.ratio = s.ratio.as<double>();
    a.slots.m4 = s.m4.as<double>();
    a.red.red = RED_NONE;
    a.nslots = 1;
    a.sratio = space_hop_ratios(c);
    int nparts = 0;
    DP_HIP(c, launch_hop(a, c->stream, &nparts));
  }
  return DP_OK;
}

dim3 site_grid(const Geom& g) { return dim3((g.Vh + kBlock - 1) / kBlock, 2); }

int vec_update(dp_ctx* c, int op, zc a, const Field& x, const Field& y) {
  hipLaunchKernelGGL(vec_update_kernel, site_grid(c->g), dim3(kBlock), 0, c->stream, c->g, op, a.real(), a.imag(),
                     x.ref(), y.ref());
  DP_HIP(c, hipGetLastError());
  return DP_OK;
}

// <x, y> summed on the host in block order
int vec_dot(dp_ctx* c, SapState& s, const Field& x, const Field& y, zc* out) {
  hipLaunchKernelGGL(vec_dot_kernel, dim3(kDotBlocks), dim3(kBlock), 0, c->stream, c->g, x.ref(), y.ref(),
                     s.partials.as<double>());
  DP_HIP(c, hipGetLastError());
  DP_HIP(c, hipMemcpyAsync(s.h_part.data(), s.partials.p, sizeof(double) * 2 * kDotBlocks, hipMemcpyDeviceToHost,
                           c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  double re = 0.0, im = 0.0;
  for (int k = 0; k < kDotBlocks; ++k) {
    re += s.h_part[2 * k];
    im += s.h_part[2 * k + 1];
  }
  *out = zc(re, im);
  return DP_OK;
}

// out = the finished <x, y> on the device (dot_finish_kernel's mode)
int vec_dot_dev(dp_ctx* c, SapState& s, const Field& x, const Field& y, int mode, const double* guard, double* out) {
  hipLaunchKernelGGL(vec_dot_kernel, dim3(kDotBlocks), dim3(kBlock), 0, c->stream, c->g, x.ref(), y.ref(),
                     s.partials.as<double>());
  DP_HIP(c, hipGetLastError());
  hipLaunchKernelGGL(dot_finish_kernel, dim3(1), dim3(64), 0, c->stream, s.partials.as<double>(), mode, guard, out);
  DP_HIP(c, hipGetLastError());
  return DP_OK;
}

// y updated by vec_update_dot_kernel's op, then out = the dot product of its
// dmode (finished in dot_finish_kernel's fmode)
int vec_update_dot_dev(dp_ctx* c, SapState& s, int op, const double* coef, double sgn, const Field& x,
                       const Field& y, int dmode, const Field& z, int fmode, const double* guard, double* out) {
  hipLaunchKernelGGL(vec_update_dot_kernel, dim3(kDotBlocks), dim3(kBlock), 0, c->stream, c->g, op, coef, sgn,
                     x.ref(), y.ref(), dmode, z.ref(), s.partials.as<double>());
  DP_HIP(c, hipGetLastError());
  hipLaunchKernelGGL(dot_finish_kernel, dim3(1), dim3(64), 0, c->stream, s.partials.as<double>(), fmode, guard, out);
  DP_HIP(c, hipGetLastError());
  return DP_OK;
}


template <int PI, int PO>
int convert(dp_ctx* c, const Field& x, const Field& y) {
  hipLaunchKernelGGL((vec_convert_kernel<PI, PO>), site_grid(c->g), dim3(kBlock), 0, c->stream, c->g, x.ref(),
                     y.ref());
  DP_HIP(c, hipGetLastError());
  return DP_OK;
}

template <int P>
int sap_apply(dp_ctx* c, SapState& s, const Blocking& b, int ncy, int nmr) {
  const dim3 mr_grid(b.nhalf);
  bool psi_zero = true;
  for (int cy = 0; cy < ncy; ++cy)
    for (int colour = 0; colour < 2; ++colour) {
      if (!psi_zero) DP_TRY(apply_full(c, s, P, s.q_psi, s.q_a));
      hipLaunchKernelGGL((sap_residual_kernel<P>), site_grid(c->g), dim3(kBlock), 0, c->stream, c->g, b, colour,
                         s.q_r.ref(), s.q_a.ref(), s.q_rho.ref(), psi_zero ? 0 : 1);
      DP_HIP(c, hipGetLastError());
      if (psi_zero) {  // psi = 0 before the first block solve (no site has colour -1)
        hipLaunchKernelGGL((sap_residual_kernel<P>), site_grid(c->g), dim3(kBlock), 0, c->stream, c->g, b, -1,
                           s.q_r.ref(), s.q_a.ref(), s.q_psi.ref(), 0);
        DP_HIP(c, hipGetLastError());
        psi_zero = false;
      }
      for (int k = 0; k < nmr; ++k) {
        DP_TRY(apply_full(c, s, P, s.q_rho, s.q_a));
        hipLaunchKernelGGL((sap_mr_kernel<P>), mr_grid, dim3(kBlock), 0, c->stream, c->g, b, colour, s.q_a.ref(),
                           s.q_rho.ref(), s.q_psi.ref());
        DP_HIP(c, hipGetLastError());
      }
    }
  return DP_OK;
}

// The fused block solves take FP32 block solves on blocks of at most
// kSapBigSites sites (DP_SAP_FUSED=0 keeps the launch-per-step path).
bool sap_fused_enabled(int prec, const Blocking& b) {
  if (prec != F32 || b.vol > kSapBigSites) return false;
  const char* e = std::getenv("DP_SAP_FUSED");
  return !(e && e[0] == '0');
}

// block-layout buffers and the links and clover gathered into them
int sap_fused_setup(dp_ctx* c, SapState& s, const Blocking& b) {
  const long V = 2L * c->g.Vh;
  DP_HIP(c, s.ubl.reserve(sizeof(float2) * 36 * V));
  DP_HIP(c, s.cbl.reserve(sizeof(float4) * 18 * V));
  DP_HIP(c, s.rbl.reserve(sizeof(float4) * 6 * V));
  DP_HIP(c, s.pbl.reserve(sizeof(float4) * 6 * V));
  if (b.vol > kSapThreads) DP_HIP(c, s.abl.reserve(sizeof(float4) * 6 * V));
  hipLaunchKernelGGL(sap_gather_kernel, site_grid(c->g), dim3(kBlock), 0, c->stream, c->g, b,
                     c->U[F32][0].as<float2>(), c->U[F32][1].as<float2>(), c->C32[0].as<float4>(),
                     c->C32[1].as<float4>(), s.ubl.as<float2>(), s.cbl.as<float4>());
  DP_HIP(c, hipGetLastError());
  return DP_OK;
}

// psi = M r with one kernel per colour pass (r, psi in s.rbl, s.pbl)
int sap_apply_fused(dp_ctx* c, SapState& s, const Blocking& b, int ncy, int nmr) {
  SapPass a;
  a.g = c->g;
  a.b = b;
  a.nmr = nmr;
  a.r = s.rbl.as<float4>();
  a.psi = s.pbl.as<float4>();
  a.U = s.ubl.as<float2>();
  a.C = s.cbl.as<float4>();
  a.av = s.abl.as<float4>();
  a.rt = s.ratio.as<double>();
  a.sratio = space_hop_ratios(c);
  a.m4 = (float)(4.0 + c->M);
  for (int cy = 0; cy < ncy; ++cy)
    for (int colour = 0; colour < 2; ++colour) {
      a.colour = colour;
      a.own_zero = cy == 0;
      const bool first = cy == 0 && colour == 0;
      if (b.vol <= kSapThreads) {
        if (first)
          hipLaunchKernelGGL(sap_block_kernel<true>, dim3(b.nhalf), dim3(kSapThreads), 0, c->stream, a);
        else
          hipLaunchKernelGGL(sap_block_kernel<false>, dim3(b.nhalf), dim3(kSapThreads), 0, c->stream, a);
      } else {
        if (first)
          hipLaunchKernelGGL(sap_block_big_kernel<true>, dim3(b.nhalf), dim3(kSapBigThreads), 0, c->stream, a);
        else
          hipLaunchKernelGGL(sap_block_big_kernel<false>, dim3(b.nhalf), dim3(kSapBigThreads), 0, c->stream, a);
      }
      DP_HIP(c, hipGetLastError());
    }
  return DP_OK;
}

// z = M r (r, z FP64)
int precondition(dp_ctx* c, SapState& s, const Blocking& b, int ncy, int nmr, const Field& r, const Field& z) {
  TraceRange tr("sap_precondition");
  if (s.fused) {
    hipLaunchKernelGGL(sap_to_block_kernel, site_grid(c->g), dim3(kBlock), 0, c->stream, c->g, b, r.ref(),
                       s.rbl.as<float4>());
    DP_HIP(c, hipGetLastError());
    DP_TRY(sap_apply_fused(c, s, b, ncy, nmr));
    hipLaunchKernelGGL(sap_from_block_kernel, site_grid(c->g), dim3(kBlock), 0, c->stream, c->g, b,
                       s.pbl.as<float4>(), z.ref());
    DP_HIP(c, hipGetLastError());
  } else if (s.prec == F64) {
    DP_TRY((convert<F64, F64>(c, r, s.q_r)));
    DP_TRY(sap_apply<F64>(c, s, b, ncy, nmr));
    DP_TRY((convert<F64, F64>(c, s.q_psi, z)));
  } else {
    DP_TRY((convert<F64, F32>(c, r, s.q_r)));
    DP_TRY(sap_apply<F32>(c, s, b, ncy, nmr));
    DP_TRY((convert<F32, F64>(c, s.q_psi, z)));
  }
  return DP_OK;
}

}  // namespace

void sap_free(SapState* s) { delete s; }

}  // namespace dp

namespace dp {
namespace {

// Shared set-up of dp_solve_sap and dp_sap_precondition: the blocking, the
// work space, the tables of the one right-hand side (time ratios, 4 + M,
// alpha) and, for fused block solves, the block-layout links and clover.
int sap_prepare(dp_ctx* c, const dp_sap_params* p, int nkv, Blocking* bo) {
  const Geom& g = c->g;
  Blocking& b = *bo;
  b.vol = 1;
  int nblocks = 1;
  for (int mu = 0; mu < 4; ++mu) {
    const int L = mu == 0 ? g.T : mu == 1 ? g.L1 : mu == 2 ? g.L2 : g.L3;
    b.bs[mu] = p->block[mu];
    if (b.bs[mu] < 1 || L % b.bs[mu] || (L / b.bs[mu]) % 2)
      return fail(c, DP_ERR_INVALID_ARG, "each block extent must divide its lattice extent an even number of times");
    b.nb[mu] = L / b.bs[mu];
    b.vol *= b.bs[mu];
    nblocks *= b.nb[mu];
  }
  b.nhalf = nblocks / 2;
  if (p->ncy < 1 || p->nmr < 1) return fail(c, DP_ERR_INVALID_ARG, "bad ncy or nmr");
  if (p->precision != DP_PREC_F64 && p->precision != DP_PREC_F32)
    return fail(c, DP_ERR_INVALID_ARG, "the block solves run in FP64 or FP32");
  DP_HIP(c, hipSetDevice(c->device));
  if (!c->have_U[F64]) return fail(c, DP_ERR_BAD_STATE, "gauge field not set");
  if (!c->sap) {
    c->sap = new (std::nothrow) SapState;
    if (!c->sap) return fail(c, DP_ERR_OOM, "host allocation failed");
  }
  SapState& s = *c->sap;
  DP_TRY(sap_alloc(c, s, nkv, p->precision));
  std::vector<double> rt(4 * g.T);
  ratio_tables(g.T, c->bc_t, c->alpha.data(), rt.data());
  DP_TRY(h2d(c, s.ratio.p, rt.data(), sizeof(double) * 4 * g.T));
  const double m4 = 4.0 + c->M;
  DP_TRY(h2d(c, s.m4.p, &m4, sizeof(double)));
  DP_TRY(h2d(c, s.alpha.p, c->alpha.data(), sizeof(double) * g.T));
  s.fused = sap_fused_enabled(p->precision, b);
  if (s.fused) DP_TRY(sap_fused_setup(c, s, b));
  return DP_OK;
}

}  // namespace
}  // namespace dp

extern "C" int dp_sap_precondition(dp_ctx* c, const double* r, const dp_sap_params* p, double* psi) {
  if (!c || !r || !p || !psi) return DP_ERR_INVALID_ARG;
  const Geom& g = c->g;
  Blocking b;
  DP_TRY(sap_prepare(c, p, 1, &b));
  SapState& s = *c->sap;
  const size_t bytes = (size_t)2 * g.Vh * 12 * sizeof(double2);
  DP_HIP(c, c->scratch_aos.reserve(bytes));
  DP_HIP(c, hipMemcpyAsync(c->scratch_aos.p, r, bytes, hipMemcpyHostToDevice, c->stream));
  for (int par = 0; par < 2; ++par)
    DP_HIP(c, launch_spinor_import(g, c->scratch_aos.as<double2>(), 1, 0, par, s.r.ref(par), nullptr, nullptr,
                                   c->stream));
  DP_TRY(precondition(c, s, b, p->ncy, p->nmr, s.r, s.z[0]));
  DP_HIP(c, launch_spinor_export(g, s.z[0].ref(0), s.z[0].ref(1), 1, nullptr, nullptr, c->scratch_aos.as<double2>(),
                                 0, c->stream));
  DP_HIP(c, hipMemcpyAsync(psi, c->scratch_aos.p, bytes, hipMemcpyDeviceToHost, c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  return DP_OK;
}

namespace dp {
namespace {

// The SAP+GCR solve (after sap_prepare) from a source in device memory (host
// layout); the solution goes to S_dev (device, host layout) if not null, then
// to S_host; t0 is the start of the timed solve.
int sap_solve(dp_ctx* c, const Blocking& b, const double2* eta_dev, const dp_sap_params* p, double2* S_dev,
              double* S_host, double* cpp, dp_info* info, double t0) {
  const Geom& g = c->g;
  SapState& s = *c->sap;
  const size_t bytes = (size_t)2 * g.Vh * 12 * sizeof(double2);
  // eta' = beta eta
  for (int par = 0; par < 2; ++par)
    DP_HIP(c, launch_spinor_import(g, eta_dev, 1, 0, par, s.eta.ref(par), s.alpha.as<double>(), space_profile(c),
                                   c->stream));
  zc e2;
  DP_TRY(vec_dot(c, s, s.eta, s.eta, &e2));
  const double target = p->r * std::sqrt(e2.real());
  // x = 0, r = eta'
  DP_TRY(vec_update(c, 2, zc(0.0, 0.0), s.x, s.x));
  DP_TRY(vec_update(c, 3, zc(0.0, 0.0), s.eta, s.r));
  int iters = 0, status = DP_ERR_NOT_CONVERGED, outer = 0;
  double rn = std::sqrt(e2.real());
  if (!std::isfinite(rn)) status = DP_ERR_NONFINITE;
  else if (rn <= target) status = DP_OK;
  const int nkv = p->nkv;
  std::vector<zc> cc((size_t)nkv * nkv), gam(nkv), al(nkv);
  std::vector<double> bn(nkv);
  while (status == DP_ERR_NOT_CONVERGED && iters < p->max_iter) {
    int k = 0;
    bool breakdown = false;
    for (; k < nkv && iters < p->max_iter; ++k) {
      DP_TRY(precondition(c, s, b, p->ncy, p->nmr, s.r, s.z[k]));
      DP_TRY(apply_full(c, s, F64, s.z[k], s.w[k]));
      ++iters;
      // modified Gram-Schmidt against the earlier w_j, normalisation,
      // gamma_k = <w_k, r> and r -= gamma_k w_k, with every coefficient
      // formed and used on the device (each update shares its pass with the
      // next dot product); one copy to the host per iteration
      double* gd = s.gcr.as<double>();
      double* bk = gd + gcr_bn(nkv, k);
      double* gk = gd + gcr_gam(nkv, k);
      if (k == 0) {
        DP_TRY(vec_dot_dev(c, s, s.w[k], s.w[k], 1, nullptr, bk));
      } else {
        DP_TRY(vec_dot_dev(c, s, s.w[0], s.w[k], 0, nullptr, gd + gcr_cc(nkv, 0, k)));
        for (int j = 1; j < k; ++j)  // w_k -= c_{j-1,k} w_{j-1}, then c_jk = <w_j, w_k>
          DP_TRY(vec_update_dot_dev(c, s, 0, gd + gcr_cc(nkv, j - 1, k), -1.0, s.w[j - 1], s.w[k], 0, s.w[j], 0,
                                    nullptr, gd + gcr_cc(nkv, j, k)));
        DP_TRY(vec_update_dot_dev(c, s, 0, gd + gcr_cc(nkv, k - 1, k), -1.0, s.w[k - 1], s.w[k], 2, s.w[k], 1,
                                  nullptr, bk));
      }
      // w_k /= b_k, then gamma_k = <w_k, r>; r -= gamma_k w_k, then |r|^2
      DP_TRY(vec_update_dot_dev(c, s, 1, bk, 1.0, s.w[k], s.w[k], 1, s.r, 2, bk, gk));
      DP_TRY(vec_update_dot_dev(c, s, 0, gk, -1.0, s.w[k], s.r, 2, s.r, 0, nullptr, gd + gcr_rn(nkv)));
      DP_HIP(c, hipMemcpyAsync(s.h_gcr.data(), gd, sizeof(double) * gcr_len(nkv), hipMemcpyDeviceToHost, c->stream));
      DP_HIP(c, hipStreamSynchronize(c->stream));
      const double* hg = s.h_gcr.data();
      for (int j = 0; j < k; ++j)
        cc[(size_t)j * nkv + k] = zc(hg[gcr_cc(nkv, j, k)], hg[gcr_cc(nkv, j, k) + 1]);
      bn[k] = hg[gcr_bn(nkv, k)];
      if (!(bn[k] > 0) || !std::isfinite(bn[k])) {
        breakdown = true;
        break;
      }
      gam[k] = zc(hg[gcr_gam(nkv, k)], hg[gcr_gam(nkv, k) + 1]);
      rn = std::sqrt(hg[gcr_rn(nkv)]);
      if (rn <= target) {
        ++k;
        break;
      }
    }
    if (breakdown) {
      status = std::isfinite(bn[k]) ? DP_ERR_BREAKDOWN : DP_ERR_NONFINITE;
      break;
    }
    for (int j = k - 1; j >= 0; --j) {
      zc v = gam[j];
      for (int l = j + 1; l < k; ++l) v -= cc[(size_t)j * nkv + l] * al[l];
      al[j] = v / bn[j];
    }
    for (int j = 0; j < k; ++j) DP_TRY(vec_update(c, 0, al[j], s.z[j], s.x));
    // true residual r = eta' - D' x
    DP_TRY(apply_full(c, s, F64, s.x, s.r));
    DP_TRY(vec_update(c, 1, zc(0.0, 0.0), s.eta, s.r));
    zc r2;
    DP_TRY(vec_dot(c, s, s.r, s.r, &r2));
    rn = std::sqrt(r2.real());
    ++outer;
    if (!std::isfinite(rn)) status = DP_ERR_NONFINITE;
    else if (rn <= target) status = DP_OK;
  }
  // S = x / beta, C_PP
  if (S_dev) {
    DP_HIP(c, launch_spinor_export(g, s.x.ref(0), s.x.ref(1), 1, s.alpha.as<double>(), space_profile(c), S_dev, 0,
                                   c->stream));
    if (S_host) DP_HIP(c, hipMemcpyAsync(S_host, S_dev, bytes, hipMemcpyDeviceToHost, c->stream));
  }
  if (cpp) {
    DP_HIP(c, s.cpp.reserve(sizeof(double) * g.T));
    DP_HIP(c, launch_cpp(g, s.x.ref(0), s.x.ref(1), 1, s.alpha.as<double>(), space_profile(c), nullptr,
                         s.cpp.as<double>(), c->stream));
    DP_HIP(c, hipMemcpyAsync(cpp, s.cpp.p, sizeof(double) * g.T, hipMemcpyDeviceToHost, c->stream));
  }
  DP_HIP(c, hipStreamSynchronize(c->stream));
  DP_TRY(timing_harvest(c));
  if (info) {
    dp_info& o = *info;
    o.status = status;
    o.iters = iters;
    o.outer = outer;
    o.hop_calls = 0;
    o.restarts = 0;
    o.fallback = 0;
    o.true_res = e2.real() > 0 ? rn / std::sqrt(e2.real()) : 0.0;
    o.seconds = now_s() - t0;
  }
  if (status == DP_ERR_NOT_CONVERGED) return fail(c, status, "SAP+GCR did not converge within max_iter");
  if (status == DP_ERR_BREAKDOWN) return fail(c, status, "GCR broke down (zero preconditioned direction)");
  if (status == DP_ERR_NONFINITE) return fail(c, status, "a residual became NaN or Inf");
  return DP_OK;
}

int sap_check(dp_ctx* c, const dp_sap_params* p) {
  if (!(p->r > 0) || !std::isfinite(p->r) || p->nkv < 1 || p->nkv > 64 || p->max_iter < 1)
    return fail(c, DP_ERR_INVALID_ARG, "bad residue, ncy, nmr, nkv (1..64) or max_iter");
  return DP_OK;
}

}  // namespace
}  // namespace dp

extern "C" int dp_solve_sap(dp_ctx* c, const double* eta, const dp_sap_params* p, double* S, double* cpp,
                            dp_info* info) {
  if (!c || !eta || !p) return DP_ERR_INVALID_ARG;
  TraceRange tr("dp_solve_sap");
  DP_TRY(sap_check(c, p));
  Blocking b;
  DP_TRY(sap_prepare(c, p, p->nkv, &b));
  const double t0 = now_s();
  // the source through the context's staging buffer, which takes the
  // solution afterwards
  const size_t bytes = (size_t)2 * c->g.Vh * 12 * sizeof(double2);
  DP_HIP(c, c->scratch_aos.reserve(bytes));
  DP_HIP(c, hipMemcpyAsync(c->scratch_aos.p, eta, bytes, hipMemcpyHostToDevice, c->stream));
  double2* st = c->scratch_aos.as<double2>();
  return sap_solve(c, b, st, p, S ? st : nullptr, S, cpp, info, t0);
}

extern "C" int dp_solve_sap_dev(dp_ctx* c, const void* eta_dev, const dp_sap_params* p, void* S_dev, double* cpp,
                                dp_info* info, void* hip_stream) {
  if (!c || !eta_dev || !p) return DP_ERR_INVALID_ARG;
  TraceRange tr("dp_solve_sap_dev");
  DP_TRY(sap_check(c, p));
  const size_t bytes = (size_t)2 * c->g.Vh * 12 * sizeof(double2);
  const char* e0 = static_cast<const char*>(eta_dev);
  const char* s0 = static_cast<const char*>(S_dev);
  if (S_dev && e0 < s0 + bytes && s0 < e0 + bytes) return fail(c, DP_ERR_INVALID_ARG, "eta and S overlap");
  DP_HIP(c, hipSetDevice(c->device));
  if (hip_stream) DP_HIP(c, hipStreamSynchronize((hipStream_t)hip_stream));
  Blocking b;
  DP_TRY(sap_prepare(c, p, p->nkv, &b));
  const double t0 = now_s();
  return sap_solve(c, b, static_cast<const double2*>(eta_dev), p, static_cast<double2*>(S_dev), nullptr, cpp, info,
                   t0);
}
