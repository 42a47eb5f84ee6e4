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

// op 0: y += a x (a complex);  op 1: y = s y (s = a.x real);  op 2: y = x - y
__global__ void __launch_bounds__(kBlock) vec_update_kernel(Geom g, int op, double ar, double ai, SpinorRef x,
                                                            SpinorRef y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (i >= g.Vh) return;
  cx<double> vx[12], vy[12];
  SpinorIO<F64>::load(y, p, i, g.Vp, vy);
  if (op != 1) SpinorIO<F64>::load(x, p, i, g.Vp, vx);
  const cx<double> a{ar, ai};
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    if (op == 0) vy[c] = vy[c] + cmul(a, vx[c]);
    else if (op == 1) vy[c] = ar * vy[c];
    else vy[c] = vx[c] - vy[c];
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

constexpr int kDotBlocks = 1024;

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
  std::vector<double> h_part;
};

namespace {

using zc = std::complex<double>;

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

// z = M r (r, z FP64)
int precondition(dp_ctx* c, SapState& s, const Blocking& b, int ncy, int nmr, const Field& r, const Field& z) {
  if (s.prec == F64) {
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

extern "C" int dp_solve_sap(dp_ctx* c, const double* eta, const dp_sap_params* p, double* S, double* cpp,
                            dp_info* info) {
  if (!c || !eta || !p) return DP_ERR_INVALID_ARG;
  const Geom& g = c->g;
  Blocking b;
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
  if (!(p->r > 0) || !std::isfinite(p->r) || p->ncy < 1 || p->nmr < 1 || p->nkv < 1 || p->nkv > 64 ||
      p->max_iter < 1)
    return fail(c, DP_ERR_INVALID_ARG, "bad residue, ncy, nmr, nkv (1..64) or max_iter");
  if (p->precision != DP_PREC_F64 && p->precision != DP_PREC_F32)
    return fail(c, DP_ERR_INVALID_ARG, "the block solves run in FP64 or FP32");
  DP_HIP(c, hipSetDevice(c->device));
  if (!c->have_U[F64]) return fail(c, DP_ERR_BAD_STATE, "gauge field not set");
  if (!c->sap) {
    c->sap = new (std::nothrow) SapState;
    if (!c->sap) return fail(c, DP_ERR_OOM, "host allocation failed");
  }
  SapState& s = *c->sap;
  DP_TRY(sap_alloc(c, s, p->nkv, p->precision));
  const double t0 = now_s();
  // tables of the one right-hand side: time ratios, 4 + M, alpha
  {
    std::vector<double> rt(4 * g.T);
    ratio_tables(g.T, c->bc_t, c->alpha.data(), rt.data());
    DP_TRY(h2d(c, s.ratio.p, rt.data(), sizeof(double) * 4 * g.T));
    const double m4 = 4.0 + c->M;
    DP_TRY(h2d(c, s.m4.p, &m4, sizeof(double)));
    DP_TRY(h2d(c, s.alpha.p, c->alpha.data(), sizeof(double) * g.T));
  }
  // eta' = beta eta
  const size_t bytes = (size_t)2 * g.Vh * 12 * sizeof(double2);
  DP_HIP(c, c->scratch_aos.reserve(bytes));
  DP_HIP(c, hipMemcpyAsync(c->scratch_aos.p, eta, bytes, hipMemcpyHostToDevice, c->stream));
  for (int par = 0; par < 2; ++par)
    DP_HIP(c, launch_spinor_import(g, c->scratch_aos.as<double2>(), 1, 0, par, s.eta.ref(par), s.alpha.as<double>(),
                                   space_profile(c), c->stream));
  zc e2;
  DP_TRY(vec_dot(c, s, s.eta, s.eta, &e2));
  const double target = p->r * std::sqrt(e2.real());
  // x = 0, r = eta'
  DP_TRY(vec_update(c, 1, zc(0.0, 0.0), s.x, s.x));
  DP_TRY(vec_update(c, 1, zc(0.0, 0.0), s.r, s.r));
  DP_TRY(vec_update(c, 0, zc(1.0, 0.0), s.eta, s.r));
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
      for (int j = 0; j < k; ++j) {
        zc cj;
        DP_TRY(vec_dot(c, s, s.w[j], s.w[k], &cj));
        cc[(size_t)j * nkv + k] = cj;
        DP_TRY(vec_update(c, 0, -cj, s.w[j], s.w[k]));
      }
      zc b2;
      DP_TRY(vec_dot(c, s, s.w[k], s.w[k], &b2));
      bn[k] = std::sqrt(b2.real());
      if (!(bn[k] > 0) || !std::isfinite(bn[k])) {
        breakdown = true;
        break;
      }
      DP_TRY(vec_update(c, 1, zc(1.0 / bn[k], 0.0), s.w[k], s.w[k]));
      DP_TRY(vec_dot(c, s, s.w[k], s.r, &gam[k]));
      DP_TRY(vec_update(c, 0, -gam[k], s.w[k], s.r));
      zc r2;
      DP_TRY(vec_dot(c, s, s.r, s.r, &r2));
      rn = std::sqrt(r2.real());
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
    DP_TRY(vec_update(c, 2, zc(0.0, 0.0), s.eta, s.r));
    zc r2;
    DP_TRY(vec_dot(c, s, s.r, s.r, &r2));
    rn = std::sqrt(r2.real());
    ++outer;
    if (!std::isfinite(rn)) status = DP_ERR_NONFINITE;
    else if (rn <= target) status = DP_OK;
  }
  // S = x / beta, C_PP
  DP_HIP(c, launch_spinor_export(g, s.x.ref(0), s.x.ref(1), 1, s.alpha.as<double>(), space_profile(c),
                                 c->scratch_aos.as<double2>(), 0, c->stream));
  if (S) DP_HIP(c, hipMemcpyAsync(S, c->scratch_aos.p, bytes, hipMemcpyDeviceToHost, c->stream));
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
