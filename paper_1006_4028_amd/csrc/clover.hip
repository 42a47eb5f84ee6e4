// Clover term of the O(a)-improved Wilson operator (the operator the paper
// works with, heavy-quark section):
//   C(x) = c_sw (i/4) sum_{mu,nu} sigma_mu_nu Fhat_mu_nu(x),
//   Fhat = (Q_mu_nu - Q_nu_mu) / 8, Q the four same-orientation plaquette
//   leaves at x in the (mu,nu) plane.
// In the chiral basis sigma_0k = diag(sigma_k, -sigma_k) and
// sigma_ij = -eps_ijk diag(sigma_k, sigma_k), so C splits into two Hermitian
// 6x6 blocks (chirality s = +1 upper, s = -1 lower):
//   block_s = c_sw (i/2) sum_k sigma_k (x) G_k,
//   G_1 = s F01 - F23,  G_2 = s F02 + F13,  G_3 = s F03 - F12.
// Also: packing of a caller-supplied dense clover field, the per-mass inverse
// (C + 4 + M)^-1 of every block, and conversion to the inner precisions.
#include "dp_device.h"

namespace dp {

namespace {

using z = cx<double>;

struct M3 {
  z m[9];
};

__device__ __forceinline__ M3 load_link64(const Geom& g, const double2* const* U, int x0, int x1, int x2, int x3,
                                          int mu) {
  const int p = (x0 + x1 + x2 + x3) & 1;
  const int i = eo_index(g, x0, x1, x2, x3);
  const double2* b = U[p] + (long)mu * 9 * g.Vp;
  M3 r;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double2 v = b[(long)k * g.Vp + i];
    r.m[k] = z{v.x, v.y};
  }
  return r;
}

__device__ __forceinline__ M3 mul(const M3& A, const M3& B) {
  M3 C;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      z t = cmul(A.m[3 * i], B.m[j]);
      cfma(t, A.m[3 * i + 1], B.m[3 + j]);
      cfma(t, A.m[3 * i + 2], B.m[6 + j]);
      C.m[3 * i + j] = t;
    }
  return C;
}

__device__ __forceinline__ M3 dag(const M3& A) {
  M3 B;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) B.m[3 * i + j] = z{A.m[3 * j + i].x, -A.m[3 * j + i].y};
  return B;
}

struct Site {
  int x[4];
};

__device__ __forceinline__ Site shift(const Geom& g, Site s, int mu, int d) {
  const int L = mu == 0 ? g.T : mu == 1 ? g.L1 : mu == 2 ? g.L2 : g.L3;
  s.x[mu] = (s.x[mu] + d + L) % L;
  return s;
}

__device__ __forceinline__ M3 U_at(const Geom& g, const double2* const* U, const Site& s, int mu) {
  return load_link64(g, U, s.x[0], s.x[1], s.x[2], s.x[3], mu);
}

// Fhat_mu_nu(x) = (Q - Q^+)/8 with Q the sum of the four leaves (mu < nu)
__device__ M3 field_strength(const Geom& g, const double2* const* U, const Site& x, int mu, int nu) {
  const Site xpm = shift(g, x, mu, +1), xmm = shift(g, x, mu, -1);
  const Site xpn = shift(g, x, nu, +1), xmn = shift(g, x, nu, -1);
  const Site xmm_pn = shift(g, xmm, nu, +1), xmm_mn = shift(g, xmm, nu, -1);
  const Site xpm_mn = shift(g, xpm, nu, -1);
  // leaf in the +mu,+nu quadrant
  M3 Q = mul(mul(U_at(g, U, x, mu), U_at(g, U, xpm, nu)), mul(dag(U_at(g, U, xpn, mu)), dag(U_at(g, U, x, nu))));
  // -mu,+nu quadrant
  M3 L2 = mul(mul(U_at(g, U, x, nu), dag(U_at(g, U, xmm_pn, mu))), mul(dag(U_at(g, U, xmm, nu)), U_at(g, U, xmm, mu)));
  // -mu,-nu quadrant
  M3 L3 = mul(mul(dag(U_at(g, U, xmm, mu)), dag(U_at(g, U, xmm_mn, nu))), mul(U_at(g, U, xmm_mn, mu), U_at(g, U, xmn, nu)));
  // +mu,-nu quadrant
  M3 L4 = mul(mul(dag(U_at(g, U, xmn, nu)), U_at(g, U, xmn, mu)), mul(U_at(g, U, xpm_mn, nu), dag(U_at(g, U, x, mu))));
  M3 F;
#pragma unroll
  for (int k = 0; k < 9; ++k) Q.m[k] = Q.m[k] + L2.m[k] + L3.m[k] + L4.m[k];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const z a = Q.m[3 * i + j], b = Q.m[3 * j + i];  // Q_ij and Q_ji -> (Q - Q^+)_ij
      F.m[3 * i + j] = z{(a.x - b.x) * 0.125, (a.y + b.y) * 0.125};
    }
  return F;
}

__device__ __forceinline__ void store_block(double2* dst, int Vh, int i, int h, const z (&A)[6][6]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) dst[(long)(h * 18 + k) * Vh + i] = make_double2(A[2 * k][2 * k].x, A[2 * k + 1][2 * k + 1].x);
  int n = 0;
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r + 1; c < 6; ++c, ++n) dst[(long)(h * 18 + 3 + n) * Vh + i] = make_double2(A[r][c].x, A[r][c].y);
}

__device__ __forceinline__ void load_block(const double2* src, int Vh, int i, int h, z (&A)[6][6]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double2 v = src[(long)(h * 18 + k) * Vh + i];
    A[2 * k][2 * k] = z{v.x, 0.0};
    A[2 * k + 1][2 * k + 1] = z{v.y, 0.0};
  }
  int n = 0;
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r + 1; c < 6; ++c, ++n) {
      const double2 v = src[(long)(h * 18 + 3 + n) * Vh + i];
      A[r][c] = z{v.x, v.y};
      A[c][r] = z{v.x, -v.y};
    }
}

__global__ void __launch_bounds__(128) clover_build_kernel(Geom g, const double2* Ue, const double2* Uo, double csw,
                                                           double2* Ce, double2* Co) {
  const long V = 2L * g.Vh;
  const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= V) return;
  const double2* U[2] = {Ue, Uo};
  Site x;
  {
    long t = s;
    x.x[3] = (int)(t % g.L3); t /= g.L3;
    x.x[2] = (int)(t % g.L2); t /= g.L2;
    x.x[1] = (int)(t % g.L1);
    x.x[0] = (int)(t / g.L1);
  }
  const int p = (x.x[0] + x.x[1] + x.x[2] + x.x[3]) & 1;
  const int i = (int)(s >> 1);
  const M3 F01 = field_strength(g, U, x, 0, 1), F02 = field_strength(g, U, x, 0, 2), F03 = field_strength(g, U, x, 0, 3);
  const M3 F12 = field_strength(g, U, x, 1, 2), F13 = field_strength(g, U, x, 1, 3), F23 = field_strength(g, U, x, 2, 3);
  double2* dst = p ? Co : Ce;
  for (int h = 0; h < 2; ++h) {
    const double sg = h == 0 ? 1.0 : -1.0;
    z A[6][6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int k = 3 * a + b;
        const z G1 = sg * F01.m[k] - F23.m[k];
        const z G2 = sg * F02.m[k] + F13.m[k];
        const z G3 = sg * F03.m[k] - F12.m[k];
        // (i/2) c_sw times sigma_1 G1 + sigma_2 G2 + sigma_3 G3
        const double f = 0.5 * csw;
        A[a][b] = f * ti(G3);
        A[3 + a][3 + b] = -f * ti(G3);
        A[a][3 + b] = f * ti(G1 - ti(G2));
        A[3 + a][b] = f * ti(G1 + ti(G2));
      }
    store_block(dst, g.Vp, i, h, A);
  }
}

// dense [site][12][12] -> packed blocks, flagging structure violations
__global__ void clover_pack_kernel(Geom g, const double2* __restrict__ C, double2* Ce, double2* Co, int* bad) {
  const long V = 2L * g.Vh;
  const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= V) return;
  long t = s;
  const int x3 = (int)(t % g.L3); t /= g.L3;
  const int x2 = (int)(t % g.L2); t /= g.L2;
  const int x1 = (int)(t % g.L1);
  const int x0 = (int)(t / g.L1);
  const int p = (x0 + x1 + x2 + x3) & 1;
  const double2* c = C + s * 144;
  double mx = 0.0;
  for (int k = 0; k < 144; ++k) mx = fmax(mx, fmax(fabs(c[k].x), fabs(c[k].y)));
  const double tol = 1e-12 * (mx > 0 ? mx : 1.0);
  int flag = 0;
  for (int r = 0; r < 12; ++r)
    for (int q = 0; q < 12; ++q) {
      const double2 a = c[r * 12 + q], b = c[q * 12 + r];
      if ((r < 6) != (q < 6) && (fabs(a.x) > tol || fabs(a.y) > tol)) flag = 1;
      if (fabs(a.x - b.x) > tol || fabs(a.y + b.y) > tol) flag = 1;
    }
  if (flag) atomicOr(bad, 1);
  for (int h = 0; h < 2; ++h) {
    z A[6][6];
    for (int r = 0; r < 6; ++r)
      for (int q = 0; q < 6; ++q) {
        const double2 v = c[(6 * h + r) * 12 + 6 * h + q];
        A[r][q] = z{v.x, v.y};
      }
    store_block(p ? Co : Ce, g.Vp, (int)(s >> 1), h, A);
  }
}

// (B + m4)^-1 by Gauss-Jordan elimination with partial pivoting, FP64.
__global__ void __launch_bounds__(128) clover_invert_kernel(Geom g, const double2* __restrict__ C, double m4,
                                                            double2* Ainv, int* bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int h = blockIdx.y;
  if (i >= g.Vh) return;
  z A[6][6], X[6][6];
  load_block(C, g.Vp, i, h, A);
  for (int r = 0; r < 6; ++r) {
    A[r][r].x += m4;
    for (int c = 0; c < 6; ++c) X[r][c] = z{r == c ? 1.0 : 0.0, 0.0};
  }
  int singular = 0;
  for (int k = 0; k < 6; ++k) {
    int piv = k;
    double best = A[k][k].x * A[k][k].x + A[k][k].y * A[k][k].y;
    for (int r = k + 1; r < 6; ++r) {
      const double m = A[r][k].x * A[r][k].x + A[r][k].y * A[r][k].y;
      if (m > best) { best = m; piv = r; }
    }
    if (!(best > 0.0)) { singular = 1; break; }
    if (piv != k)
      for (int c = 0; c < 6; ++c) {
        z t = A[k][c]; A[k][c] = A[piv][c]; A[piv][c] = t;
        t = X[k][c]; X[k][c] = X[piv][c]; X[piv][c] = t;
      }
    const z d = A[k][k];
    const double dn = d.x * d.x + d.y * d.y;
    const z inv = z{d.x / dn, -d.y / dn};
    for (int c = 0; c < 6; ++c) {
      A[k][c] = cmul(A[k][c], inv);
      X[k][c] = cmul(X[k][c], inv);
    }
    for (int r = 0; r < 6; ++r) {
      if (r == k) continue;
      const z f = A[r][k];
      for (int c = 0; c < 6; ++c) {
        A[r][c] = A[r][c] - cmul(f, A[k][c]);
        X[r][c] = X[r][c] - cmul(f, X[k][c]);
      }
    }
  }
  if (singular) atomicOr(bad, 1);
  // the inverse of a Hermitian matrix is Hermitian: keep the averaged upper part
  for (int r = 0; r < 6; ++r) {
    X[r][r] = z{X[r][r].x, 0.0};
    for (int c = r + 1; c < 6; ++c) X[r][c] = z{0.5 * (X[r][c].x + X[c][r].x), 0.5 * (X[r][c].y - X[c][r].y)};
  }
  store_block(Ainv, g.Vp, i, h, X);
}

template <int P>
__global__ void clover_convert_kernel(Geom g, const double2* __restrict__ C, void* out, float* scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.Vh) return;
  double r[72];
  for (int k = 0; k < 36; ++k) {
    const double2 v = C[(long)k * g.Vp + i];
    r[2 * k] = v.x;
    r[2 * k + 1] = v.y;
  }
  if constexpr (P == F32) {
    float4* o = static_cast<float4*>(out);
    for (int k = 0; k < 18; ++k)
      o[(long)k * g.Vp + i] = make_float4((float)r[4 * k], (float)r[4 * k + 1], (float)r[4 * k + 2], (float)r[4 * k + 3]);
  } else {
    double m = 0.0;
    for (int k = 0; k < 72; ++k) m = fmax(m, fabs(r[k]));
    const double inv = m > 0 ? 1.0 / m : 0.0;
    scale[i] = (float)m;
    uint4* o = static_cast<uint4*>(out);
    for (int k = 0; k < 9; ++k) {
      uint4 v;
      v.x = f2h((float)(r[8 * k + 0] * inv), (float)(r[8 * k + 1] * inv));
      v.y = f2h((float)(r[8 * k + 2] * inv), (float)(r[8 * k + 3] * inv));
      v.z = f2h((float)(r[8 * k + 4] * inv), (float)(r[8 * k + 5] * inv));
      v.w = f2h((float)(r[8 * k + 6] * inv), (float)(r[8 * k + 7] * inv));
      o[(long)k * g.Vp + i] = v;
    }
  }
}

// out = A^-1 in with the slot's A^-1 field, FP64 parity fields.
__global__ void clover_apply_kernel(Geom g, SlotTable slots, SpinorRef in, SpinorRef out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int slot = blockIdx.y;
  if (i >= g.Vh || (slots.mask && !slots.mask[slot])) return;
  z a[12], b[12];
  SpinorIO<F64>::load(in, slot, i, g.Vp, a);
  HermBlock<double> B[2];
  CloverIO<F64>::load(slots.ainv[slot], nullptr, i, g.Vp, B);
  herm_apply(B[0], 0.0, &a[0], &b[0]);
  herm_apply(B[1], 0.0, &a[6], &b[6]);
  SpinorIO<F64>::store(out, slot, i, g.Vp, b);
}

// The interior of a Schroedinger-functional lattice from the clover term
// built on the lattice padded by one timeslice at each end (the boundaries,
// which carry the boundary links): interior site (x0, xs) is padded site
// (x0 + 1, xs), of the other parity and at index i + Vsh there.  ctm1 =
// ct_tilde - 1 is added to the diagonal of both blocks on the first and last
// interior timeslices (the fermion boundary counterterm).
__global__ void clover_sf_interior_kernel(Geom g, Geom gp, const double2* __restrict__ Cpe,
                                          const double2* __restrict__ Cpo, double ctm1, double2* Ce, double2* Co) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (i >= g.Vh) return;
  const double2* src = p ? Cpe : Cpo;  // the padded lattice's parity is the other one
  double2* dst = p ? Co : Ce;
  const int x0 = i / g.Vsh;
  const bool edge = x0 == 0 || x0 == g.T - 1;
  for (int k = 0; k < 36; ++k) {
    double2 v = src[(long)k * gp.Vp + i + g.Vsh];
    if (edge && (k % 18) < 3) {
      v.x += ctm1;
      v.y += ctm1;
    }
    dst[(long)k * g.Vp + i] = v;
  }
}

}  // namespace

hipError_t launch_clover_sf_interior(const Geom& g, const Geom& gp, const double2* Cp_eo[2], double ctm1,
                                     double2* C_eo[2], hipStream_t st) {
  if (gp.T != g.T + 2 || gp.Vsh != g.Vsh) return hipErrorInvalidValue;
  hipLaunchKernelGGL(clover_sf_interior_kernel, dim3((g.Vh + kBlock - 1) / kBlock, 2), dim3(kBlock), 0, st, g, gp,
                     Cp_eo[0], Cp_eo[1], ctm1, C_eo[0], C_eo[1]);
  return hipGetLastError();
}

hipError_t launch_clover_apply(const Geom& g, const SlotTable& slots, SpinorRef in, SpinorRef out, int nslots,
                               hipStream_t st) {
  if (in.prec != F64 || out.prec != F64 || nslots <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(clover_apply_kernel, dim3((g.Vh + kBlock - 1) / kBlock, nslots), dim3(kBlock), 0, st, g, slots,
                     in, out);
  return hipGetLastError();
}

hipError_t launch_clover_build(const Geom& g, const double2* U64_eo[2], double csw, double2* C_eo[2], hipStream_t st) {
  const long V = 2L * g.Vh;
  hipLaunchKernelGGL(clover_build_kernel, dim3((unsigned)((V + 127) / 128)), dim3(128), 0, st, g, U64_eo[0], U64_eo[1],
                     csw, C_eo[0], C_eo[1]);
  return hipGetLastError();
}

hipError_t launch_clover_pack(const Geom& g, const double2* C_aos, double2* C_eo[2], int* bad, hipStream_t st) {
  const long V = 2L * g.Vh;
  hipLaunchKernelGGL(clover_pack_kernel, dim3((unsigned)((V + 127) / 128)), dim3(128), 0, st, g, C_aos, C_eo[0],
                     C_eo[1], bad);
  return hipGetLastError();
}

hipError_t launch_clover_invert(const Geom& g, const double2* C64, double m4, double2* Ainv64, int* bad,
                                hipStream_t st) {
  hipLaunchKernelGGL(clover_invert_kernel, dim3((g.Vh + 127) / 128, 2), dim3(128), 0, st, g, C64, m4, Ainv64, bad);
  return hipGetLastError();
}

hipError_t launch_clover_convert(const Geom& g, const double2* C64, void* out, float* scale, int prec,
                                 hipStream_t st) {
  const dim3 grid((g.Vh + kBlock - 1) / kBlock);
  switch (prec) {
    case F32: hipLaunchKernelGGL(clover_convert_kernel<F32>, grid, dim3(kBlock), 0, st, g, C64, out, scale); break;
    case F16: hipLaunchKernelGGL(clover_convert_kernel<F16>, grid, dim3(kBlock), 0, st, g, C64, out, scale); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dp
