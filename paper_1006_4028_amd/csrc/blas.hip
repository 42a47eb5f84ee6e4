// Fused vector kernels of the Krylov solvers (BiCGStab of van der Vorst 1992
// and CG on the normal equations) over the even sites of every active slot,
// with their global reductions fused in (block partials, then a finalise
// kernel on the same stream; see block_reduce_store).  The
// arithmetic is FP64 whatever the storage precision; scalars come from the
// slot's device-resident SlotScalars.
#include "dp_device.h"

namespace dp {

namespace {

using z = cx<double>;

// Every vector of a vector kernel is touched once: streamed past L2
// (measured on MI355X at 24^3x48 with 12 slots: 1% per solve, the hop
// kernels that follow keep more of their neighbours cached).
template <int P>
__device__ __forceinline__ void ld(const SpinorRef& f, int slot, int i, int Vh, z (&s)[12]) {
  SpinorIO<P>::template load<true>(f, slot, i, Vh, s);
}
template <int P>
__device__ __forceinline__ void st(const SpinorRef& f, int slot, int i, int Vh, const z (&s)[12]) {
  SpinorIO<P>::template store<true>(f, slot, i, Vh, s);
}

// Integer hash of Wellons' "lowbias32" (an xor-shift-multiply finaliser).
__device__ __forceinline__ unsigned hash32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ double norm2(const z (&a)[12]) {
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 12; ++c) s += a[c].x * a[c].x + a[c].y * a[c].y;
  return s;
}

template <int P, int OP>
__global__ void __launch_bounds__(kBlock) blas_kernel(BlasArgs a) {
  constexpr int PX = P == F16 ? F32 : P;
  const Geom& g = a.g;
  const int slot = blockIdx.y;
  if (a.mask && !a.mask[slot]) return;  // uniform over the slot's blocks
  const int i = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const int Vh = g.Vh, Vp = g.Vp;
  double red[kRedMax] = {};
  int nv = 0;
  if constexpr (OP == OP_CG_XR || OP == OP_SUB64 || OP == OP_NORM || OP == OP_BICG_XRP) nv = 1;
  if constexpr (OP == OP_BICG_XR) nv = 3;
  if constexpr (OP == OP_BICG_INIT) nv = 4;
  if (i < Vh) {
    z A[12], B[12], C[12];
    if constexpr (OP == OP_ZERO) {
#pragma unroll
      for (int c = 0; c < 12; ++c) A[c] = z{0.0, 0.0};
      st<P>(a.v[0], slot, i, Vp, A);
    } else if constexpr (OP == OP_COPY) {
      ld<P>(a.v[1], slot, i, Vp, A);
      st<P>(a.v[0], slot, i, Vp, A);
    } else if constexpr (OP == OP_BICG_INIT) {
      ld<P>(a.v[1], slot, i, Vp, A);
      st<P>(a.v[2], slot, i, Vp, A);
      red[0] = norm2(A);
      // The shadow residual rh only enters dot products: any fixed vector not
      // orthogonal to r serves.  It is r itself, or, when the previous start
      // broke down (<rh, M r> = 0), a pseudo-random vector of unit entries
      // (+-1 +- i) drawn from an integer hash of (site, component), the same
      // for every slot and every start.
      const bool rnd = a.sc[slot].shadow != 0;  // uniform over the slot's blocks
      if (rnd) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const unsigned h = hash32((unsigned)i * 12u + (unsigned)c);
          C[c] = z{(h & 1u) ? 1.0 : -1.0, (h & 2u) ? 1.0 : -1.0};
        }
      } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) C[c] = A[c];
      }
      // rho = <rh, r> with rh as stored (rounded when its precision is lower)
      if constexpr (rh_prec(P) != P) {
        static_assert(rh_prec(P) == F16, "a lower-precision rh is stored in FP16");
        SpinorIO<F16>::store_decoded<true, true>(a.v[0], slot, i, Vp, C, B);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const z d = cjmul(B[c], A[c]);
          red[1] += d.x;
          red[2] += d.y;
        }
        red[3] = norm2(B);
      } else if (rnd) {
        st<P>(a.v[0], slot, i, Vp, C);  // unit entries: exact in every precision
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const z d = cjmul(C[c], A[c]);
          red[1] += d.x;
          red[2] += d.y;
        }
        red[3] = norm2(C);
      } else {
        st<P>(a.v[0], slot, i, Vp, A);
        red[1] = red[0];
        red[3] = red[0];
      }
#pragma unroll
      for (int c = 0; c < 12; ++c) B[c] = z{0.0, 0.0};
      st<P>(a.v[3], slot, i, Vp, B);
      st<PX>(a.v[4], slot, i, Vp, B);
    } else if constexpr (OP == OP_BICG_P) {
      const SlotScalars& s = a.sc[slot];
      const z beta{s.beta[0], s.beta[1]}, omega{s.omega[0], s.omega[1]};
      ld<P>(a.v[0], slot, i, Vp, A);  // p
      ld<P>(a.v[1], slot, i, Vp, B);  // r
      ld<P>(a.v[2], slot, i, Vp, C);  // v
#pragma unroll
      for (int c = 0; c < 12; ++c) A[c] = B[c] + cmul(beta, A[c] - cmul(omega, C[c]));
      st<P>(a.v[0], slot, i, Vp, A);
    } else if constexpr (OP == OP_BICG_S) {
      const SlotScalars& s = a.sc[slot];
      const z alpha{s.alpha[0], s.alpha[1]};
      ld<P>(a.v[1], slot, i, Vp, B);  // r
      ld<P>(a.v[2], slot, i, Vp, C);  // v
#pragma unroll
      for (int c = 0; c < 12; ++c) A[c] = B[c] - cmul(alpha, C[c]);
      st<P>(a.v[0], slot, i, Vp, A);
    } else if constexpr (OP == OP_BICG_XR) {
      const SlotScalars& s = a.sc[slot];
      const z alpha{s.alpha[0], s.alpha[1]}, omega{s.omega[0], s.omega[1]};
      z D[12], E[12];
      // every load before the first store, so that they can all be in flight
      ld<PX>(a.v[0], slot, i, Vp, A);  // x
      ld<P>(a.v[1], slot, i, Vp, B);   // p
      ld<P>(a.v[2], slot, i, Vp, C);   // s
      ld<P>(a.v[4], slot, i, Vp, D);   // t
      ld<rh_prec(P)>(a.v[5], slot, i, Vp, E);  // rh
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        A[c] = A[c] + cmul(alpha, B[c]) + cmul(omega, C[c]);
        C[c] = C[c] - cmul(omega, D[c]);  // r
        const z d = cjmul(E[c], C[c]);
        red[0] += d.x;
        red[1] += d.y;
      }
      red[2] = norm2(C);
      st<PX>(a.v[0], slot, i, Vp, A);
      st<P>(a.v[3], slot, i, Vp, C);
    } else if constexpr (OP == OP_BICG_XRP) {
      const SlotScalars& s = a.sc[slot];
      const z alpha{s.alpha[0], s.alpha[1]}, omega{s.omega[0], s.omega[1]}, beta{s.beta[0], s.beta[1]};
      z D[12], E[12];
      ld<PX>(a.v[0], slot, i, Vp, A);  // x
      ld<P>(a.v[1], slot, i, Vp, B);   // p
      ld<P>(a.v[2], slot, i, Vp, C);   // s
      ld<P>(a.v[4], slot, i, Vp, D);   // t
      ld<P>(a.v[5], slot, i, Vp, E);   // v
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        A[c] = A[c] + cmul(alpha, B[c]) + cmul(omega, C[c]);
        C[c] = C[c] - cmul(omega, D[c]);                     // r
        B[c] = C[c] + cmul(beta, B[c] - cmul(omega, E[c]));  // next p
      }
      red[0] = norm2(C);
      st<PX>(a.v[0], slot, i, Vp, A);
      st<P>(a.v[1], slot, i, Vp, B);
      st<P>(a.v[3], slot, i, Vp, C);
    } else if constexpr (OP == OP_CG_XR) {
      const double ca = a.sc[slot].cg_a;
      z D[12];
      ld<PX>(a.v[0], slot, i, Vp, A);  // x
      ld<P>(a.v[1], slot, i, Vp, B);   // p
      ld<P>(a.v[2], slot, i, Vp, C);   // r
      ld<P>(a.v[3], slot, i, Vp, D);   // w
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        A[c] = A[c] + ca * B[c];
        C[c] = C[c] - ca * D[c];
      }
      red[0] = norm2(C);
      st<PX>(a.v[0], slot, i, Vp, A);
      st<P>(a.v[2], slot, i, Vp, C);
    } else if constexpr (OP == OP_CG_P) {
      const double cb = a.sc[slot].cg_b;
      ld<P>(a.v[0], slot, i, Vp, A);  // p
      ld<P>(a.v[1], slot, i, Vp, B);  // z
#pragma unroll
      for (int c = 0; c < 12; ++c) A[c] = B[c] + cb * A[c];
      st<P>(a.v[0], slot, i, Vp, A);
    } else if constexpr (OP == OP_SCALE_COPY) {
      const double f = a.slot_scale[slot];
      ld<F64>(a.v[1], slot, i, Vp, B);
#pragma unroll
      for (int c = 0; c < 12; ++c) A[c] = f * B[c];
      st<P>(a.v[0], slot, i, Vp, A);
    } else if constexpr (OP == OP_AXPY_SCALED) {
      const double f = a.slot_scale[slot];
      ld<F64>(a.v[0], slot, i, Vp, A);
      ld<PX>(a.v[1], slot, i, Vp, B);
#pragma unroll
      for (int c = 0; c < 12; ++c) A[c] = A[c] + f * B[c];
      st<F64>(a.v[0], slot, i, Vp, A);
    } else if constexpr (OP == OP_SUB64) {
      ld<F64>(a.v[1], slot, i, Vp, B);
      ld<F64>(a.v[2], slot, i, Vp, C);
#pragma unroll
      for (int c = 0; c < 12; ++c) A[c] = B[c] - C[c];
      st<F64>(a.v[0], slot, i, Vp, A);
      red[0] = norm2(A);
    } else if constexpr (OP == OP_TO64) {
      ld<P>(a.v[1], slot, i, Vp, B);
      st<F64>(a.v[0], slot, i, Vp, B);
    } else if constexpr (OP == OP_NORM) {
      ld<P>(a.v[1], slot, i, Vp, B);
      red[0] = norm2(B);
    }
  }
  if (nv > 0 && a.red.fin != FIN_NONE) block_reduce_store(a.red, nv, red, slot, blockIdx.x, gridDim.x);
}

// one block per slot: fold the block partials in a fixed order, then
// finalise.  The fold is latency bound (a few thousand partials per slot), so
// the block is wide and each thread keeps four partials in flight.
constexpr int kFinBlock = 1024;
__global__ void __launch_bounds__(kFinBlock) finalize_kernel(ReduceRef red, int nv, int nblocks, const int* mask) {
  const int slot = blockIdx.x;
  if (mask && !mask[slot]) return;
  __shared__ double lds[kRedMax][kFinBlock / 64];
  const double* part = red.partials + (long)slot * nblocks * kRedMax;
  double acc[kRedMax] = {};
  int b = threadIdx.x;
  for (; b + 3 * kFinBlock < nblocks; b += 4 * kFinBlock) {
    double q[4][kRedMax];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < kRedMax; ++k) q[u][k] = k < nv ? part[(long)(b + u * kFinBlock) * kRedMax + k] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < kRedMax; ++k) acc[k] += q[u][k];
  }
  for (; b < nblocks; b += kFinBlock)
    for (int k = 0; k < nv; ++k) acc[k] += part[(long)b * kRedMax + k];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < nv; ++k) {
    const double w = wave_sum(acc[k]);
    if (lane == 0) lds[k][wid] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[kRedMax] = {};
    for (int k = 0; k < nv; ++k)
      for (int w = 0; w < kFinBlock / 64; ++w) s[k] += lds[k][w];
    run_finaliser(red, slot, s);
  }
}

template <int P>
hipError_t launch_p(int op, const BlasArgs& a, dim3 grid, hipStream_t st) {
  switch (op) {
#define DP_BLAS_CASE(OPV) \
  case OPV: hipLaunchKernelGGL((blas_kernel<P, OPV>), grid, dim3(kBlock), 0, st, a); break;
    DP_BLAS_CASE(OP_ZERO)
    DP_BLAS_CASE(OP_COPY)
    DP_BLAS_CASE(OP_BICG_INIT)
    DP_BLAS_CASE(OP_BICG_P)
    DP_BLAS_CASE(OP_BICG_S)
    DP_BLAS_CASE(OP_BICG_XR)
    DP_BLAS_CASE(OP_BICG_XRP)
    DP_BLAS_CASE(OP_CG_XR)
    DP_BLAS_CASE(OP_CG_P)
    DP_BLAS_CASE(OP_SCALE_COPY)
    DP_BLAS_CASE(OP_AXPY_SCALED)
    DP_BLAS_CASE(OP_SUB64)
    DP_BLAS_CASE(OP_NORM)
    DP_BLAS_CASE(OP_TO64)
#undef DP_BLAS_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_finalize(const ReduceRef& red, int nv, int nblocks, int nslots, const int* mask, hipStream_t st) {
  if (nslots <= 0 || nv < 1 || nv > kRedMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(finalize_kernel, dim3(nslots), dim3(kFinBlock), 0, st, red, nv, nblocks, mask);
  return hipGetLastError();
}

hipError_t launch_blas(int op, const BlasArgs& a, hipStream_t st) {
  if (a.nslots <= 0 || a.g.Vh <= 0) return hipErrorInvalidValue;
  const int nb = reduction_blocks(a.g);
  const dim3 grid(nb, a.nslots);
  hipError_t e;
  switch (a.prec) {
    case F64: e = launch_p<F64>(op, a, grid, st); break;
    case F32: e = launch_p<F32>(op, a, grid, st); break;
    case F16: e = launch_p<F16>(op, a, grid, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess || a.red.fin == FIN_NONE) return e;
  const int nv = op == OP_BICG_INIT                                                              ? 4
                 : op == OP_BICG_XR                                                           ? 3
                 : (op == OP_CG_XR || op == OP_SUB64 || op == OP_NORM || op == OP_BICG_XRP) ? 1
                                                                                             : 0;
  if (nv == 0) return hipErrorInvalidValue;
  return launch_finalize(a.red, nv, nb, a.nslots, a.mask, st);
}

}  // namespace dp
