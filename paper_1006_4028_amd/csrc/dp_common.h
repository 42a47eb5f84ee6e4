// Internal declarations shared by the HIP translation units of libdp.
//
// Device data layout (all fields split by checkerboard parity p = (x0+x1+x2+x3)&1,
// index within a parity i = lexicographic_site >> 1 with x0 slowest, so a
// timeslice is a contiguous range of Vsh = L1*L2*L3/2 indices):
//
//   spinor, FP64 : double2 [12][Vh]        component c = 3*spin + colour
//   spinor, FP32 : float4  [6][Vh]         components (2k, 2k+1) packed
//   spinor, FP16 : uint4   [3][Vh]         8 halves (4 complex) per uint4,
//                  + float scale[Vh]       value = half * scale (per-site max)
//   links, FP64  : double2 [4][9][Vh]      U_mu(x)[a][b] at the sites of one parity
//   links, FP32  : float2  [4][9][Vh]
//   links, FP16  : __half2 [4][9][Vh]      |U_ab| <= 1 for SU(3), no scale
//   clover, FP64 : double2 [36][Vh]        two Hermitian 6x6 blocks (upper and
//   clover, FP32 : float4  [18][Vh]        lower chirality), 36 reals each:
//   clover, FP16 : uint4   [9][Vh]         6 diagonal reals, then the 15 upper
//                  + float scale[Vh]       off-diagonal entries (i<j, row-major)
//
// Several right-hand sides ("slots") are stored one after the other with a
// fixed slot stride.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace dp {

enum Prec { F64 = 0, F32 = 1, F16 = 2 };

struct Geom {
  int T, L1, L2, L3;
  int L3h;  // L3 / 2
  int Vsh;  // sites of one parity in one timeslice
  int Vh;   // sites of one parity
  int Vp;   // component stride of every structure-of-arrays field (Vh padded)
};

// Bytes of one site of one parity in each storage format.
inline size_t spinor_site_bytes(int prec) { return prec == F64 ? 192 : prec == F32 ? 96 : 48; }
inline size_t spinor_scale_bytes(int prec) { return prec == F16 ? 4 : 0; }
inline size_t link_site_bytes(int prec) { return prec == F64 ? 576 : prec == F32 ? 288 : 144; }
inline size_t clover_site_bytes(int prec) { return prec == F64 ? 576 : prec == F32 ? 288 : 144; }

// A spinor field of one parity for nslots right-hand sides.
struct SpinorRef {
  void* data = nullptr;     // storage units as documented above
  float* scale = nullptr;   // FP16 only
  long slot_stride = 0;     // elements of the storage unit between slots
  long scale_stride = 0;    // floats between slots
  int prec = F64;
};

// A clover-block field of one parity (C or A^-1).
struct CloverRef {
  const void* data = nullptr;
  const float* scale = nullptr;
  int prec = F64;
};

// Per-slot parameters in device memory.
struct SlotTable {
  const double* ratio = nullptr;  // [nslots][4][T]: fwd, bwd, fwd_dag, bwd_dag
  const double* m4 = nullptr;     // [nslots] 4 + M
  const int* mask = nullptr;      // [nslots] nonzero = slot takes part
  const void* const* ainv = nullptr;          // [nslots] A_oo^-1 field of the slot's mass
  const float* const* ainv_scale = nullptr;   // [nslots] FP16 scales (or null)
  // the A_oo^-1 field when every slot of the launch has the same mass (the
  // slots' own ainv entries then point to it too), else null
  const void* ainv_common = nullptr;
  const float* ainv_common_scale = nullptr;
};

// Solver scalars of one slot, device resident (written by the finalisers of
// fused reductions, read by the following kernels of the same iteration).
struct SlotScalars {
  double rho[2], alpha[2], omega[2], beta[2];  // BiCGStab, complex
  double rr;      // |r|^2 of the iterated residual
  double rh2;     // |rh|^2 of the shadow residual
  double zz;      // CGNR |z|^2
  double cg_a;    // CGNR step length
  double cg_b;    // CGNR beta
  double tol2;    // the slot leaves the inner solve once rr <= tol2
  int iters;      // inner iterations done by the slot (over all its inner solves)
  int max_iter;   // ... or once iters reaches max_iter
  int breakdown;  // 1: rho collapsed, 2: <rh, v> = 0, 3: omega = 0
  int left;       // why it left: 1 converged, 2 breakdown, 3 max_iter, 4 non-finite
  int shadow;     // BiCGStab shadow residual of the next start: 0 the start
                  // residual, 1 a fixed pseudo-random vector (after a breakdown)
};

// Epilogues of the hop kernel.
enum Epi {
  EPI_HOP = 0,      // out = H in
  EPI_INV = 1,      // out = A^-1 (H in)               (slot mass)
  EPI_DIAG = 2,     // out = (C + m4) xin + sign * H in
  EPI_SUB = 3,      // out = xin - H in
  EPI_INV_SUB = 4,  // out = A^-1 (xin - H in)
};

// Reductions fused into a kernel's epilogue; results land in per-slot block
// partials, and a finalise kernel on the same stream folds them in a fixed
// order and runs a finaliser.
enum Red {
  RED_NONE = 0,
  RED_DOT_EXT = 1,  // <w, out>      (w = extra vector, e.g. the shadow residual)
  RED_TS = 2,       // <out, xin>, |out|^2
  RED_NORM = 3,     // |out|^2
  RED_TS4 = 4,      // <out, xin>, |out|^2, <w, xin>, <w, out>
};

// Storage precision of BiCGStab's shadow residual rh for inner precision P.
// rh only enters dot products and may be any fixed vector not orthogonal to
// the start residual: with an FP32 inner solver it is the start residual
// rounded to FP16 (with per-site scales), which halves the bytes the two
// even-site kernels of an iteration read for it.
__host__ __device__ constexpr int rh_prec(int p) { return p == F32 ? F16 : p; }

// values per reduction partial (at most 7 are used)
constexpr int kRedMax = 8;
__host__ __device__ constexpr int red_values(int red) {
  return red == RED_DOT_EXT ? 2 : red == RED_TS ? 3 : red == RED_TS4 ? 7 : red == RED_NORM ? 1 : 0;
}

enum Fin {
  FIN_NONE = 0,
  FIN_BICG_ALPHA = 1,  // sums <rh, v>            -> alpha = rho / <rh, v>
  FIN_BICG_OMEGA = 2,  // sums <t, s>, |t|^2      -> omega
  FIN_BICG_RHO = 3,    // sums <rh, r>, |r|^2     -> rho, beta, rr, breakdown
  FIN_BICG_INIT = 4,   // sums |r|^2, <rh, r>, |rh|^2 -> rho, rr, rh2, alpha = omega = 1
  FIN_CG_ALPHA = 5,    // sums |w|^2              -> cg_a = zz / |w|^2
  FIN_CG_BETA = 6,     // sums |z|^2              -> cg_b = |z|^2 / zz, zz
  FIN_CG_INIT = 7,     // sums |z|^2              -> zz
  FIN_RR = 8,          // sums |r|^2              -> rr
  FIN_STORE = 9,       // raw sums                -> out_sums[slot][k]
  FIN_BICG_OMEGA_RHO = 10,  // sums <t,s>, |t|^2, <rh,s>, <rh,t> -> omega, rho = <rh, s - omega t>, beta
  FIN_BICG_RR = 11,         // sums |r|^2             -> rr, breakdown test, end of the iteration
};

struct ReduceRef {
  int red = RED_NONE;
  int fin = FIN_NONE;
  SpinorRef w;               // RED_DOT_EXT partner
  double* partials = nullptr;   // [nslots][nblocks][kRedMax]
  SlotScalars* sc = nullptr;    // [nslots]
  double* out_sums = nullptr;   // FIN_STORE: [nslots][4]
  int* inner_mask = nullptr;    // [nslots] cleared when a slot leaves the inner solve
};

struct HopArgs {
  Geom g;
  int p;               // parity of the output sites
  int dag;             // 1: adjoint hop (projectors flipped, reciprocal ratios)
  int epi;
  double sign;         // EPI_DIAG sign of the hop term
  const void* U_out;   // links at output-parity sites
  const void* U_in;    // links at input-parity sites
  int link_prec;
  SpinorRef in, out, xin;
  CloverRef clov;      // C of the output parity (EPI_DIAG)
  SlotTable slots;
  ReduceRef red;
  int nslots;
  // spatial hop ratios of the light-quark factorisation (nullptr: all ones):
  // direction k = 1, 2, 3 at offset 4 (L1 + .. + L_{k-1}), four tables of L_k
  // entries each: fwd[x_k] = a_k(x_k)/a_k(x_k+1), bwd[x_k] = a_k(x_k)/a_k(x_k-1)
  // (periodic), then the same for 1/a_k (the adjoint)
  const double* sratio;
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `stream` and return hipSuccess or the launch error.

// The hop kernel alone; *nparts receives the number of per-slot block partials
// it stored for a fused reduction (a.red.red != RED_NONE), which the caller
// folds next with launch_finalize(a.red, nv, *nparts, ...).
hipError_t launch_hop(const HopArgs& a, hipStream_t stream, int* nparts);

// FP64 host-layout gauge field [site][mu][3][3] (device copy) -> SoA parity fields;
// U_aos == nullptr gives unit links
hipError_t launch_gauge_reorder(const Geom& g, const double2* U_aos, void* U_eo[2], int prec,
                                hipStream_t stream);
// Clover blocks from the FP64 parity links: out_eo[p] = packed C (FP64), both parities.
hipError_t launch_clover_build(const Geom& g, const double2* U64_eo[2], double csw, double2* C_eo[2],
                               hipStream_t stream);
// Host-layout dense clover [site][12][12] (device copy) -> packed blocks; flags
// nonzero on entries outside the two chiral blocks or non-Hermitian parts.
hipError_t launch_clover_pack(const Geom& g, const double2* C_aos, double2* C_eo[2], int* bad,
                              hipStream_t stream);
// A^-1 = (C + m4)^-1 per block (FP64 Gauss-Jordan with pivoting), packed; *bad is
// set when a block is singular.
hipError_t launch_clover_invert(const Geom& g, const double2* C64, double m4, double2* Ainv64, int* bad,
                                hipStream_t stream);
// out = A^-1 in per slot (the slot's A^-1 field), FP64 parity fields.
hipError_t launch_clover_apply(const Geom& g, const SlotTable& slots, SpinorRef in, SpinorRef out, int nslots,
                               hipStream_t stream);
// Convert packed FP64 clover blocks to FP32 / FP16(+scale).
hipError_t launch_clover_convert(const Geom& g, const double2* C64, void* out, float* scale, int prec,
                                 hipStream_t stream);

// Host-layout spinors [slot][site][4][3] complex128 (device) <-> parity fields.
// alpha_mul: optional [nslots][T] factors applied on the way (nullptr = 1).
// alpha_mul / alpha_div: per-slot time profiles [slot][T] (nullable); sprof:
// the spatial profiles a_1[L1], a_2[L2], a_3[L3] one after the other (nullable)
hipError_t launch_spinor_import(const Geom& g, const double2* aos, int nslots, long aos_slot_stride,
                                int p, SpinorRef dst, const double* alpha_mul, const double* sprof,
                                hipStream_t stream);
hipError_t launch_spinor_export(const Geom& g, SpinorRef even, SpinorRef odd, int nslots,
                                const double* alpha_div, const double* sprof, double2* aos, long aos_slot_stride,
                                hipStream_t stream);
// Schroedinger functional: the interior clover blocks from those built on the
// lattice padded with the two boundary timeslices (gp: T + 2 timeslices),
// plus ctm1 on the diagonal of the first and last interior timeslices.
hipError_t launch_clover_sf_interior(const Geom& g, const Geom& gp, const double2* Cp_eo[2], double ctm1,
                                     double2* C_eo[2], hipStream_t stream);
// Schroedinger functional boundary sources: side 0, U_0(0, xs)^+ P+ e_c on
// the first interior timeslice; side 1, U_0(T, xs) P- e_c on the last (U_t:
// the links of that boundary-adjacent timeslice of the padded lattice, x0 = 0
// or x0 = T, host layout [xs][mu][3][3] complex).
hipError_t launch_sf_wall_sources(const Geom& g, const double2* U_t, int side, int c0, int ncols, double2* out,
                                  hipStream_t st);
// ncols unit point sources (host layout, double2 per complex): column j is 1
// in spin-colour component c0 + j at site {x0, x1, x2, x3}, 0 elsewhere.
hipError_t launch_point_sources(const Geom& g, const int site[4], int c0, int ncols, double2* out,
                                hipStream_t stream);
// Per-timeslice sum of |psi|^2 over both parities, written to cpp[slot][t]
// (as -sum, t = (x0 - x0_src[slot]) mod T), FP64 fields, divided by alpha^2.
hipError_t launch_cpp(const Geom& g, SpinorRef even, SpinorRef odd, int nslots, const double* alpha,
                      const double* sprof, const int* x0_src, double* cpp, hipStream_t stream);

// ------------------------------------------------------------- BLAS kernels
// Vector kernels over the even sites of every active slot.  Krylov vectors
// are in the inner precision P; the inner solution x is FP32 when P is FP16
// (P otherwise); FP64 vectors are named as such.
struct BlasArgs {
  Geom g;
  int nslots;
  int prec;                    // inner precision P
  const int* mask = nullptr;   // [nslots]
  SlotScalars* sc = nullptr;   // [nslots]
  const double* slot_scale = nullptr;  // [nslots] per-slot factor (scale ops)
  SpinorRef v[6];
  ReduceRef red;
};

enum BlasOp {
  OP_ZERO = 0,        // v0 = 0
  OP_COPY = 1,        // v0 = v1                                  (P)
  OP_BICG_INIT = 2,   // v0(rh) = v1(r) (or the pseudo-random shadow); v2(p) = r; v3(v) = 0; v4(x) = 0;
                      // red |r|^2, <rh, r>, |rh|^2 -> FIN_BICG_INIT
  OP_BICG_P = 3,      // v0(p) = v1(r) + beta (p - omega v2(v))
  OP_BICG_S = 4,      // v0(s) = v1(r) - alpha v2(v)
  OP_BICG_XR = 5,     // v0(x) += alpha v1(p) + omega v2(s); v3(r) = s - omega v4(t); red <v5(rh), r>, |r|^2
  OP_CG_XR = 6,       // v0(x) += a v1(p); v2(r) -= a v3(w);      red |r|^2
  OP_CG_P = 7,        // v0(p) = v1(z) + b p
  OP_SCALE_COPY = 8,  // v0(P) = slot_scale * v1(F64)
  OP_AXPY_SCALED = 9, // v0(F64) += slot_scale * v1(x precision)
  OP_SUB64 = 10,      // v0(F64) = v1(F64) - v2(F64);             red |v0|^2
  OP_NORM = 11,       // red |v1|^2                               (precision of v1)
  OP_TO64 = 12,       // v0(F64) = v1(P)
  OP_BICG_XRP = 13,   // v0(x) += alpha v1(p) + omega v2(s); v3(r) = s - omega v4(t);
                      // p = r + beta (p - omega v5(v));  red |r|^2 -> FIN_BICG_RR
};

hipError_t launch_blas(int op, const BlasArgs& a, hipStream_t stream);

// Fold the per-block partials of every active slot (mask may be null) in block
// order and run red.fin; nv values per block, nblocks blocks per slot.
hipError_t launch_finalize(const ReduceRef& red, int nv, int nblocks, int nslots, const int* mask,
                           hipStream_t stream);

// Number of blocks a BLAS launch (reduction_blocks) and a hop launch
// (hop_blocks) use for a given geometry, to size the partials buffer.
int reduction_blocks(const Geom& g);
int hop_blocks(const Geom& g);
constexpr int kBlock = 256;

}  // namespace dp
