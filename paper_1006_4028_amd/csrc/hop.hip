// The alpha-hop Wilson kernel with clover epilogues.
//
// For an output site x of parity p it computes the hopping term of the
// preconditioned operator D' = alpha (D + M) alpha^-1 (eq. linsysprec),
//
//   H psi(x) = -1/2 sum_mu [ c+_mu(x) (1 - gamma_mu) U_mu(x) psi(x+mu)
//                          + c-_mu(x) (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
//
// where the time factors are the ratios of the modified time derivatives
// (heavy-quark section): c+_0(x) = alpha(x0)/alpha(x0+1) and c-_0(x) =
// alpha(x0)/alpha(x0-1), per slot, with the fermion boundary sign folded in at
// the wrap-around (the boundary rule eq. redeftbc reduces to exactly this),
// and the spatial factors are 1, or the same ratios of the spatial profiles
// of the light-quark factorisation (eqs. betaa, redefcovs; periodic).
// The adjoint hop (dag = 1) swaps the projectors and uses the reciprocal
// ratios; it is the hopping part of gamma5 D'(1/alpha) gamma5 = D'(alpha)^+.
//
// Spin projection in the chiral basis, with psi = (u0, u1, l0, l1) in spin and
// s = +1 for (1 - gamma_mu), s = -1 for (1 + gamma_mu):
//   mu = 0: h = u + s l,                 lower = s h
//   mu = k: h = u + s (i sigma_k) l,     lower = -s (i sigma_k) h
// so only the two upper spins are multiplied by the link.
//
// One thread per output site and group of one or two right-hand sides
// ("slots"); the links of the site are loaded once for the group.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "dp_device.h"

namespace dp {

namespace {

template <typename R>
struct Half {
  cx<R> h[2][3];
};

template <int MU, int S, typename R>
__device__ __forceinline__ void project(const cx<R> (&s)[12], Half<R>& o) {
  constexpr R sg = R(S);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cx<R> u0 = s[a], u1 = s[3 + a], l0 = s[6 + a], l1 = s[9 + a];
    if constexpr (MU == 0) {
      o.h[0][a] = u0 + sg * l0;
      o.h[1][a] = u1 + sg * l1;
    } else if constexpr (MU == 1) {  // i sigma_1 l = (i l1, i l0)
      o.h[0][a] = u0 + sg * ti(l1);
      o.h[1][a] = u1 + sg * ti(l0);
    } else if constexpr (MU == 2) {  // i sigma_2 l = (l1, -l0)
      o.h[0][a] = u0 + sg * l1;
      o.h[1][a] = u1 - sg * l0;
    } else {  // i sigma_3 l = (i l0, -i l1)
      o.h[0][a] = u0 + sg * ti(l0);
      o.h[1][a] = u1 - sg * ti(l1);
    }
  }
}

// acc += c * (1 - s gamma_mu)-reconstruction of the link-multiplied half spinor
template <int MU, int S, typename R>
__device__ __forceinline__ void accumulate(cx<R> (&acc)[12], const Half<R>& w, R c) {
  constexpr R sg = R(S);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cx<R> w0 = c * w.h[0][a], w1 = c * w.h[1][a];
    acc[a] = acc[a] + w0;
    acc[3 + a] = acc[3 + a] + w1;
    if constexpr (MU == 0) {
      acc[6 + a] = acc[6 + a] + sg * w0;
      acc[9 + a] = acc[9 + a] + sg * w1;
    } else if constexpr (MU == 1) {  // -s i sigma_1 w = -s (i w1, i w0)
      acc[6 + a] = acc[6 + a] - sg * ti(w1);
      acc[9 + a] = acc[9 + a] - sg * ti(w0);
    } else if constexpr (MU == 2) {  // -s i sigma_2 w = -s (w1, -w0)
      acc[6 + a] = acc[6 + a] - sg * w1;
      acc[9 + a] = acc[9 + a] + sg * w0;
    } else {  // -s i sigma_3 w = -s (i w0, -i w1)
      acc[6 + a] = acc[6 + a] - sg * ti(w0);
      acc[9 + a] = acc[9 + a] + sg * ti(w1);
    }
  }
}

template <typename R>
__device__ __forceinline__ void link_mul(const cx<R> (&u)[9], const Half<R>& h, Half<R>& o) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> t = cmul(u[3 * a], h.h[s][0]);
      cfma(t, u[3 * a + 1], h.h[s][1]);
      cfma(t, u[3 * a + 2], h.h[s][2]);
      o.h[s][a] = t;
    }
}

template <typename R>
__device__ __forceinline__ void link_dag_mul(const cx<R> (&u)[9], const Half<R>& h, Half<R>& o) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> t = cjmul(u[a], h.h[s][0]);
      cjfma(t, u[3 + a], h.h[s][1]);
      cjfma(t, u[6 + a], h.h[s][2]);
      o.h[s][a] = t;
    }
}

// One direction mu, both hops, for the active slots of this thread's group.
// The link is loaded once and used for every slot.  DAG selects the adjoint's
// projectors at compile time (the signs then cost no arithmetic); an FP16
// spinor's per-site scale multiplies the hop's coefficient instead of the 24
// loaded components (the projection and the link product are linear).
// With LDS the links come from the workgroup's copy lu[8][9][64] (direction
// 2 mu for the forward hop, 2 mu + 1 for the backward one; lane = site).
template <int P, int MU, int NS, bool DAG, bool LDS>
__device__ __forceinline__ void hop_dir(const HopArgs& a, const int (&sl)[NS], const bool (&on)[NS], int i,
                                        const int (&x)[4],
                                        const typename Tr<P>::R (&cf)[NS], const typename Tr<P>::R (&cb)[NS],
                                        const typename Tr<P>::R (&sp)[6], cx<typename Tr<P>::R> (&acc)[NS][12],
                                        const cx<typename Tr<P>::R>* lu, int lane) {
  using R = typename Tr<P>::R;
  constexpr int S = DAG ? -1 : 1;
  const Geom& g = a.g;
  const int L = MU == 0 ? g.T : MU == 1 ? g.L1 : MU == 2 ? g.L2 : g.L3;
  // spatial ratios of the light-quark factorisation (the time ones are per slot)
  const R sf = MU == 0 ? R(1) : sp[2 * MU - 2], sb = MU == 0 ? R(1) : sp[2 * MU - 1];
  int y[4] = {x[0], x[1], x[2], x[3]};
  cx<R> psi[12], u[9];
  Half<R> h, w;
  // forward neighbour x + mu
  y[MU] = x[MU] + 1 == L ? 0 : x[MU] + 1;
  const int jf = eo_index(g, y[0], y[1], y[2], y[3]);
  if constexpr (LDS) {
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = lu[((2 * MU) * 9 + k) * 64 + lane];
  } else {
    LinkIO<P>::load(a.U_out, MU, i, g.Vp, u);
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    if (on[k]) {
      const R sc = SpinorIO<P>::load_unscaled(a.in, sl[k], jf, g.Vp, psi);
      project<MU, S>(psi, h);
      link_mul(u, h, w);
      accumulate<MU, S>(acc[k], w, (MU == 0 ? cf[k] : sf) * sc);
    }
  }
  // backward neighbour x - mu
  y[MU] = x[MU] == 0 ? L - 1 : x[MU] - 1;
  const int jb = eo_index(g, y[0], y[1], y[2], y[3]);
  if constexpr (LDS) {
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = lu[((2 * MU + 1) * 9 + k) * 64 + lane];
  } else {
    LinkIO<P>::load(a.U_in, MU, jb, g.Vp, u);
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    if (on[k]) {
      const R sc = SpinorIO<P>::load_unscaled(a.in, sl[k], jb, g.Vp, psi);
      project<MU, -S>(psi, h);
      link_dag_mul(u, h, w);
      accumulate<MU, -S>(acc[k], w, (MU == 0 ? cb[k] : sb) * sc);
    }
  }
}

// ---------------------------------------------------------------- batched
// The shared-tile kernel's hop for one slot, neighbour by neighbour in the
// order of hop_dir (K = 2 mu forward, 2 mu + 1 backward) and with its
// arithmetic, but the loads of PF neighbours are issued together before the
// first of them is used (a scheduling barrier keeps the compiler from
// spreading them out again): more bytes in flight per wave.

// Number of neighbours whose loads are issued together, per storage precision.
#ifndef DP_SHARED_PF32
#define DP_SHARED_PF32 4
#endif
#ifndef DP_SHARED_PF16
#define DP_SHARED_PF16 4
#endif
template <int P>
constexpr int shared_pf() {
  return P == F16 ? DP_SHARED_PF16 : P == F32 ? DP_SHARED_PF32 : 2;
}

// The one-slot FP32 slab kernel runs the same batched code with the links
// read from memory, prefetched with the spinors (measured on MI355X at
// 24^3x48: 3% faster than the per-direction code); FP16 keeps the latter.
#ifndef DP_SLAB_PF32
#define DP_SLAB_PF32 4
#endif
#ifndef DP_SLAB_PF16
#define DP_SLAB_PF16 0
#endif
template <int P>
constexpr int slab_pf() {
  return P == F32 ? DP_SLAB_PF32 : P == F16 ? DP_SLAB_PF16 : 0;
}

template <int P>
struct RawLink;
template <>
struct RawLink<F64> {
  double2 v[9];
};
template <>
struct RawLink<F32> {
  float2 v[9];
};
template <>
struct RawLink<F16> {
  unsigned v[9];
};

template <int P>
__device__ __forceinline__ void load_raw_link(const void* base, int mu, int i, int Vh, RawLink<P>& r) {
  using T = decltype(r.v[0]);
  using E = typename std::remove_reference<T>::type;
  const E* b = static_cast<const E*>(base) + (long)mu * 9 * Vh;
#pragma unroll
  for (int k = 0; k < 9; ++k) r.v[k] = b[(long)k * Vh + i];
}

template <int P, typename R>
__device__ __forceinline__ void decode_link(const RawLink<P>& r, cx<R> (&u)[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if constexpr (P == F16) {
      const float2 v = h2f(r.v[k]);
      u[k] = cx<R>{(R)v.x, (R)v.y};
    } else {
      u[k] = cx<R>{(R)r.v[k].x, (R)r.v[k].y};
    }
  }
}

template <int P, int K, bool DAG, bool LDSL>
__device__ __forceinline__ void nb_compute(const RawSpinor<P>& raw, const RawLink<P>& rl, typename Tr<P>::R coef,
                                           const cx<typename Tr<P>::R>* lu, int lane,
                                           cx<typename Tr<P>::R> (&acc)[12]) {
  using R = typename Tr<P>::R;
  constexpr int MU = K >> 1;
  constexpr bool FWD = (K & 1) == 0;
  constexpr int S = (DAG ? -1 : 1) * (FWD ? 1 : -1);
  cx<R> psi[12], u[9];
  Half<R> h, w;
  if constexpr (LDSL) {
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = lu[(K * 9 + k) * 64 + lane];
  } else {
    decode_link<P>(rl, u);
  }
  const R sc = decode_spinor<P>(raw, psi);
  project<MU, S>(psi, h);
  if constexpr (FWD) link_mul(u, h, w);
  else link_dag_mul(u, h, w);
  accumulate<MU, S>(acc, w, coef * sc);
}

template <int P, int K, int END, bool DAG, bool LDSL>
struct NbSeq {
  __device__ static __forceinline__ void run(const RawSpinor<P>* raw, const RawLink<P>* rl,
                                             const typename Tr<P>::R (&coef)[8], const cx<typename Tr<P>::R>* lu,
                                             int lane, cx<typename Tr<P>::R> (&acc)[12]) {
    nb_compute<P, K, DAG, LDSL>(raw[0], rl[0], coef[K], lu, lane, acc);
    NbSeq<P, K + 1, END, DAG, LDSL>::run(raw + 1, rl + 1, coef, lu, lane, acc);
  }
};
template <int P, int END, bool DAG, bool LDSL>
struct NbSeq<P, END, END, DAG, LDSL> {
  __device__ static __forceinline__ void run(const RawSpinor<P>*, const RawLink<P>*, const typename Tr<P>::R (&)[8],
                                             const cx<typename Tr<P>::R>*, int, cx<typename Tr<P>::R> (&)[12]) {}
};

// LDSL: links from the workgroup's LDS copy, else loaded with the spinors
// (forward hops from U_out at the output site, backward ones from U_in at the
// neighbour).
template <int P, int K0, int PF, bool DAG, bool LDSL>
__device__ __forceinline__ void nb_batches(const HopArgs& a, int slot, int i, const int (&nb)[8],
                                           const typename Tr<P>::R (&coef)[8], const cx<typename Tr<P>::R>* lu,
                                           int lane, cx<typename Tr<P>::R> (&acc)[12]) {
  static_assert(PF > 0 && 8 % PF == 0, "the batches must split the 8 neighbours evenly");
  if constexpr (K0 < 8) {
    RawSpinor<P> raw[PF];
    RawLink<P> rl[PF];  // unused (and eliminated) with LDS links
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      load_raw_spinor<P>(a.in, slot, nb[K0 + q], a.g.Vp, raw[q]);
      if constexpr (!LDSL) {
        const int K = K0 + q;
        if ((K & 1) == 0) load_raw_link<P>(a.U_out, K >> 1, i, a.g.Vp, rl[q]);
        else load_raw_link<P>(a.U_in, K >> 1, nb[K], a.g.Vp, rl[q]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    NbSeq<P, K0, K0 + PF, DAG, LDSL>::run(raw, rl, coef, lu, lane, acc);
    nb_batches<P, K0 + PF, PF, DAG, LDSL>(a, slot, i, nb, coef, lu, lane, acc);
  }
}

// Epilogue and fused reduction terms for one slot.  NT marks the epilogue's
// own inputs and the output as streamed (read or written once per launch).
// With LDS the clover blocks come from the workgroup's copy lc[72][64] of the
// stored values times the FP16 per-site scale (the same product the direct
// load forms, so the block is bitwise the same).
// Whether the shared-tile kernel stages the clover blocks of the even-site
// epilogue in LDS (else each wave reads them from memory, through L2).
#ifndef DP_SHARED_CLOVER32
#define DP_SHARED_CLOVER32 1
#endif
template <int P, int EPI>
constexpr bool shared_clover() {
  return EPI == EPI_DIAG && (P != F32 || DP_SHARED_CLOVER32);
}

// Chirality block h of the workgroup's LDS copy lc[72][64] (values in the
// order of the stored blocks: 6 diagonal reals, then 15 complex entries).
template <typename R>
__device__ __forceinline__ void lds_block(const float* lc, int h, int lane, HermBlock<R>& B) {
#pragma unroll
  for (int k = 0; k < 6; ++k) B.d[k] = (R)lc[(36 * h + k) * 64 + lane];
#pragma unroll
  for (int k = 0; k < 15; ++k)
    B.o[k] = cx<R>{(R)lc[(36 * h + 6 + 2 * k) * 64 + lane], (R)lc[(36 * h + 7 + 2 * k) * 64 + lane]};
}

template <int P, int EPI, int RED, bool NT, bool LDS, bool LINV>
__device__ __forceinline__ void epilogue(const HopArgs& a, int slot, int i, cx<typename Tr<P>::R> (&acc)[12],
                                         double (&red)[kRedMax], const float* lc, int lane) {
  using R = typename Tr<P>::R;
  const Geom& g = a.g;
  cx<R> out[12], xin[12], wv[12];
  if constexpr (EPI == EPI_DIAG || EPI == EPI_SUB || EPI == EPI_INV_SUB)
    SpinorIO<P>::template load<NT>(a.xin, slot, i, g.Vp, xin);
  // the dot partner w is loaded after the output is formed (fewer live registers)
  if constexpr (EPI == EPI_HOP) {
#pragma unroll
    for (int c = 0; c < 12; ++c) out[c] = R(-0.5) * acc[c];
  } else if constexpr (EPI == EPI_DIAG) {
    const R m4 = (R)a.slots.m4[slot];
    if constexpr (LDS && shared_clover<P, EPI>()) {
      // one chirality block at a time (fewer live registers); the values
      // are already scaled
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        HermBlock<R> Bh;
        lds_block(lc, h, lane, Bh);
        herm_apply(Bh, m4, &xin[6 * h], &out[6 * h]);
      }
    } else {
      HermBlock<R> B[2];
      CloverIO<P>::load(a.clov.data, a.clov.scale, i, g.Vp, B);
      herm_apply(B[0], m4, &xin[0], &out[0]);
      herm_apply(B[1], m4, &xin[6], &out[6]);
    }
    const R hs = (R)(-0.5 * a.sign);
#pragma unroll
    for (int c = 0; c < 12; ++c) out[c] = out[c] + hs * acc[c];
  } else if constexpr (EPI == EPI_SUB) {
#pragma unroll
    for (int c = 0; c < 12; ++c) out[c] = xin[c] + R(0.5) * acc[c];
  } else {  // EPI_INV, EPI_INV_SUB
    cx<R> t[12];
    if constexpr (EPI == EPI_INV_SUB) {
#pragma unroll
      for (int c = 0; c < 12; ++c) t[c] = xin[c] + R(0.5) * acc[c];
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) t[c] = R(-0.5) * acc[c];
    }
    if constexpr (LDS && LINV) {  // every slot's A^-1 is the workgroup's copy (scaled)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        HermBlock<R> Bh;
        lds_block(lc, h, lane, Bh);
        herm_apply(Bh, R(0), &t[6 * h], &out[6 * h]);
      }
    } else {
      HermBlock<R> B[2];
      const float* sc = a.slots.ainv_scale ? a.slots.ainv_scale[slot] : nullptr;
      CloverIO<P>::load(a.slots.ainv[slot], sc, i, g.Vp, B);
      herm_apply(B[0], R(0), &t[0], &out[0]);
      herm_apply(B[1], R(0), &t[6], &out[6]);
    }
  }
  SpinorIO<P>::template store<NT>(a.out, slot, i, g.Vp, out);
  if constexpr (RED == RED_DOT_EXT || RED == RED_TS4)
    SpinorIO<rh_prec(P)>::template load<NT>(a.red.w, slot, i, g.Vp, wv);
  // The 12 components are summed in the arithmetic precision R per lane and
  // added to the FP64 partials once; the wave, block and launch sums are
  // FP64 (measured on MI355X at 24^3x48 with 12 slots: FP32 even-site kernel
  // in the solve 355 -> 348 us against per-component FP64 sums).
  if constexpr (RED == RED_DOT_EXT) {
    R s0 = R(0), s1 = R(0);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      s0 += wv[c].x * out[c].x + wv[c].y * out[c].y;
      s1 += wv[c].x * out[c].y - wv[c].y * out[c].x;
    }
    red[0] += (double)s0;
    red[1] += (double)s1;
  } else if constexpr (RED == RED_TS || RED == RED_TS4) {
    R s0 = R(0), s1 = R(0), s2 = R(0);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      s0 += out[c].x * xin[c].x + out[c].y * xin[c].y;
      s1 += out[c].x * xin[c].y - out[c].y * xin[c].x;
      s2 += out[c].x * out[c].x + out[c].y * out[c].y;
    }
    red[0] += (double)s0;
    red[1] += (double)s1;
    red[2] += (double)s2;
    if constexpr (RED == RED_TS4) {
      R s3 = R(0), s4 = R(0), s5 = R(0), s6 = R(0);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        s3 += wv[c].x * xin[c].x + wv[c].y * xin[c].y;
        s4 += wv[c].x * xin[c].y - wv[c].y * xin[c].x;
        s5 += wv[c].x * out[c].x + wv[c].y * out[c].y;
        s6 += wv[c].x * out[c].y - wv[c].y * out[c].x;
      }
      red[3] += (double)s3;
      red[4] += (double)s4;
      red[5] += (double)s5;
      red[6] += (double)s6;
    }
  } else if constexpr (RED == RED_NORM) {
    R s0 = R(0);
#pragma unroll
    for (int c = 0; c < 12; ++c) s0 += out[c].x * out[c].x + out[c].y * out[c].y;
    red[0] += (double)s0;
  }
}

// The work of one thread: the hop for output site i (if valid) and the active
// slots of its group, the epilogue, and its share of the fused reductions
// (stored as the partial `part` of `nparts` per slot).
// With LDS (one wave per slot group in a workgroup sharing links and clover)
// each wave stores its own reduction partials.
template <int P, int EPI, int RED, int NS, bool NT, bool DAG, bool LDS = false, bool LINV = false>
__device__ __forceinline__ void site_work(const HopArgs& a, int grp, int i, bool valid, int part, int nparts,
                                          const cx<typename Tr<P>::R>* lu = nullptr,
                                          const float* lc = nullptr, int lane = 0) {
  using R = typename Tr<P>::R;
  const Geom& g = a.g;
  // active slots of the group (uniform over the block)
  int sl[NS];
  bool on[NS];
  bool any = false;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    sl[k] = grp * NS + k;
    on[k] = sl[k] < a.nslots && (!a.slots.mask || a.slots.mask[sl[k]]);
    if (!on[k]) sl[k] = 0;
    any = any || on[k];
  }
  if (!any) return;
  double red[NS][kRedMax];
#pragma unroll
  for (int k = 0; k < NS; ++k)
#pragma unroll
    for (int q = 0; q < kRedMax; ++q) red[k][q] = 0.0;
  if (valid) {
    int x[4];
    eo_coords(g, a.p, i, x[0], x[1], x[2], x[3]);
    R cf[NS], cb[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const double* rt = a.slots.ratio + (long)sl[k] * 4 * g.T;
      cf[k] = (R)(DAG ? rt[2 * g.T + x[0]] : rt[x[0]]);
      cb[k] = (R)(DAG ? rt[3 * g.T + x[0]] : rt[g.T + x[0]]);
    }
    cx<R> acc[NS][12];
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[k][c] = cx<R>{R(0), R(0)};
    // spatial ratios of the light-quark factorisation: fwd, bwd per direction
    R sp[6] = {R(1), R(1), R(1), R(1), R(1), R(1)};
    if (a.sratio) {  // uniform over the launch
      const int Ls[3] = {g.L1, g.L2, g.L3};
      int off = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sp[2 * k] = (R)a.sratio[off + (DAG ? 2 * Ls[k] : 0) + x[k + 1]];
        sp[2 * k + 1] = (R)a.sratio[off + (DAG ? 3 * Ls[k] : Ls[k]) + x[k + 1]];
        off += 4 * Ls[k];
      }
    }
    constexpr int PF = LDS ? shared_pf<P>() : slab_pf<P>();
    if constexpr (NS == 1 && PF > 0) {
      // neighbour loads issued in batches (the shared-tile kernel, and the
      // one-slot FP32 slab kernel with the same arithmetic)
      const Geom& gg = a.g;
      const int Ls[4] = {gg.T, gg.L1, gg.L2, gg.L3};
      int nb[8];
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
        int y[4] = {x[0], x[1], x[2], x[3]};
        y[mu] = x[mu] + 1 == Ls[mu] ? 0 : x[mu] + 1;
        nb[2 * mu] = eo_index(gg, y[0], y[1], y[2], y[3]);
        y[mu] = x[mu] == 0 ? Ls[mu] - 1 : x[mu] - 1;
        nb[2 * mu + 1] = eo_index(gg, y[0], y[1], y[2], y[3]);
      }
      const R coef[8] = {cf[0], cb[0], sp[0], sp[1], sp[2], sp[3], sp[4], sp[5]};
      if (on[0]) nb_batches<P, 0, PF, DAG, LDS>(a, sl[0], i, nb, coef, lu, lane, acc[0]);
    } else {
      hop_dir<P, 0, NS, DAG, LDS>(a, sl, on, i, x, cf, cb, sp, acc, lu, lane);
      hop_dir<P, 1, NS, DAG, LDS>(a, sl, on, i, x, cf, cb, sp, acc, lu, lane);
      hop_dir<P, 2, NS, DAG, LDS>(a, sl, on, i, x, cf, cb, sp, acc, lu, lane);
      hop_dir<P, 3, NS, DAG, LDS>(a, sl, on, i, x, cf, cb, sp, acc, lu, lane);
    }
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (on[k]) epilogue<P, EPI, RED, NT, LDS, LINV>(a, sl[k], i, acc[k], red[k], lc, lane);
  }
  if constexpr (RED != RED_NONE) {
    constexpr int nv = red_values(RED);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      if (!on[k]) continue;
      if constexpr (LDS) {
        // the same sum as block_reduce_store over a 64-thread block
        double* pt = a.red.partials + ((long)sl[k] * nparts + part) * kRedMax;
        for (int q = 0; q < nv; ++q) {
          const double w = wave_sum(red[k][q]);
          if (lane == 0) pt[q] = 0.0 + w;
        }
      } else {
        block_reduce_store(a.red, nv, red[k], sl[k], part, nparts);
      }
    }
  }
}

// Contiguous mapping: one block per (tile of kBlock consecutive sites, group
// of NS slots); the blocks of each XCD cover a contiguous range of tiles with
// all slot groups of a tile next to each other, so the groups share its links
// in L2.
template <int P, int EPI, int RED, int NS, bool DAG>
__global__ void __launch_bounds__(kBlock) hop_kernel(HopArgs a) {
  const int ngroups = (a.nslots + NS - 1) / NS;
  const int f = xcd_tile(blockIdx.x, gridDim.x);
  const int tile = f / ngroups, grp = f - tile * ngroups;
  const int i = tile * kBlock + threadIdx.x;
  site_work<P, EPI, RED, NS, false, DAG>(a, grp, i, i < a.g.Vh, tile, gridDim.x / ngroups);
}

// Slab mapping: every XCD owns a fixed range of 64-site chunks of each
// timeslice (a spatial slab) and sweeps the timeslices in order, one wave per
// block; the x0 -+ 1 neighbour spinors of all slots then stay in that XCD's L2
// (about 3 timeslices of its slab).  Block b runs on XCD b mod 8.
struct SlabMap {
  int nch, maxc, ngroups, order;
  int tmap, tlen;  // time mapping (see time_item) and the longest XCD time range
};

__device__ __forceinline__ int slab_lo(int nch, int xcd) { return (nch * xcd) >> 3; }

// Time mapping (tmap = 1): XCD k owns the timeslices [T k / 8, T (k+1) / 8)
// of every chunk instead of a spatial slab of every timeslice, and takes
// its (chunk, timeslice) items chunk by chunk, the timeslices innermost.
// Block j of an XCD (after the slot groups, slab kernel) is timeslice
// j mod tlen of its range and chunk j / tlen; blocks past the range or the
// last chunk own nothing.  The reduction partial of an item is x0 nch +
// chunk (nparts = T nch), the same in both kernels and in the slab mapping.
struct Item {
  int chunk, x0, part;
  bool in;
};
__device__ __forceinline__ Item time_item(const SlabMap& m, int T, int xcd, int j, bool backwards) {
  Item it;
  const int lo = (T * xcd) >> 3, hi = (T * (xcd + 1)) >> 3;
  const int dt = j % m.tlen;
  it.chunk = j / m.tlen;
  it.in = lo + dt < hi && it.chunk < m.nch;
  it.x0 = backwards ? hi - 1 - dt : lo + dt;
  it.part = it.x0 * m.nch + it.chunk;
  return it;
}

// No minimum-waves hint: measured on MI355X at 24^3x48 with 12 slots, asking
// for 3 waves per SIMD in FP32 (two slots per thread) or 4 in FP16 makes the
// compiler spill and the kernels slower.
template <int P, int EPI, int RED, int NS, bool NT, bool DAG>
__global__ void __launch_bounds__(64) hop_kernel_slab(HopArgs a, SlabMap m) {
  const int xcd = blockIdx.x & 7;
  int j = blockIdx.x >> 3;
  if (m.tmap) {
    const int grp = j % m.ngroups;
    const Item it = time_item(m, a.g.T, xcd, j / m.ngroups, EPI == EPI_DIAG);
    if (!it.in) return;  // owns no partial
    const int sp = it.chunk * 64 + threadIdx.x;
    const bool valid = sp < a.g.Vsh;
    site_work<P, EPI, RED, NS, NT, DAG>(a, grp, valid ? it.x0 * a.g.Vsh + sp : 0, valid, it.part, a.g.T * m.nch);
    return;
  }
  int grp, cl, x0;
  if (m.order == 0) {  // slot groups of a chunk together, then chunks, then timeslices
    grp = j % m.ngroups;
    j /= m.ngroups;
    cl = j % m.maxc;
    x0 = j / m.maxc;
  } else if (m.order == 1) {  // chunks, then slot groups, then timeslices
    cl = j % m.maxc;
    j /= m.maxc;
    grp = j % m.ngroups;
    x0 = j / m.ngroups;
  } else {  // chunks, then timeslices, then slot groups
    cl = j % m.maxc;
    j /= m.maxc;
    x0 = j % a.g.T;
    grp = j / a.g.T;
  }
  // the even-site kernel sweeps the timeslices backwards, as in the
  // shared-tile kernel (measured on MI355X: 2% on the 12-slot FP16 kernel)
  if constexpr (EPI == EPI_DIAG) x0 = a.g.T - 1 - x0;
  const int chunk = slab_lo(m.nch, xcd) + cl;
  if (chunk >= slab_lo(m.nch, xcd + 1)) return;  // past the slab: owns no partial
  const int sp = chunk * 64 + threadIdx.x;
  const bool valid = sp < a.g.Vsh;
  const int i = valid ? x0 * a.g.Vsh + sp : 0;
  site_work<P, EPI, RED, NS, NT, DAG>(a, grp, i, valid, x0 * m.nch + chunk, a.g.T * m.nch);
}

// Shared-tile mapping: the slab mapping's (XCD chunk, timeslice) with every
// slot group in one workgroup (one wave per group).  The links of the chunk's
// 64 sites in the 8 hop directions (and the clover blocks of the even-site
// epilogue, or the A^-1 blocks of the odd-site ones when all slots share one
// mass) are loaded once into LDS, converted to the arithmetic precision,
// instead of once per slot group.  Per-slot arithmetic and reduction
// partials are those of the slab mapping.
template <int P>
constexpr size_t shared_tile_bytes(bool clover) {
  using R = typename Tr<P>::R;
  return 8 * 9 * 64 * sizeof(cx<R>) + (clover ? 72 * 64 * sizeof(float) : 0);
}

// Workgroups of 4 waves at two waves per SIMD (up to 256 registers per lane:
// the batched neighbour loads hold four spinors and links in flight), two
// workgroups per CU (the LDS tile takes 55 KB); each wave takes slot groups
// wv, wv + nw, ...  Measured on MI355X at 24^3x48 with 12 slots (FP32): three
// waves per SIMD (two batched neighbours, at most 168 registers) in 12-, 6-
// or 4-wave workgroups, one workgroup per CU, or eight neighbours in flight
// were all 1-35% slower.  The build knobs DP_SHARED_WG32 / DP_SHARED_MINW32
// set the FP32 workgroup size bound and the waves per SIMD.
#ifndef DP_SHARED_WG32
#define DP_SHARED_WG32 256
#endif
#ifndef DP_SHARED_MINW32
#define DP_SHARED_MINW32 2
#endif
template <int P>
constexpr int shared_max_threads(int red) {
  return P == F16 ? 256 : red == RED_TS4 ? 512 : DP_SHARED_WG32;
}
#ifndef DP_SHARED_MINW16
#define DP_SHARED_MINW16 2
#endif
template <int P>
constexpr int shared_min_waves(int red) {
  return P == F16 ? DP_SHARED_MINW16 : red == RED_TS4 ? 2 : DP_SHARED_MINW32;
}

// The staged links and blocks are read once per launch: streamed past L2
// (measured on MI355X at 24^3x48 with 12 slots: 2-3% faster).
constexpr bool kFillNT = true;

// LINV: the odd-site epilogue's A^-1, the same for every slot, is staged too.
template <int P, int EPI, int RED, int NS, bool NT, bool DAG, bool LINV>
__global__ void __launch_bounds__(shared_max_threads<P>(RED), shared_min_waves<P>(RED)) hop_kernel_shared(HopArgs a,
                                                                                                   SlabMap m) {
  using R = typename Tr<P>::R;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<R>* lu = reinterpret_cast<cx<R>*>(smem);
  float* lc = reinterpret_cast<float*>(smem + 8 * 9 * 64 * sizeof(cx<R>));
  const Geom& g = a.g;
  const int xcd = blockIdx.x & 7;
  const int j = blockIdx.x >> 3;
  // the even-site kernel sweeps the timeslices backwards: it reads the odd
  // field the preceding odd-site kernel wrote in forward order, whose last
  // timeslices are then still in the caches (measured on MI355X at 24^3x48
  // with 12 slots: 3% faster).  The reduction partials are indexed by x0, so
  // the sums do not depend on the order.
  int chunk, x0;
  if (m.tmap) {
    const Item it = time_item(m, g.T, xcd, j, EPI == EPI_DIAG);
    if (!it.in) return;  // the whole workgroup owns no partial (before any barrier)
    chunk = it.chunk;
    x0 = it.x0;
  } else {
    const int cl = j % m.maxc;
    x0 = EPI == EPI_DIAG ? g.T - 1 - j / m.maxc : j / m.maxc;
    chunk = slab_lo(m.nch, xcd) + cl;
    if (chunk >= slab_lo(m.nch, xcd + 1)) return;  // past the slab (before any barrier)
  }
  // one reduction partial per (timeslice, chunk), whatever the mapping
  const int part = x0 * m.nch + chunk, nparts = g.T * m.nch;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int sp = chunk * 64 + lane;
  const bool valid = sp < g.Vsh;
  const int i = valid ? x0 * g.Vsh + sp : 0;
  // fill: tasks 0..7 are the link directions (2 mu forward, 2 mu + 1 backward),
  // task 8 the clover blocks (even-site epilogue) or the A^-1 blocks all
  // slots share (odd-site epilogues); wave w takes tasks w, w + nw, ...
  constexpr bool blocks = shared_clover<P, EPI>() || LINV;
  if (valid) {
    int x[4];
    eo_coords(g, a.p, i, x[0], x[1], x[2], x[3]);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      if (t % nw != wv || (t == 8 && !blocks)) continue;
      if (t < 8) {
        const int mu = t >> 1;  // a constant once unrolled
        int li = i;  // forward hops: the link at the site; backward: at the neighbour
        if (t & 1) {
          int y[4] = {x[0], x[1], x[2], x[3]};
          const int L = mu == 0 ? g.T : mu == 1 ? g.L1 : mu == 2 ? g.L2 : g.L3;
          y[mu] = x[mu] == 0 ? L - 1 : x[mu] - 1;
          li = eo_index(g, y[0], y[1], y[2], y[3]);
        }
        cx<R> u[9];
        LinkIO<P>::template load<R, kFillNT>((t & 1) ? a.U_in : a.U_out, mu, li, g.Vp, u);
#pragma unroll
        for (int k = 0; k < 9; ++k) lu[(t * 9 + k) * 64 + lane] = u[k];
      } else {
        float r[72];
        const float sc =
            LINV ? CloverIO<P>::template load_raw<kFillNT>(a.slots.ainv_common, a.slots.ainv_common_scale, i, g.Vp, r)
                 : CloverIO<P>::template load_raw<kFillNT>(a.clov.data, a.clov.scale, i, g.Vp, r);
#pragma unroll
        for (int k = 0; k < 72; ++k) lc[k * 64 + lane] = P == F16 ? r[k] * sc : r[k];
      }
    }
  }
  __syncthreads();
#pragma unroll 1
  for (int grp = wv; grp < m.ngroups; grp += nw) {
    // keeps the compiler from hoisting the LDS reads out of this loop into
    // (many) registers
    asm volatile("" ::: "memory");
    site_work<P, EPI, RED, NS, NT, DAG, true, LINV>(a, grp, i, valid, part, nparts, lu, lc, lane);
  }
}

int env_knob(const char* name, int dflt) {
  const char* e = getenv(name);
  return e ? atoi(e) : dflt;
}

int hop_map_choice() {
  // tuning knob: DP_HOP_MAP = 0 contiguous tiles, 1 slabs swept along x0
  static const int v = env_knob("DP_HOP_MAP", -1);
  return v;
}

template <int P, int EPI, int RED, bool DAG>
hipError_t launch_ns(const HopArgs& a, int ntiles, hipStream_t st, int* nparts_out) {
  // slots per thread (measured on MI355X, 24^3x48 with 12 slots): two in
  // FP32, one in FP16 (the L2 keeps more neighbour spinors), one for the FP64
  // clover epilogue (it already fills the register file)
  int ns = P == F32 ? (a.nslots >= 2 ? 2 : 1) : 1;
  if (P == F64 && EPI != EPI_DIAG && a.nslots >= 2) ns = 2;
  // tuning knob: DP_HOP_NS in {1, 2} overrides the slots per thread (4 was
  // measured slower everywhere and is not built)
  static const int forced = [] {
    const char* e = getenv("DP_HOP_NS");
    const int v = e ? atoi(e) : 0;
    return (v == 1 || v == 2) ? v : 0;
  }();
  if (forced) ns = std::min(forced, a.nslots >= 2 ? 2 : 1);
  const int ngroups = (a.nslots + ns - 1) / ns;
  // The mapping fixes how the fused reductions are partitioned, so it must not
  // depend on the number of slots: a slot's result is then bitwise the same
  // alone and in any batch.  Slabs (measured on MI355X at 24^3x48: 5% faster
  // with 12 slots, 1-4% slower with one) are the default.
  const int map = hop_map_choice() >= 0 ? hop_map_choice() : 1;
  // the slab kernel streams the epilogue inputs and the output past L2
  // (non-temporal; measured on MI355X: 3% faster at 24^3x48 with 12 slots,
  // FP32); tuning knob: DP_HOP_NT = 0 turns that off
  static const bool nt = env_knob("DP_HOP_NT", 1) == 1;
  int nparts;
  if (map == 1) {
    SlabMap m;
    m.nch = (a.g.Vsh + 63) / 64;
    m.maxc = (m.nch + 7) / 8;
    m.ngroups = ngroups;
    // tuning knob: DP_HOP_ORDER in {0, 1, 2} (block order within an XCD)
    static const int order = std::min(2, std::max(0, env_knob("DP_HOP_ORDER", 0)));
    m.order = order;
    // XCD mapping: spatial slabs (tmap 0) or timeslice ranges (tmap 1,
    // time_item), chosen per launch; both give one reduction partial per
    // (timeslice, chunk), so the results are bitwise the same either way.
    // Measured on MI355X: timeslice ranges 2-6% faster for one FP32 or FP16
    // slot and for 12 FP16 slots at 24^3x48 and 32^3x64, slabs 6% faster for
    // 12 FP32 slots; FP64 keeps the slabs (one slot: 2% faster on timeslice
    // ranges at 24^3x48, 4-10% slower at 32^3x64).  Tuning knob:
    // DP_HOP_TMAP = 0 / 1 forces one of them.
    static const int tmap_knob = env_knob("DP_HOP_TMAP", -1);
    const int tmap = tmap_knob == 0 || tmap_knob == 1 ? tmap_knob
                                                      : (P != F64 && (a.nslots == 1 || P == F16) ? 1 : 0);
    m.tmap = tmap;
    m.tlen = (a.g.T + 7) / 8;
    nparts = a.g.T * m.nch;
    const int nblocks = tmap ? 8 * m.tlen * m.nch : 8 * a.g.T * m.maxc;  // blocks per slot group
    const dim3 grid(nblocks * ngroups);
    // tuning knob: DP_HOP_LDS = bytes of (unused) LDS per block, which caps the
    // blocks resident per CU (160 KB of LDS per CU) and so the sweep front
    static const int lds = std::min(65536, std::max(0, env_knob("DP_HOP_LDS", 0)));
    // Two or more slots in FP32 or FP16: the shared-tile kernel, one slot per
    // wave (measured on MI355X at 24^3x48 with 12 slots: FP32 16% faster
    // than the slab kernel with two slots per thread, FP16 12% faster on the
    // even sites).  Not for the FP16 reconstruction epilogue: at the
    // shared-tile kernel's two waves per SIMD it spills.  One slot: the slab kernel (a one-wave shared-tile
    // workgroup holds as much LDS as a full one, and the CUs would run one
    // wave each).  The library is built with contraction limited to single
    // expressions, so both kernels round alike and a slot's results are
    // bitwise the same alone and in any batch.  Tuning knob: DP_HOP_SHARED
    // = 0 keeps one workgroup per slot group.
    static const bool shared = env_knob("DP_HOP_SHARED", 1) == 1;
    constexpr bool shared_ok = P == F32 || (P == F16 && EPI != EPI_INV_SUB);
    if constexpr (shared_ok) {
      if (shared && nt && !forced && a.nslots >= 2) {
        m.ngroups = a.nslots;
        // waves per workgroup: the fewest passes of at most the bound's
        // waves (four by default; the RED_TS4 kernel four of its eight).
        // Tuning knobs: DP_HOP_MAXW, DP_HOP_TS4_WAVES.
        static const int maxw_ts4 = std::min(8, std::max(1, env_knob("DP_HOP_TS4_WAVES", 4)));
        // tuning knob: DP_HOP_SHARED_LDS = bytes of (unused) LDS added per
        // workgroup, which caps the workgroups resident per CU
        static const int lds_extra = std::min(65536, std::max(0, env_knob("DP_HOP_SHARED_LDS", 0)));
        static const int maxw_other =
            std::min(shared_max_threads<P>(RED) / 64, std::max(1, env_knob("DP_HOP_MAXW", 12)));
        const int maxw = P == F16 ? shared_max_threads<P>(RED) / 64 : RED == RED_TS4 ? maxw_ts4 : maxw_other;
        const int passes = (a.nslots + maxw - 1) / maxw;
        const dim3 sgrid(nblocks), sblock(64 * ((a.nslots + passes - 1) / passes));
        constexpr bool inv = EPI == EPI_INV || EPI == EPI_INV_SUB;
        if (inv && a.slots.ainv_common)
          hipLaunchKernelGGL((hop_kernel_shared<P, EPI, RED, 1, true, DAG, inv>), sgrid, sblock,
                             shared_tile_bytes<P>(true) + lds_extra, st, a, m);
        else
          hipLaunchKernelGGL((hop_kernel_shared<P, EPI, RED, 1, true, DAG, false>), sgrid, sblock,
                             shared_tile_bytes<P>(shared_clover<P, EPI>()) + lds_extra, st, a, m);
        *nparts_out = nparts;
        return hipGetLastError();
      }
    }
    if (nt) {
      switch (ns) {
        case 2: hipLaunchKernelGGL((hop_kernel_slab<P, EPI, RED, 2, true, DAG>), grid, dim3(64), lds, st, a, m); break;
        default: hipLaunchKernelGGL((hop_kernel_slab<P, EPI, RED, 1, true, DAG>), grid, dim3(64), lds, st, a, m); break;
      }
    } else {
      switch (ns) {
        case 2: hipLaunchKernelGGL((hop_kernel_slab<P, EPI, RED, 2, false, DAG>), grid, dim3(64), lds, st, a, m); break;
        default: hipLaunchKernelGGL((hop_kernel_slab<P, EPI, RED, 1, false, DAG>), grid, dim3(64), lds, st, a, m); break;
      }
    }
  } else {
    nparts = ntiles;
    const dim3 grid(ntiles * ngroups);
    switch (ns) {
      case 2: hipLaunchKernelGGL((hop_kernel<P, EPI, RED, 2, DAG>), grid, dim3(kBlock), 0, st, a); break;
      default: hipLaunchKernelGGL((hop_kernel<P, EPI, RED, 1, DAG>), grid, dim3(kBlock), 0, st, a); break;
    }
  }
  *nparts_out = nparts;
  return hipGetLastError();
}

template <int P, bool DAG>
hipError_t launch_epi(const HopArgs& a, int ntiles, hipStream_t st, int* np) {
  // fused reductions are only used with the even-site Schur epilogue
  if (a.red.red != RED_NONE && a.epi != EPI_DIAG) return hipErrorInvalidValue;
  switch (a.epi) {
    case EPI_HOP: return launch_ns<P, EPI_HOP, RED_NONE, DAG>(a, ntiles, st, np);
    case EPI_INV: return launch_ns<P, EPI_INV, RED_NONE, DAG>(a, ntiles, st, np);
    case EPI_SUB: return launch_ns<P, EPI_SUB, RED_NONE, DAG>(a, ntiles, st, np);
    case EPI_INV_SUB: return launch_ns<P, EPI_INV_SUB, RED_NONE, DAG>(a, ntiles, st, np);
    case EPI_DIAG:
      switch (a.red.red) {
        case RED_NONE: return launch_ns<P, EPI_DIAG, RED_NONE, DAG>(a, ntiles, st, np);
        // the reductions with the shadow residual belong to BiCGStab, which
        // never applies the adjoint: those variants are not built
        case RED_DOT_EXT:
          if constexpr (DAG) return hipErrorInvalidValue;
          else return launch_ns<P, EPI_DIAG, RED_DOT_EXT, DAG>(a, ntiles, st, np);
        case RED_TS: return launch_ns<P, EPI_DIAG, RED_TS, DAG>(a, ntiles, st, np);
        case RED_NORM: return launch_ns<P, EPI_DIAG, RED_NORM, DAG>(a, ntiles, st, np);
        case RED_TS4:
          if constexpr (DAG) return hipErrorInvalidValue;
          else return launch_ns<P, EPI_DIAG, RED_TS4, DAG>(a, ntiles, st, np);
        default: return hipErrorInvalidValue;
      }
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int reduction_blocks(const Geom& g) { return (g.Vh + kBlock - 1) / kBlock; }

int hop_blocks(const Geom& g) {
  const int nch = (g.Vsh + 63) / 64;
  return std::max(reduction_blocks(g), 8 * g.T * ((nch + 7) / 8));
}

hipError_t launch_hop(const HopArgs& a, hipStream_t st, int* nparts) {
  *nparts = 0;
  if (a.nslots <= 0 || a.g.Vh <= 0) return hipErrorInvalidValue;
  if (a.in.prec != a.out.prec || a.link_prec != a.in.prec) return hipErrorInvalidValue;
  const int ntiles = reduction_blocks(a.g);
  switch (a.in.prec) {
    case F64: return a.dag ? launch_epi<F64, true>(a, ntiles, st, nparts) : launch_epi<F64, false>(a, ntiles, st, nparts);
    case F32: return a.dag ? launch_epi<F32, true>(a, ntiles, st, nparts) : launch_epi<F32, false>(a, ntiles, st, nparts);
    case F16: return a.dag ? launch_epi<F16, true>(a, ntiles, st, nparts) : launch_epi<F16, false>(a, ntiles, st, nparts);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dp
