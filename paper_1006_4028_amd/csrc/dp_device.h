// Device-side helpers: complex arithmetic, field loads/stores per storage
// format, geometry, and the fused block reduction with its finalisers.
#pragma once
#include "dp_common.h"

namespace dp {

template <typename R>
struct cx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.x, s * a.y}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// conj(a) * b
template <typename R>
__device__ __forceinline__ cx<R> cjmul(cx<R> a, cx<R> b) { return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }
// i * a
template <typename R>
__device__ __forceinline__ cx<R> ti(cx<R> a) { return {-a.y, a.x}; }
// a += b * c
template <typename R>
__device__ __forceinline__ void cfma(cx<R>& a, cx<R> b, cx<R> c) {
  a.x += b.x * c.x - b.y * c.y;
  a.y += b.x * c.y + b.y * c.x;
}
// a += conj(b) * c
template <typename R>
__device__ __forceinline__ void cjfma(cx<R>& a, cx<R> b, cx<R> c) {
  a.x += b.x * c.x + b.y * c.y;
  a.y += b.x * c.y - b.y * c.x;
}

template <int P>
struct Tr;
template <>
struct Tr<F64> {
  using R = double;
};
template <>
struct Tr<F32> {
  using R = float;
};
template <>
struct Tr<F16> {
  using R = float;
};

// ------------------------------------------------------------ geometry

__device__ __forceinline__ void eo_coords(const Geom& g, int p, int i, int& x0, int& x1, int& x2, int& x3) {
  x0 = i / g.Vsh;
  const int r = i - x0 * g.Vsh;
  const int t = r / g.L3h;
  const int x3h = r - t * g.L3h;
  x1 = t / g.L2;
  x2 = t - x1 * g.L2;
  x3 = 2 * x3h + ((p + x0 + x1 + x2) & 1);
}

__device__ __forceinline__ int eo_index(const Geom& g, int x0, int x1, int x2, int x3) {
  return (((x0 * g.L1 + x1) * g.L2 + x2) * g.L3 + x3) >> 1;
}

// Blocks are handed to the 8 XCDs round-robin; give each XCD a contiguous
// range of tiles so that neighbouring sites share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, k = b >> 3;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

// ------------------------------------------------------------ streamed access
//
// Loads and stores of data touched once per launch (the epilogue's inputs and
// the output) can be marked non-temporal, so that they do not displace the
// neighbour spinors and links that other sites of the sweep read again.

typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ float4 vld(const float4* p) {
  if constexpr (NT) {
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ double2 vld(const double2* p) {
  if constexpr (NT) {
    const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
    return make_double2(v.x, v.y);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ uint4 vld(const uint4* p) {
  if constexpr (NT) {
    const u4v v = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ float2 vld(const float2* p) {
  if constexpr (NT) {
    const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
    return make_float2(v.x, v.y);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ float vld(const float* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT>
__device__ __forceinline__ unsigned vld(const unsigned* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT>
__device__ __forceinline__ void vst(float4* p, float4 v) {
  if constexpr (NT) {
    const f4v w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<f4v*>(p));
  } else {
    *p = v;
  }
}
template <bool NT>
__device__ __forceinline__ void vst(double2* p, double2 v) {
  if constexpr (NT) {
    const d2v w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<d2v*>(p));
  } else {
    *p = v;
  }
}
template <bool NT>
__device__ __forceinline__ void vst(uint4* p, uint4 v) {
  if constexpr (NT) {
    const u4v w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<u4v*>(p));
  } else {
    *p = v;
  }
}
template <bool NT>
__device__ __forceinline__ void vst(float* p, float v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// ------------------------------------------------------------ spinors

template <int P>
struct SpinorIO;

template <>
struct SpinorIO<F64> {
  // the components and the factor that multiplies them (1 without a scale)
  template <typename R>
  __device__ static __forceinline__ R load_unscaled(const SpinorRef& f, int slot, int i, int Vh, cx<R> (&s)[12]) {
    load(f, slot, i, Vh, s);
    return R(1);
  }
  template <bool NT = false, typename R>
  __device__ static __forceinline__ void load(const SpinorRef& f, int slot, int i, int Vh, cx<R> (&s)[12]) {
    const double2* b = static_cast<const double2*>(f.data) + (long)slot * f.slot_stride;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const double2 v = vld<NT>(b + (long)c * Vh + i);
      s[c] = cx<R>{(R)v.x, (R)v.y};
    }
  }
  template <bool NT = false, typename R>
  __device__ static __forceinline__ void store(const SpinorRef& f, int slot, int i, int Vh, const cx<R> (&s)[12]) {
    double2* b = static_cast<double2*>(f.data) + (long)slot * f.slot_stride;
#pragma unroll
    for (int c = 0; c < 12; ++c) vst<NT>(b + (long)c * Vh + i, make_double2((double)s[c].x, (double)s[c].y));
  }
};

template <>
struct SpinorIO<F32> {
  template <typename R>
  __device__ static __forceinline__ R load_unscaled(const SpinorRef& f, int slot, int i, int Vh, cx<R> (&s)[12]) {
    load(f, slot, i, Vh, s);
    return R(1);
  }
  template <bool NT = false, typename R>
  __device__ static __forceinline__ void load(const SpinorRef& f, int slot, int i, int Vh, cx<R> (&s)[12]) {
    const float4* b = static_cast<const float4*>(f.data) + (long)slot * f.slot_stride;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const float4 v = vld<NT>(b + (long)k * Vh + i);
      s[2 * k] = cx<R>{(R)v.x, (R)v.y};
      s[2 * k + 1] = cx<R>{(R)v.z, (R)v.w};
    }
  }
  template <bool NT = false, typename R>
  __device__ static __forceinline__ void store(const SpinorRef& f, int slot, int i, int Vh, const cx<R> (&s)[12]) {
    float4* b = static_cast<float4*>(f.data) + (long)slot * f.slot_stride;
#pragma unroll
    for (int k = 0; k < 6; ++k)
      vst<NT>(b + (long)k * Vh + i, make_float4((float)s[2 * k].x, (float)s[2 * k].y, (float)s[2 * k + 1].x,
                                               (float)s[2 * k + 1].y));
  }
};

__device__ __forceinline__ float2 h2f(unsigned u) {
  __half2 h = *reinterpret_cast<__half2*>(&u);
  return __half22float2(h);
}
__device__ __forceinline__ unsigned f2h(float a, float b) {
  __half2 h = __floats2half2_rn(a, b);
  return *reinterpret_cast<unsigned*>(&h);
}

template <>
struct SpinorIO<F16> {
  // the stored binary16 values (|v| <= 1) and the site's scale
  template <typename R>
  __device__ static __forceinline__ R load_unscaled(const SpinorRef& f, int slot, int i, int Vh, cx<R> (&s)[12]) {
    const uint4* b = static_cast<const uint4*>(f.data) + (long)slot * f.slot_stride;
    const float sc = f.scale[(long)slot * f.scale_stride + i];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint4 v = b[(long)k * Vh + i];
      const float2 a0 = h2f(v.x), a1 = h2f(v.y), a2 = h2f(v.z), a3 = h2f(v.w);
      s[4 * k + 0] = cx<R>{(R)a0.x, (R)a0.y};
      s[4 * k + 1] = cx<R>{(R)a1.x, (R)a1.y};
      s[4 * k + 2] = cx<R>{(R)a2.x, (R)a2.y};
      s[4 * k + 3] = cx<R>{(R)a3.x, (R)a3.y};
    }
    return (R)sc;
  }
  template <bool NT = false, typename R>
  __device__ static __forceinline__ void load(const SpinorRef& f, int slot, int i, int Vh, cx<R> (&s)[12]) {
    const uint4* b = static_cast<const uint4*>(f.data) + (long)slot * f.slot_stride;
    const float sc = vld<NT>(f.scale + (long)slot * f.scale_stride + i);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint4 v = vld<NT>(b + (long)k * Vh + i);
      float2 a0 = h2f(v.x), a1 = h2f(v.y), a2 = h2f(v.z), a3 = h2f(v.w);
      s[4 * k + 0] = cx<R>{(R)(a0.x * sc), (R)(a0.y * sc)};
      s[4 * k + 1] = cx<R>{(R)(a1.x * sc), (R)(a1.y * sc)};
      s[4 * k + 2] = cx<R>{(R)(a2.x * sc), (R)(a2.y * sc)};
      s[4 * k + 3] = cx<R>{(R)(a3.x * sc), (R)(a3.y * sc)};
    }
  }
  template <bool NT = false, typename R>
  __device__ static __forceinline__ void store(const SpinorRef& f, int slot, int i, int Vh, const cx<R> (&s)[12]) {
    cx<R> unused[12];
    store_decoded<NT, false>(f, slot, i, Vh, s, unused);
  }
  // store, and (DEC) return in q what load() will read back
  template <bool NT, bool DEC, typename R>
  __device__ static __forceinline__ void store_decoded(const SpinorRef& f, int slot, int i, int Vh,
                                                       const cx<R> (&s)[12], cx<R> (&q)[12]) {
    uint4* b = static_cast<uint4*>(f.data) + (long)slot * f.slot_stride;
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf((float)s[c].x), fabsf((float)s[c].y)));
    // A site whose largest component is below the smallest normal float is
    // stored as zero: 1/m would overflow to Inf (and 0 * Inf is NaN).  Such
    // sites arise from rounding residues of cancellations, which shrink by
    // about the FP32 epsilon at every application of the operator; the
    // solvers' fields are normalised to O(1), so dropping them is exact to
    // far below the FP16 resolution.
    if (!(m >= 1.17549435e-38f)) m = 0.f;  // FLT_MIN
    const float inv = m > 0.f ? 1.0f / m : 0.f;
    vst<NT>(f.scale + (long)slot * f.scale_stride + i, m);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint4 v;
      v.x = f2h((float)s[4 * k + 0].x * inv, (float)s[4 * k + 0].y * inv);
      v.y = f2h((float)s[4 * k + 1].x * inv, (float)s[4 * k + 1].y * inv);
      v.z = f2h((float)s[4 * k + 2].x * inv, (float)s[4 * k + 2].y * inv);
      v.w = f2h((float)s[4 * k + 3].x * inv, (float)s[4 * k + 3].y * inv);
      vst<NT>(b + (long)k * Vh + i, v);
      if constexpr (DEC) {
        const float2 a0 = h2f(v.x), a1 = h2f(v.y), a2 = h2f(v.z), a3 = h2f(v.w);
        q[4 * k + 0] = cx<R>{(R)(a0.x * m), (R)(a0.y * m)};
        q[4 * k + 1] = cx<R>{(R)(a1.x * m), (R)(a1.y * m)};
        q[4 * k + 2] = cx<R>{(R)(a2.x * m), (R)(a2.y * m)};
        q[4 * k + 3] = cx<R>{(R)(a3.x * m), (R)(a3.y * m)};
      }
    }
  }
};

// ------------------------------------------------------------ raw spinors
//
// A neighbour spinor as stored (no conversion), so that the loads of several
// neighbours can be issued before the first is used; decode() converts it
// and returns the factor its components carry (the FP16 per-site scale, else 1).

template <int P>
struct RawSpinor;
template <>
struct RawSpinor<F64> {
  double2 v[12];
};
template <>
struct RawSpinor<F32> {
  float4 v[6];
};
template <>
struct RawSpinor<F16> {
  uint4 v[3];
  float sc;
};

template <int P>
__device__ __forceinline__ void load_raw_spinor(const SpinorRef& f, int slot, int i, int Vh, RawSpinor<P>& r) {
  if constexpr (P == F64) {
    const double2* b = static_cast<const double2*>(f.data) + (long)slot * f.slot_stride;
#pragma unroll
    for (int c = 0; c < 12; ++c) r.v[c] = b[(long)c * Vh + i];
  } else if constexpr (P == F32) {
    const float4* b = static_cast<const float4*>(f.data) + (long)slot * f.slot_stride;
#pragma unroll
    for (int k = 0; k < 6; ++k) r.v[k] = b[(long)k * Vh + i];
  } else {
    const uint4* b = static_cast<const uint4*>(f.data) + (long)slot * f.slot_stride;
#pragma unroll
    for (int k = 0; k < 3; ++k) r.v[k] = b[(long)k * Vh + i];
    r.sc = f.scale[(long)slot * f.scale_stride + i];
  }
}

// the same values and factor SpinorIO<P>::load_unscaled gives
template <int P, typename R>
__device__ __forceinline__ R decode_spinor(const RawSpinor<P>& r, cx<R> (&s)[12]) {
  if constexpr (P == F64) {
#pragma unroll
    for (int c = 0; c < 12; ++c) s[c] = cx<R>{(R)r.v[c].x, (R)r.v[c].y};
    return R(1);
  } else if constexpr (P == F32) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      s[2 * k] = cx<R>{(R)r.v[k].x, (R)r.v[k].y};
      s[2 * k + 1] = cx<R>{(R)r.v[k].z, (R)r.v[k].w};
    }
    return R(1);
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float2 a0 = h2f(r.v[k].x), a1 = h2f(r.v[k].y), a2 = h2f(r.v[k].z), a3 = h2f(r.v[k].w);
      s[4 * k + 0] = cx<R>{(R)a0.x, (R)a0.y};
      s[4 * k + 1] = cx<R>{(R)a1.x, (R)a1.y};
      s[4 * k + 2] = cx<R>{(R)a2.x, (R)a2.y};
      s[4 * k + 3] = cx<R>{(R)a3.x, (R)a3.y};
    }
    return (R)r.sc;
  }
}

// ------------------------------------------------------------ links

template <int P>
struct LinkIO;
template <>
struct LinkIO<F64> {
  template <typename R, bool NT = false>
  __device__ static __forceinline__ void load(const void* base, int mu, int i, int Vh, cx<R> (&u)[9]) {
    const double2* b = static_cast<const double2*>(base) + (long)mu * 9 * Vh;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double2 v = vld<NT>(b + (long)k * Vh + i);
      u[k] = cx<R>{(R)v.x, (R)v.y};
    }
  }
};
template <>
struct LinkIO<F32> {
  template <typename R, bool NT = false>
  __device__ static __forceinline__ void load(const void* base, int mu, int i, int Vh, cx<R> (&u)[9]) {
    const float2* b = static_cast<const float2*>(base) + (long)mu * 9 * Vh;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float2 v = vld<NT>(b + (long)k * Vh + i);
      u[k] = cx<R>{(R)v.x, (R)v.y};
    }
  }
};
template <>
struct LinkIO<F16> {
  template <typename R, bool NT = false>
  __device__ static __forceinline__ void load(const void* base, int mu, int i, int Vh, cx<R> (&u)[9]) {
    const unsigned* b = static_cast<const unsigned*>(base) + (long)mu * 9 * Vh;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float2 v = h2f(vld<NT>(b + (long)k * Vh + i));
      u[k] = cx<R>{(R)v.x, (R)v.y};
    }
  }
};

// ------------------------------------------------------------ clover blocks
// Packed Hermitian 6x6: d[0..5] real diagonal, then o[k] for (i<j) row-major.

template <typename R>
struct HermBlock {
  R d[6];
  cx<R> o[15];
};

__host__ __device__ constexpr int herm_off(int i, int j) {  // i < j
  return i * 5 - (i * (i - 1)) / 2 + (j - i - 1);
}

template <int P>
struct CloverIO;
template <>
struct CloverIO<F64> {
  template <typename R>
  __device__ static __forceinline__ void load(const void* base, const float*, int i, int Vh, HermBlock<R> (&B)[2]) {
    const double2* b = static_cast<const double2*>(base);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double2 v = b[(long)(h * 18 + k) * Vh + i];
        B[h].d[2 * k] = (R)v.x;
        B[h].d[2 * k + 1] = (R)v.y;
      }
#pragma unroll
      for (int k = 0; k < 15; ++k) {
        const double2 v = b[(long)(h * 18 + 3 + k) * Vh + i];
        B[h].o[k] = cx<R>{(R)v.x, (R)v.y};
      }
    }
  }
};
// FP32 and FP16 blocks also load in two steps: the stored values as floats
// (with the FP16 per-site scale; 1 for FP32), then the block assembled from
// them.  A copy of the raw values (in LDS) assembled the same way gives
// bitwise the same block and the same arithmetic after it.
template <>
struct CloverIO<F32> {
  template <bool NT = false>
  __device__ static __forceinline__ float load_raw(const void* base, const float*, int i, int Vh, float (&r)[72]) {
    const float4* b = static_cast<const float4*>(base);
#pragma unroll
    for (int k = 0; k < 18; ++k) {
      const float4 v = vld<NT>(b + (long)k * Vh + i);
      r[4 * k] = v.x; r[4 * k + 1] = v.y; r[4 * k + 2] = v.z; r[4 * k + 3] = v.w;
    }
    return 1.f;
  }
  template <typename R>
  __device__ static __forceinline__ void assemble(const float (&r)[72], float, HermBlock<R> (&B)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int k = 0; k < 6; ++k) B[h].d[k] = (R)r[36 * h + k];
#pragma unroll
      for (int k = 0; k < 15; ++k) B[h].o[k] = cx<R>{(R)r[36 * h + 6 + 2 * k], (R)r[36 * h + 7 + 2 * k]};
    }
  }
  template <typename R>
  __device__ static __forceinline__ void load(const void* base, const float* scale, int i, int Vh,
                                              HermBlock<R> (&B)[2]) {
    float r[72];
    const float sc = load_raw(base, scale, i, Vh, r);
    assemble(r, sc, B);
  }
};
template <>
struct CloverIO<F16> {
  template <bool NT = false>
  __device__ static __forceinline__ float load_raw(const void* base, const float* scale, int i, int Vh,
                                                   float (&r)[72]) {
    const uint4* b = static_cast<const uint4*>(base);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const uint4 v = vld<NT>(b + (long)k * Vh + i);
      float2 a0 = h2f(v.x), a1 = h2f(v.y), a2 = h2f(v.z), a3 = h2f(v.w);
      r[8 * k + 0] = a0.x; r[8 * k + 1] = a0.y; r[8 * k + 2] = a1.x; r[8 * k + 3] = a1.y;
      r[8 * k + 4] = a2.x; r[8 * k + 5] = a2.y; r[8 * k + 6] = a3.x; r[8 * k + 7] = a3.y;
    }
    return vld<NT>(scale + i);
  }
  template <typename R>
  __device__ static __forceinline__ void assemble(const float (&r)[72], float sc, HermBlock<R> (&B)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int k = 0; k < 6; ++k) B[h].d[k] = (R)(r[36 * h + k] * sc);
#pragma unroll
      for (int k = 0; k < 15; ++k)
        B[h].o[k] = cx<R>{(R)(r[36 * h + 6 + 2 * k] * sc), (R)(r[36 * h + 7 + 2 * k] * sc)};
    }
  }
  template <typename R>
  __device__ static __forceinline__ void load(const void* base, const float* scale, int i, int Vh,
                                              HermBlock<R> (&B)[2]) {
    float r[72];
    const float sc = load_raw(base, scale, i, Vh, r);
    assemble(r, sc, B);
  }
};

// y = (B + shift) x on one chirality block (components 6h .. 6h+5 of the spinor)
template <typename R>
__device__ __forceinline__ void herm_apply(const HermBlock<R>& B, R shift, const cx<R>* x, cx<R>* y) {
#pragma unroll
  for (int r = 0; r < 6; ++r) y[r] = (B.d[r] + shift) * x[r];
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r + 1; c < 6; ++c) {
      const cx<R> a = B.o[herm_off(r, c)];
      cfma(y[r], a, x[c]);   // A_rc x_c
      cjfma(y[c], a, x[r]);  // A_cr = conj(A_rc)
    }
}

// ------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// complex a / b
__device__ __forceinline__ void cdiv(const double* a, const double* b, double* out) {
  const double den = b[0] * b[0] + b[1] * b[1];
  const double re = (a[0] * b[0] + a[1] * b[1]) / den;
  const double im = (a[1] * b[0] - a[0] * b[1]) / den;
  out[0] = re;
  out[1] = im;
}

// End of an inner iteration: count it and take the slot out of the inner
// mask when it converged, broke down, ran out of iterations or went non-finite.
__device__ inline void end_of_iteration(const ReduceRef& red, int slot, SlotScalars& c) {
  c.iters++;
  int why = 0;
  if (!isfinite(c.rr)) why = 4;
  else if (c.breakdown) why = 2;
  else if (c.rr <= c.tol2) why = 1;
  else if (c.iters >= c.max_iter) why = 3;
  if (why) {
    c.left = why;
    if (red.inner_mask) red.inner_mask[slot] = 0;
  }
}

// Solver finalisers: turn the folded sums of one slot into its scalars.
__device__ inline void run_finaliser(const ReduceRef& red, int slot, const double (&s)[kRedMax]) {
  if (red.fin == FIN_STORE) {
    for (int k = 0; k < 4; ++k) red.out_sums[slot * 4 + k] = s[k];
    return;
  }
  SlotScalars& c = red.sc[slot];
  switch (red.fin) {
    case FIN_BICG_ALPHA: {
      if (s[0] == 0.0 && s[1] == 0.0) {
        c.breakdown = 2;
        c.alpha[0] = c.alpha[1] = 0.0;
        c.left = 2;
        c.iters++;  // counted, so that max_iter bounds a run of breakdowns
        if (red.inner_mask) red.inner_mask[slot] = 0;
      } else {
        cdiv(c.rho, s, c.alpha);
      }
      break;
    }
    case FIN_BICG_OMEGA: {
      if (s[2] > 0.0) {
        c.omega[0] = s[0] / s[2];
        c.omega[1] = s[1] / s[2];
      } else {
        c.omega[0] = c.omega[1] = 0.0;
      }
      break;
    }
    case FIN_BICG_RHO: {
      c.rr = s[2];
      const double mag = sqrt(s[0] * s[0] + s[1] * s[1]);
      if (!(mag > 1e-14 * sqrt(c.rh2 * s[2]))) c.breakdown = 1;
      if (c.omega[0] == 0.0 && c.omega[1] == 0.0) c.breakdown = 3;
      if (c.breakdown == 0) {
        double q[2], w[2];
        cdiv(s, c.rho, q);          // rho_new / rho
        cdiv(c.alpha, c.omega, w);  // alpha / omega
        c.beta[0] = q[0] * w[0] - q[1] * w[1];
        c.beta[1] = q[0] * w[1] + q[1] * w[0];
      } else {
        c.beta[0] = c.beta[1] = 0.0;
      }
      c.rho[0] = s[0];
      c.rho[1] = s[1];
      end_of_iteration(red, slot, c);
      break;
    }
    case FIN_BICG_OMEGA_RHO: {
      // omega = <t,s> / |t|^2, and the next rho = <rh, r> with r = s - omega t
      // (r itself is formed afterwards, in the same kernel as the next search
      // direction).  <rh, s> vanishes in exact arithmetic, but its measured
      // value keeps rho tied to the stored vectors: without it the recurrence
      // drifts and the FP32 solve stagnates (measured at 24^3x48).
      if (s[2] > 0.0) {
        c.omega[0] = s[0] / s[2];
        c.omega[1] = s[1] / s[2];
      } else {
        c.omega[0] = c.omega[1] = 0.0;
      }
      double rn[2];
      rn[0] = s[3] - (c.omega[0] * s[5] - c.omega[1] * s[6]);
      rn[1] = s[4] - (c.omega[0] * s[6] + c.omega[1] * s[5]);
      if (c.omega[0] == 0.0 && c.omega[1] == 0.0) c.breakdown = 3;
      if (c.breakdown == 0 && (c.rho[0] != 0.0 || c.rho[1] != 0.0)) {
        double q[2], w[2];
        cdiv(rn, c.rho, q);         // rho_new / rho
        cdiv(c.alpha, c.omega, w);  // alpha / omega
        c.beta[0] = q[0] * w[0] - q[1] * w[1];
        c.beta[1] = q[0] * w[1] + q[1] * w[0];
      } else {
        c.beta[0] = c.beta[1] = 0.0;
      }
      c.rho[0] = rn[0];
      c.rho[1] = rn[1];
      break;
    }
    case FIN_BICG_RR: {
      c.rr = s[0];
      const double mag = sqrt(c.rho[0] * c.rho[0] + c.rho[1] * c.rho[1]);
      if (!(mag > 1e-14 * sqrt(c.rh2 * s[0]))) c.breakdown = 1;
      end_of_iteration(red, slot, c);
      break;
    }
    case FIN_BICG_INIT: {
      c.rho[0] = s[1];
      c.rho[1] = s[2];
      c.rr = s[0];
      c.rh2 = s[3];
      c.alpha[0] = c.omega[0] = 1.0;
      c.alpha[1] = c.omega[1] = 0.0;
      c.beta[0] = c.beta[1] = 0.0;
      c.breakdown = 0;
      c.left = 0;
      break;
    }
    case FIN_CG_ALPHA:
      c.cg_a = s[0] > 0.0 ? c.zz / s[0] : 0.0;
      break;
    case FIN_CG_BETA:
      c.cg_b = c.zz > 0.0 ? s[0] / c.zz : 0.0;
      c.zz = s[0];
      end_of_iteration(red, slot, c);
      break;
    case FIN_CG_INIT:
      c.zz = s[0];
      c.breakdown = 0;
      c.left = 0;
      break;
    case FIN_RR:
      c.rr = s[0];
      break;
    default:
      break;
  }
}

// Sum nv values over the block (fixed tree) and store the block's partial
// for the slot.  A finalise kernel launched next on the same stream folds the
// partials in block order (deterministic for a fixed launch shape; a slot's
// result depends only on that slot's data).  Every thread of the block must
// call this (no early return before it).
__device__ inline void block_reduce_store(const ReduceRef& red, int nv, double (&v)[kRedMax], int slot, int block,
                                          int nblocks) {
  __shared__ double lds[kRedMax][kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < nv; ++k) {
    const double w = wave_sum(v[k]);
    if (lane == 0) lds[k][wid] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* part = red.partials + ((long)slot * nblocks + block) * kRedMax;
    const int nw = blockDim.x >> 6;  // blocks of 64 or kBlock threads
    for (int k = 0; k < nv; ++k) {
      double t = 0.0;
      for (int w = 0; w < nw; ++w) t += lds[k][w];
      part[k] = t;
    }
  }
  __syncthreads();
}

}  // namespace dp
