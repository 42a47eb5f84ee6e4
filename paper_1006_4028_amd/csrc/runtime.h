// Host runtime of libdp: device buffers, the context, and the batched solver.
#pragma once
#include <map>
#include <string>
#include <vector>

#include "../../include/dp.h"
#include "dp_common.h"

namespace dp {

// Owned device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // grow to at least n bytes (contents not preserved)
  hipError_t reserve(size_t n) {
    if (n <= bytes) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    bytes = n;
    return hipSuccess;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// Pinned host staging buffer.
struct HostBuf {
  void* p = nullptr;
  size_t bytes = 0;
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
  hipError_t reserve(size_t n) {
    if (n <= bytes) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipHostMalloc(&p, n, hipHostMallocDefault);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// A spinor field of one parity for nslots slots in one precision.
struct Field {
  DevBuf data, scale;
  int prec = F64;
  int nslots = 0;
  long slot_stride = 0, scale_stride = 0;
  hipError_t alloc(const Geom& g, int prec_, int nslots_);
  SpinorRef ref() const {
    SpinorRef r;
    r.data = data.p;
    r.scale = scale.as<float>();
    r.slot_stride = slot_stride;
    r.scale_stride = scale_stride;
    r.prec = prec;
    return r;
  }
};

// A per-mass inverse clover A_oo^-1 = (C_oo + 4 + M)^-1 in every precision.
struct MassEntry {
  double M = 0.0;
  DevBuf a64, a32, a16, s16;
  bool have32 = false, have16 = false;
};

// Work space of the batched solver for nslots slots at one inner precision.
struct Workspace {
  int nslots = 0, prec = -1;
  // FP64
  Field eta_e, eta_o, b64, x64, r64, t64, to64;
  // inner precision (x in FP32 when the inner precision is FP16)
  Field r, rh, p, v, s, t, x, to;
  // per-slot device tables
  DevBuf ratio, m4, mask_all, mask_inner, mask_outer, ainv_ptr[3], ainv_scale_ptr, sc, partials, out_sums,
      slot_scale, x0src, alpha, cpp, sp_aos;
  HostBuf h_sc, h_sums, h_mask, h_scale;
};

}  // namespace dp

struct dp_ctx {
  int device = 0;
  int bc_t = -1;
  int dims[4] = {0, 0, 0, 0};
  dp::Geom g{};
  hipStream_t stream = nullptr;
  std::string err;

  // gauge field per precision and parity
  dp::DevBuf U[3][2];
  bool have_U[3] = {false, false, false};
  // mass-independent clover C, packed blocks, both parities, every precision
  dp::DevBuf C64[2], C32[2], C16[2], C16s[2];
  double csw = 0.0;
  int clover_kind = 0;  // 0: none (c_sw = 0), 1: built from links, 2: caller field
  std::vector<dp::MassEntry*> masses;

  double M = 0.0;
  std::vector<double> alpha;

  dp::Workspace ws;
  dp::DevBuf scratch_aos, bad_flag;

  // per-launch HIP-event timing of the library's kernels (dp_set_timing)
  struct KStat {
    long long launches = 0;
    double ms = 0.0, bytes = 0.0, flops = 0.0;
  };
  struct Pending {
    std::string name;
    double bytes, flops;
    hipEvent_t a, b;
  };
  bool timing = false;
  std::vector<hipEvent_t> ev_free;
  std::vector<Pending> pending;
  std::map<std::string, KStat> kstats;
  std::map<const void*, int> mask_count;  // active slots of each device mask

  ~dp_ctx();
};
