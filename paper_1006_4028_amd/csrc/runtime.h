// Host runtime of libdp: device buffers, the context, the batch of slots and
// the launch helpers shared by the translation units of the runtime.
#pragma once
#include <map>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/dp.h"
#include "dp_common.h"

namespace dp {

// Owned device allocation, or a view of memory owned elsewhere (view()).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = true;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p && owned) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // a view of n bytes at q (never freed here, never grown)
  void view(void* q, size_t n) {
    release();
    p = q;
    bytes = n;
    owned = false;
  }
  // grow to at least n bytes (contents not preserved)
  hipError_t reserve(size_t n) {
    if (n <= bytes) return hipSuccess;
    if (!owned) return hipErrorInvalidValue;  // a view cannot grow
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
  // reference starting at slot s0
  SpinorRef ref(int s0 = 0) const;
};

// A per-mass inverse clover A_oo^-1 = (C_oo + 4 + M)^-1 in every precision.
struct MassEntry {
  double M = 0.0;
  DevBuf a64, a32, a16, s16;
};

// Device work space of a set of slots at one inner precision.
// Work space of the SAP+GCR solver (csrc/sap.hip), created on first use.
struct SapState;
void sap_free(SapState* s);

struct Workspace {
  int nslots = 0, prec = -1;
  const double* sratio = nullptr;  // the ctx's spatial hop ratios these slots use
  // FP64: redefined source (both parities), Schur right-hand side, solution,
  // FP64 residual, Schur result, odd temporary / odd solution
  Field eta_e, eta_o, b64, x64, r64, t64, to64;
  // inner precision (x in FP32 when the inner precision is FP16)
  Field r, rh, p, v, s, t, x, to;
  // per-slot device tables
  DevBuf ratio, m4, mask_inner, mask_outer, ainv_ptr[3], ainv_scale_ptr, sc, partials, out_sums, slot_scale, x0src,
      alpha, cpp;
  HostBuf h_sc, h_sums, h_mask, h_scale;
  // host copy of the slots' A_oo^-1 fields per precision and FP16 scales
  std::vector<const void*> h_ainv[3];
  std::vector<const float*> h_ainv_scale;
  size_t device_bytes() const;
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
  // Schroedinger functional (dp_set_gauge_sf): the links of the lattice padded
  // with the two boundary timeslices (host layout, FP64, on the device) and
  // the coefficient of the fermion boundary counterterm
  bool sf = false;
  double ct_tilde = 1.0;
  dp::DevBuf sf_ext;
  std::vector<dp::MassEntry*> masses;
  int open_batches = 0;

  double M = 0.0;
  std::vector<double> alpha;
  // spatial profiles a_1, a_2, a_3 of the light-quark factorisation: two
  // variants on the device (0: ones, 1: the current ones), each 4 S ratios
  // (HopArgs::sratio layout) followed by the S profile values, S = L1+L2+L3
  dp::DevBuf space;
  bool has_space = false;

  dp::Workspace ws_apply;           // for dp_apply / dp_apply_dev
  // dp_apply_dev_noalloc: views into this device's static scratch array and a
  // host staging area sized at creation
  void* scratch_dev = nullptr;
  dp::Workspace ws_noalloc;
  std::vector<double> na_host;
  std::vector<double> apply_key;    // what ws_apply's per-slot tables were built for
  dp_batch* solve_batch = nullptr;  // reused by dp_solve
  dp::SapState* sap = nullptr;      // dp_solve_sap
  dp::DevBuf scratch_aos, bad_flag;

  // per-launch HIP-event timing of the library's kernels (dp_set_timing)
  struct KStat {
    long long launches = 0;
    double ms = 0.0, bytes = 0.0, flops = 0.0;
    std::vector<float> samples;  // the first kMaxSamples launch durations
  };
  static constexpr size_t kMaxSamples = 1 << 16;
  struct Pending {
    std::string name;
    double bytes, flops;
    hipEvent_t a, b;
  };
  bool timing = false;
  bool use_graphs = true;
  std::vector<hipEvent_t> ev_free;
  std::vector<Pending> pending;
  std::map<std::string, KStat> kstats;
  std::map<const void*, int> mask_count;  // active slots of each device mask (host view)

  ~dp_ctx();
};

struct dp_batch {
  dp_ctx* c = nullptr;
  int nslots = 0, prec = 0, solver = 0;
  int api_prec = 0;     // the DP_PREC_* the batch was opened with
  bool single = false;  // DP_PREC_F32_SINGLE: one inner solve, no FP64 defect correction
  dp::Workspace w;
  enum { FREE = 0, RUNNING = 1, DONE = 2 };
  struct Slot {
    int state = FREE;
    long long tag = 0;
    void* S_dev = nullptr;
    dp::MassEntry* me = nullptr;
    std::vector<double> alpha;
    double r = 0.0, delta = 0.0;
    int max_iter = 0, x0 = 0;
    double eta2 = 0.0, res2 = 0.0, scale = 0.0;
    int iters = 0, outer = 0, restarts = 0, hops = 0, status = DP_OK;
    int last_left = 0;  // why the last inner solve ended (SlotScalars::left)
    int stall = 0;      // breakdowns in a row that left the FP64 residual where it was
    bool in_inner = false, has_inner = false;
    double t_admit = 0.0, t_done = 0.0;
    std::vector<double> cpp;
  };
  std::vector<Slot> slots;
  std::vector<int> m_inner, m_outer;  // host copies of the device masks
  std::vector<int> done_order;        // finished slots in completion order
  // captured k-iteration graph
  hipGraphExec_t graph = nullptr;
  int graph_k = 0;
  const void* graph_ainv = nullptr;  // the shared A_oo^-1 the graph's launches were captured with
  ~dp_batch();
};

namespace dp {
namespace rt {

int fail(dp_ctx* c, int code, const char* msg);
int hip_fail(dp_ctx* c, hipError_t e, const char* expr, int line);

#define DP_HIP(c, expr)                                                      \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) return dp::rt::hip_fail((c), e_, #expr, __LINE__); \
  } while (0)

#define DP_TRY(expr)              \
  do {                            \
    int rc_ = (expr);             \
    if (rc_ != DP_OK) return rc_; \
  } while (0)

// A named roctx range over a scope: the library's phases (solve, inner
// iterations, outer step, SAP application) appear in rocprofv3
// --marker-trace beside the kernels; without a tracer the calls do nothing.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

bool env_pad();
double now_s();
void ratio_tables(int T, int bc_t, const double* alpha, double* out);
int mass_entry(dp_ctx* c, double M, MassEntry** out);
int ensure_ws(dp_ctx* c, Workspace& w, int nslots, int prec);
int h2d(dp_ctx* c, void* dst, const void* src, size_t bytes);
int upload_mask(dp_ctx* c, Workspace& w, DevBuf& dst, const std::vector<int>& m, int staging);
int timing_harvest(dp_ctx* c);
// spatial tables of the light-quark factorisation (see dp_ctx::space)
int upload_space(dp_ctx* c, const double* const a[3]);
const double* space_ratios(dp_ctx* c, int variant);
const double* space_profile(dp_ctx* c);     // nullptr without spatial profiles
const double* space_hop_ratios(dp_ctx* c);  // nullptr without spatial profiles
SlotTable slot_table(Workspace& w, int T, int s0, int prec, const int* mask);
// the A_oo^-1 field (and FP16 scale) shared by the slots [s0, s0 + n) in
// precision prec, or null when their masses differ
const void* common_ainv(const Workspace& w, int s0, int n, int prec, const float** scale);

// launch helpers over slots [s0, s0 + n) of a workspace
int hop(dp_ctx* c, Workspace& w, int s0, int n, int prec, int p, int dag, int epi, double sign, const Field& in,
        const Field& out, const Field* xin, const int* mask, int red = RED_NONE, int fin = FIN_NONE,
        const Field* wv = nullptr, int* inner_mask = nullptr);
int blas(dp_ctx* c, Workspace& w, int s0, int n, int op, int prec, const int* mask,
         std::initializer_list<const Field*> v, int fin = FIN_NONE, int* inner_mask = nullptr);
// Schur operator Mhat' in -> out (even sites), to = odd temporary
int schur(dp_ctx* c, Workspace& w, int s0, int n, int prec, int dag, const Field& in, const Field& to,
          const Field& out, const int* mask, int red, int fin, const Field* wv = nullptr, int* inner_mask = nullptr);

}  // namespace rt
}  // namespace dp
