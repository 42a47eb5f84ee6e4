// Host runtime and C ABI of libdp.
//
// The solve follows the paper's procedure (field redefinition eq. redeft,
// preconditioned system eq. linsysprec, restoration) with these building
// blocks of our own:
//   * even-odd reduction: the Schur operator Mhat' = A_ee - H_eo A_oo^-1 H_oe
//     on the even sites (A = 4 + M + C, H the alpha-hop term), so that the
//     full residual of a solution reconstructed on the odd sites equals the
//     Schur residual;
//   * a precision ladder: an FP64 outer loop recomputes r = b - Mhat' x in
//     FP64 and checks the stopping rule (eq. stopping) on it; an inner Krylov
//     solve in FP64, FP32 or FP16 storage reduces the normalised residual by
//     delta; x += |r| e in FP64 (defect correction);
//   * slots: every right-hand side is a slot with its own scalars, masses and
//     alpha table on the device.  Slots enter and leave the inner solve
//     independently; the kernels of one iteration run for all slots in the
//     inner mask at once (links are shared through the caches).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "runtime.h"

using namespace dp;

namespace {

int fail(dp_ctx* c, int code, const char* msg) {
  if (c) c->err = msg;
  return code;
}

#define DP_HIP(c, expr)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      if (c) {                                                                                \
        char b_[256];                                                                         \
        snprintf(b_, sizeof b_, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                 __LINE__);                                                                   \
        (c)->err = b_;                                                                        \
      }                                                                                       \
      return e_ == hipErrorOutOfMemory ? DP_ERR_OOM : DP_ERR_DEVICE;                          \
    }                                                                                         \
  } while (0)

long storage_units_per_slot(const Geom& g, int prec) {
  // double2 x12, float4 x6 or uint4 x3 per site
  return (long)g.Vh * (prec == F64 ? 12 : prec == F32 ? 6 : 3);
}

}  // namespace

hipError_t Field::alloc(const Geom& g, int prec_, int nslots_) {
  prec = prec_;
  nslots = nslots_;
  slot_stride = storage_units_per_slot(g, prec);
  scale_stride = prec == F16 ? g.Vh : 0;
  hipError_t e = data.reserve((size_t)nslots * g.Vh * spinor_site_bytes(prec));
  if (e != hipSuccess) return e;
  if (prec == F16) e = scale.reserve((size_t)nslots * g.Vh * sizeof(float));
  return e;
}

dp_ctx::~dp_ctx() {
  for (auto& q : pending) {
    (void)hipEventDestroy(q.a);
    (void)hipEventDestroy(q.b);
  }
  for (auto e : ev_free) (void)hipEventDestroy(e);
  for (auto* m : masses) delete m;
  if (stream) (void)hipStreamDestroy(stream);
}

namespace {

// ------------------------------------------------------------- helpers

// ratio tables of the modified time hops for one alpha table:
//   fwd[x0] = s_f alpha(x0)/alpha(x0+1), bwd[x0] = s_b alpha(x0)/alpha(x0-1),
//   fwd_dag, bwd_dag the same for 1/alpha, with the fermion boundary sign s
//   at the wrap-around (the boundary rule eq. redeftbc in ratio form).
void ratio_tables(int T, int bc_t, const double* alpha, double* out) {
  for (int t = 0; t < T; ++t) {
    const int tp = (t + 1) % T, tm = (t - 1 + T) % T;
    const double sf = (t == T - 1) ? (double)bc_t : 1.0;
    const double sb = (t == 0) ? (double)bc_t : 1.0;
    out[t] = sf * alpha[t] / alpha[tp];
    out[T + t] = sb * alpha[t] / alpha[tm];
    out[2 * T + t] = sf * alpha[tp] / alpha[t];
    out[3 * T + t] = sb * alpha[tm] / alpha[t];
  }
}

int check_state(dp_ctx* c) {
  if (!c->have_U[F64]) return fail(c, DP_ERR_BAD_STATE, "gauge field not set");
  return DP_OK;
}

// Per-mass A_oo^-1 in every precision (cached per (field, clover, M)).
int mass_entry(dp_ctx* c, double M, MassEntry** out) {
  for (auto* m : c->masses)
    if (m->M == M) {
      *out = m;
      return DP_OK;
    }
  const Geom& g = c->g;
  auto* m = new (std::nothrow) MassEntry;
  if (!m) return fail(c, DP_ERR_OOM, "host allocation failed");
  m->M = M;
  const size_t n64 = (size_t)g.Vh * clover_site_bytes(F64);
  hipError_t e = m->a64.reserve(n64);
  if (e == hipSuccess) e = m->a32.reserve((size_t)g.Vh * clover_site_bytes(F32));
  if (e == hipSuccess) e = m->a16.reserve((size_t)g.Vh * clover_site_bytes(F16));
  if (e == hipSuccess) e = m->s16.reserve((size_t)g.Vh * sizeof(float));
  if (e != hipSuccess) {
    delete m;
    return fail(c, DP_ERR_OOM, "out of device memory for the inverse clover");
  }
  DP_HIP(c, c->bad_flag.reserve(sizeof(int)));
  DP_HIP(c, hipMemsetAsync(c->bad_flag.p, 0, sizeof(int), c->stream));
  DP_HIP(c, launch_clover_invert(g, c->C64[1].as<double2>(), 4.0 + M, m->a64.as<double2>(), c->bad_flag.as<int>(),
                                 c->stream));
  DP_HIP(c, launch_clover_convert(g, m->a64.as<double2>(), m->a32.p, nullptr, F32, c->stream));
  DP_HIP(c, launch_clover_convert(g, m->a64.as<double2>(), m->a16.p, m->s16.as<float>(), F16, c->stream));
  int bad = 0;
  DP_HIP(c, hipMemcpyAsync(&bad, c->bad_flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  if (bad) {
    delete m;
    return fail(c, DP_ERR_INVALID_ARG, "C + 4 + M is singular on some odd site");
  }
  c->masses.push_back(m);
  *out = m;
  return DP_OK;
}

void drop_masses(dp_ctx* c) {
  for (auto* m : c->masses) delete m;
  c->masses.clear();
}

// zero clover (c_sw = 0) in every precision
int clover_zero(dp_ctx* c) {
  const Geom& g = c->g;
  for (int p = 0; p < 2; ++p) {
    DP_HIP(c, c->C64[p].reserve((size_t)g.Vh * clover_site_bytes(F64)));
    DP_HIP(c, c->C32[p].reserve((size_t)g.Vh * clover_site_bytes(F32)));
    DP_HIP(c, c->C16[p].reserve((size_t)g.Vh * clover_site_bytes(F16)));
    DP_HIP(c, c->C16s[p].reserve((size_t)g.Vh * sizeof(float)));
    DP_HIP(c, hipMemsetAsync(c->C64[p].p, 0, c->C64[p].bytes, c->stream));
    DP_HIP(c, hipMemsetAsync(c->C32[p].p, 0, c->C32[p].bytes, c->stream));
    DP_HIP(c, hipMemsetAsync(c->C16[p].p, 0, c->C16[p].bytes, c->stream));
    DP_HIP(c, hipMemsetAsync(c->C16s[p].p, 0, c->C16s[p].bytes, c->stream));
  }
  return DP_OK;
}

int clover_convert_all(dp_ctx* c) {
  for (int p = 0; p < 2; ++p) {
    DP_HIP(c, launch_clover_convert(c->g, c->C64[p].as<double2>(), c->C32[p].p, nullptr, F32, c->stream));
    DP_HIP(c, launch_clover_convert(c->g, c->C64[p].as<double2>(), c->C16[p].p, c->C16s[p].as<float>(), F16,
                                    c->stream));
  }
  return DP_OK;
}

CloverRef clover_ref(dp_ctx* c, int p, int prec) {
  CloverRef r;
  r.prec = prec;
  if (prec == F64) r.data = c->C64[p].p;
  if (prec == F32) r.data = c->C32[p].p;
  if (prec == F16) {
    r.data = c->C16[p].p;
    r.scale = c->C16s[p].as<float>();
  }
  return r;
}

// ------------------------------------------------------------- workspace

int ensure_ws(dp_ctx* c, int nslots, int prec) {
  Workspace& w = c->ws;
  const Geom& g = c->g;
  if (w.nslots < nslots || w.prec != prec) {
    const int n = nslots > w.nslots ? nslots : w.nslots;
    const int px = prec == F16 ? F32 : prec;
    Field* f64s[] = {&w.eta_e, &w.eta_o, &w.b64, &w.x64, &w.r64, &w.t64, &w.to64};
    for (Field* f : f64s) DP_HIP(c, f->alloc(g, F64, n));
    Field* fin[] = {&w.r, &w.rh, &w.p, &w.v, &w.s, &w.t, &w.to};
    for (Field* f : fin) DP_HIP(c, f->alloc(g, prec, n));
    DP_HIP(c, w.x.alloc(g, px, n));
    const int nb = std::max(reduction_blocks(g), hop_blocks(g));
    DP_HIP(c, w.ratio.reserve(sizeof(double) * 4 * g.T * n));
    DP_HIP(c, w.m4.reserve(sizeof(double) * n));
    DP_HIP(c, w.mask_all.reserve(sizeof(int) * n));
    DP_HIP(c, w.mask_inner.reserve(sizeof(int) * n));
    DP_HIP(c, w.mask_outer.reserve(sizeof(int) * n));
    for (int k = 0; k < 3; ++k) DP_HIP(c, w.ainv_ptr[k].reserve(sizeof(void*) * n));
    DP_HIP(c, w.ainv_scale_ptr.reserve(sizeof(float*) * n));
    DP_HIP(c, w.sc.reserve(sizeof(SlotScalars) * n));
    DP_HIP(c, w.partials.reserve(sizeof(double) * 4 * nb * n));
    DP_HIP(c, w.out_sums.reserve(sizeof(double) * 4 * n));
    DP_HIP(c, w.slot_scale.reserve(sizeof(double) * n));
    DP_HIP(c, w.x0src.reserve(sizeof(int) * n));
    DP_HIP(c, w.alpha.reserve(sizeof(double) * g.T * n));
    DP_HIP(c, w.cpp.reserve(sizeof(double) * g.T * n));
    DP_HIP(c, w.h_sc.reserve(sizeof(SlotScalars) * n));
    DP_HIP(c, w.h_sums.reserve(sizeof(double) * 4 * n));
    DP_HIP(c, w.h_mask.reserve(sizeof(int) * 3 * n));
    DP_HIP(c, w.h_scale.reserve(sizeof(double) * (4 * g.T + 4) * n));
    w.nslots = n;
    w.prec = prec;
  }
  return DP_OK;
}

#define DP_TRY(expr)              \
  do {                            \
    int rc_ = (expr);             \
    if (rc_ != DP_OK) return rc_; \
  } while (0)

// host -> device copy on the ctx stream, complete on return
int h2d(dp_ctx* c, void* dst, const void* src, size_t bytes) {
  DP_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  return DP_OK;
}

// Upload per-slot tables: alpha (one table for all), m4, A^-1 pointers, x0src.
int upload_slot_tables(dp_ctx* c, int nslots, const double* alpha, MassEntry* me, int x0src) {
  Workspace& w = c->ws;
  const int T = c->g.T;
  double* h = w.h_scale.as<double>();  // staging: [nslots][4T] ratios, then [nslots][T] alpha
  std::vector<double> rt(4 * T);
  ratio_tables(T, c->bc_t, alpha, rt.data());
  for (int s = 0; s < nslots; ++s) std::memcpy(h + (size_t)s * 4 * T, rt.data(), sizeof(double) * 4 * T);
  DP_HIP(c, hipMemcpyAsync(w.ratio.p, h, sizeof(double) * 4 * T * nslots, hipMemcpyHostToDevice, c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  for (int s = 0; s < nslots; ++s) std::memcpy(h + (size_t)s * T, alpha, sizeof(double) * T);
  DP_HIP(c, hipMemcpyAsync(w.alpha.p, h, sizeof(double) * T * nslots, hipMemcpyHostToDevice, c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  std::vector<double> m4(nslots, 4.0 + me->M);
  std::vector<const void*> p64(nslots, me->a64.p), p32(nslots, me->a32.p), p16(nslots, me->a16.p);
  std::vector<const float*> s16(nslots, me->s16.as<float>());
  std::vector<int> x0(nslots, x0src);
  DP_TRY(h2d(c, w.m4.p, m4.data(), sizeof(double) * nslots));
  DP_TRY(h2d(c, w.ainv_ptr[F64].p, p64.data(), sizeof(void*) * nslots));
  DP_TRY(h2d(c, w.ainv_ptr[F32].p, p32.data(), sizeof(void*) * nslots));
  DP_TRY(h2d(c, w.ainv_ptr[F16].p, p16.data(), sizeof(void*) * nslots));
  DP_TRY(h2d(c, w.ainv_scale_ptr.p, s16.data(), sizeof(float*) * nslots));
  DP_TRY(h2d(c, w.x0src.p, x0.data(), sizeof(int) * nslots));
  return DP_OK;
}

int upload_mask(dp_ctx* c, DevBuf& dst, const std::vector<int>& m, int slot_in_staging) {
  int cnt = 0;
  for (int v : m) cnt += v != 0;
  c->mask_count[dst.p] = cnt;
  int* h = c->ws.h_mask.as<int>() + (size_t)slot_in_staging * c->ws.nslots;
  std::memcpy(h, m.data(), sizeof(int) * m.size());
  DP_HIP(c, hipMemcpyAsync(dst.p, h, sizeof(int) * m.size(), hipMemcpyHostToDevice, c->stream));
  return DP_OK;
}

SlotTable slot_table(dp_ctx* c, int prec, const int* mask) {
  Workspace& w = c->ws;
  SlotTable t;
  t.ratio = w.ratio.as<double>();
  t.m4 = w.m4.as<double>();
  t.mask = mask;
  t.ainv = static_cast<const void* const*>(w.ainv_ptr[prec].p);
  t.ainv_scale = prec == F16 ? static_cast<const float* const*>(w.ainv_scale_ptr.p) : nullptr;
  return t;
}

ReduceRef reduce_ref(dp_ctx* c, int red, int fin) {
  Workspace& w = c->ws;
  ReduceRef r;
  r.red = red;
  r.fin = fin;
  r.partials = w.partials.as<double>();
  r.sc = w.sc.as<SlotScalars>();
  r.out_sums = w.out_sums.as<double>();
  return r;
}

// ----------------------------------------------------------- launch timing

const char* prec_name(int p) { return p == F64 ? "f64" : p == F32 ? "f32" : "f16"; }

int active_slots(dp_ctx* c, const int* mask, int nslots) {
  auto it = c->mask_count.find(mask);
  return it == c->mask_count.end() ? nslots : it->second;
}

int timing_begin(dp_ctx* c, hipEvent_t* a) {
  if (!c->timing) return DP_OK;
  if (c->ev_free.size() < 2) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      DP_HIP(c, hipEventCreate(&e));
      c->ev_free.push_back(e);
    }
  }
  *a = c->ev_free.back();
  c->ev_free.pop_back();
  DP_HIP(c, hipEventRecord(*a, c->stream));
  return DP_OK;
}

int timing_end(dp_ctx* c, hipEvent_t a, const std::string& name, double bytes, double flops) {
  if (!c->timing) return DP_OK;
  hipEvent_t b = c->ev_free.back();
  c->ev_free.pop_back();
  DP_HIP(c, hipEventRecord(b, c->stream));
  c->pending.push_back({name, bytes, flops, a, b});
  return DP_OK;
}

// fold finished launches into the per-kernel statistics (after a stream sync)
int timing_harvest(dp_ctx* c) {
  for (auto& q : c->pending) {
    float ms = 0.f;
    DP_HIP(c, hipEventSynchronize(q.b));
    DP_HIP(c, hipEventElapsedTime(&ms, q.a, q.b));
    auto& k = c->kstats[q.name];
    k.launches++;
    k.ms += ms;
    k.bytes += q.bytes;
    k.flops += q.flops;
    c->ev_free.push_back(q.a);
    c->ev_free.push_back(q.b);
  }
  c->pending.clear();
  return DP_OK;
}

// Algorithmic HBM bytes of one hop launch: each link, clover block and input
// spinor once, each output once.  Per output site: 8 links (144 reals, shared by
// the slots), per active slot the input (24) and output (24) spinors, the
// clover block pair (72 reals) for the epilogues that use it, the epilogue
// input (24 per slot) and the dot partner (24 per slot); FP16 adds the 4-byte
// per-site scales.  Flops: 1320 per site and slot for the hop, 552 for a
// clover block pair, 48 for the epilogue axpy and 8-16 for a fused dot.
void hop_cost(dp_ctx* c, int prec, int epi, int red, int nact, double* bytes, double* flops) {
  const double b = prec == F64 ? 8.0 : prec == F32 ? 4.0 : 2.0;
  const double sc = prec == F16 ? 4.0 : 0.0;
  const double Vh = c->g.Vh;
  double site = 144 * b;
  double slot = 2 * (24 * b + sc);
  double fl = 1320;
  if (epi == EPI_INV || epi == EPI_INV_SUB || epi == EPI_DIAG) {
    site += 72 * b + sc;
    fl += 552;
  }
  if (epi == EPI_DIAG || epi == EPI_SUB || epi == EPI_INV_SUB) {
    slot += 24 * b + sc;
    fl += 48;
  }
  if (red == RED_DOT_EXT) {
    slot += 24 * b + sc;
    fl += 96;
  } else if (red != RED_NONE) {
    fl += 96;
  }
  *bytes = Vh * (site + nact * slot);
  *flops = Vh * nact * fl;
}

// one hop launch; p = output parity
int hop(dp_ctx* c, int nslots, int prec, int p, int dag, int epi, double sign, const Field& in, const Field& out,
        const Field* xin, const int* mask, int red = RED_NONE, int fin = FIN_NONE, const Field* w = nullptr) {
  HopArgs a;
  a.g = c->g;
  a.p = p;
  a.dag = dag;
  a.epi = epi;
  a.sign = sign;
  a.U_out = c->U[prec][p].p;
  a.U_in = c->U[prec][1 - p].p;
  a.link_prec = prec;
  a.in = in.ref();
  a.out = out.ref();
  if (xin) a.xin = xin->ref();
  a.clov = clover_ref(c, p, prec);
  a.slots = slot_table(c, prec, mask);
  a.red = reduce_ref(c, red, fin);
  if (w) a.red.w = w->ref();
  a.nslots = nslots;
  hipEvent_t ev = nullptr;
  DP_TRY(timing_begin(c, &ev));
  DP_HIP(c, launch_hop(a, c->stream));
  if (c->timing) {
    static const char* epi_names[] = {"hop", "inv", "diag", "sub", "invsub"};
    double bytes, flops;
    hop_cost(c, prec, epi, red, active_slots(c, mask, nslots), &bytes, &flops);
    std::string name = std::string("hop_") + prec_name(prec) + "_" + epi_names[epi] + (dag ? "_dag" : "");
    DP_TRY(timing_end(c, ev, name, bytes, flops));
  }
  return DP_OK;
}

int blas(dp_ctx* c, int op, int nslots, int prec, const int* mask, std::initializer_list<const Field*> v,
         int fin = FIN_NONE) {
  BlasArgs a;
  a.g = c->g;
  a.nslots = nslots;
  a.prec = prec;
  a.mask = mask;
  a.sc = c->ws.sc.as<SlotScalars>();
  a.slot_scale = c->ws.slot_scale.as<double>();
  int k = 0;
  for (const Field* f : v) {
    if (f) a.v[k] = f->ref();
    ++k;
  }
  a.red = reduce_ref(c, RED_NONE, fin);
  hipEvent_t ev = nullptr;
  DP_TRY(timing_begin(c, &ev));
  DP_HIP(c, launch_blas(op, a, c->stream));
  if (c->timing) {
    // vectors read + written per site and slot (FP64 ones counted at 8 bytes)
    static const int nvec[] = {1, 2, 5, 4, 3, 7, 6, 3, 2, 3, 3, 1, 2};
    const double b = prec == F64 ? 8.0 : prec == F32 ? 4.0 : 2.0;
    const double bytes = (double)c->g.Vh * active_slots(c, mask, nslots) * nvec[op] * 24 * b;
    DP_TRY(timing_end(c, ev, std::string("blas_") + prec_name(prec) + "_" + std::to_string(op), bytes, 0.0));
  }
  return DP_OK;
}

// Mhat' in -> out (Schur operator on even sites), in prec; to = odd temporary
int schur(dp_ctx* c, int n, int prec, int dag, const Field& in, const Field& to, const Field& out, const int* mask,
          int red, int fin, const Field* w = nullptr) {
  DP_TRY(hop(c, n, prec, 1, dag, EPI_INV, 0.0, in, to, nullptr, mask));
  DP_TRY(hop(c, n, prec, 0, dag, EPI_DIAG, -1.0, to, out, &in, mask, red, fin, w));
  return DP_OK;
}

struct SlotHost {
  int done = 0, in_inner = 0, has_inner = 0;
  int iters = 0, outer = 0, restarts = 0, hops = 0;
  int status = DP_OK;
  double eta2 = 0.0, res2 = 0.0, scale = 0.0, tol2 = 0.0;
};

// ------------------------------------------------------------- the solve

int run_solve(dp_ctx* c, const double2* eta_dev, int n, const dp_params& P, double2* S_dev, double* cpp_out,
              dp_info* info) {
  const auto t_start = std::chrono::steady_clock::now();
  const int prec = P.precision;
  const int px = prec == F16 ? F32 : prec;
  (void)px;
  DP_TRY(ensure_ws(c, n, prec));
  MassEntry* me = nullptr;
  DP_TRY(mass_entry(c, c->M, &me));
  DP_TRY(upload_slot_tables(c, n, c->alpha.data(), me, P.x0_src));
  Workspace& w = c->ws;
  const Geom& g = c->g;
  const int* m_all = w.mask_all.as<int>();
  const int* m_in = w.mask_inner.as<int>();
  const int* m_out = w.mask_outer.as<int>();
  std::vector<int> all(n, 1), inner(n, 0), outer(n, 0);
  DP_TRY(upload_mask(c, w.mask_all, all, 0));

  // eta' = alpha eta on both parities, |eta'|^2 per slot
  DP_HIP(c, launch_spinor_import(g, eta_dev, n, 2L * g.Vh * 12, 0, w.eta_e.ref(), w.alpha.as<double>(), c->stream));
  DP_HIP(c, launch_spinor_import(g, eta_dev, n, 2L * g.Vh * 12, 1, w.eta_o.ref(), w.alpha.as<double>(), c->stream));
  std::vector<SlotHost> hs(n);
  double* sums = w.h_sums.as<double>();
  for (int par = 0; par < 2; ++par) {
    DP_TRY(blas(c, OP_NORM, n, F64, m_all, {nullptr, par ? &w.eta_o : &w.eta_e}, FIN_STORE));
    DP_HIP(c, hipMemcpyAsync(sums, w.out_sums.p, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, c->stream));
    DP_HIP(c, hipStreamSynchronize(c->stream));
    for (int s = 0; s < n; ++s) hs[s].eta2 += sums[4 * s];
  }
  for (int s = 0; s < n; ++s)
    if (!std::isfinite(hs[s].eta2)) return fail(c, DP_ERR_NONFINITE, "source contains NaN or Inf");

  // Schur right-hand side b = eta'_e - H_eo A_oo^-1 eta'_o, x = 0
  {
    SlotTable st = slot_table(c, F64, m_all);
    DP_HIP(c, launch_clover_apply(g, st, w.eta_o.ref(), w.to64.ref(), n, c->stream));
  }
  DP_TRY(hop(c, n, F64, 0, 0, EPI_SUB, 0.0, w.to64, w.b64, &w.eta_e, m_all));
  DP_TRY(blas(c, OP_ZERO, n, F64, m_all, {&w.x64}));
  for (int s = 0; s < n; ++s) hs[s].hops = 2;  // source preparation and odd reconstruction

  const double r2 = P.r * P.r;
  const double delta = P.delta > 0 ? P.delta : (prec == F16 ? 5e-3 : 1e-5);
  const int cgnr = P.solver == DP_SOLVER_CGNR;
  SlotScalars* hsc = w.h_sc.as<SlotScalars>();
  double* hscale = w.h_scale.as<double>();

  // outer step for the slots in `pend`: x += |r| e (when an inner result exists),
  // r = b - Mhat' x in FP64, the stopping test, and the start of the next inner solve
  auto outer_step = [&](const std::vector<int>& pend) -> int {
    for (int s = 0; s < n; ++s) outer[s] = pend[s];
    DP_TRY(upload_mask(c, w.mask_outer, outer, 1));
    bool any_prev = false;
    for (int s = 0; s < n; ++s) {
      hscale[s] = pend[s] && hs[s].has_inner ? hs[s].scale : 0.0;
      any_prev |= pend[s] && hs[s].has_inner;
    }
    if (any_prev) {
      DP_HIP(c, hipMemcpyAsync(w.slot_scale.p, hscale, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
      // slots without an inner result get a zero scale; their x buffer is still finite
      // because every inner start zeroes it, and the first outer step skips this
      DP_TRY(blas(c, OP_AXPY_SCALED, n, prec, m_out, {&w.x64, &w.x}));
    }
    DP_TRY(schur(c, n, F64, 0, w.x64, w.to64, w.t64, m_out, RED_NONE, FIN_NONE));
    DP_TRY(blas(c, OP_SUB64, n, F64, m_out, {&w.r64, &w.b64, &w.t64}, FIN_STORE));
    DP_HIP(c, hipMemcpyAsync(sums, w.out_sums.p, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, c->stream));
    DP_HIP(c, hipStreamSynchronize(c->stream));
    std::vector<int> start(n, 0);
    bool any_start = false;
    for (int s = 0; s < n; ++s) {
      if (!pend[s]) continue;
      SlotHost& h = hs[s];
      h.outer++;
      h.hops += 2;
      h.res2 = sums[4 * s];
      if (!std::isfinite(h.res2)) {
        h.done = 1;
        h.status = DP_ERR_NONFINITE;
      } else if (h.res2 <= r2 * h.eta2) {
        h.done = 1;
        h.status = DP_OK;
      } else if (h.iters >= P.max_iter) {
        h.done = 1;
        h.status = DP_ERR_NOT_CONVERGED;
      } else {
        start[s] = 1;
        any_start = true;
        h.scale = std::sqrt(h.res2);
        double need = 0.5 * P.r * std::sqrt(h.eta2 / h.res2);
        double tol = prec == F64 ? need : (need > delta ? need : delta);
        if (tol > 0.5) tol = 0.5;
        h.tol2 = tol * tol;
      }
    }
    if (!any_start) return DP_OK;
    for (int s = 0; s < n; ++s) hscale[s] = start[s] ? 1.0 / hs[s].scale : 0.0;
    DP_HIP(c, hipMemcpyAsync(w.slot_scale.p, hscale, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    for (int s = 0; s < n; ++s) outer[s] = start[s];
    DP_TRY(upload_mask(c, w.mask_outer, outer, 1));
    DP_TRY(blas(c, OP_SCALE_COPY, n, prec, m_out, {&w.r, &w.r64}));
    DP_TRY(blas(c, OP_BICG_INIT, n, prec, m_out, {&w.rh, &w.r, &w.p, &w.v, &w.x}, FIN_BICG_INIT));
    if (cgnr) {
      DP_TRY(schur(c, n, prec, 1, w.r, w.to, w.s, m_out, RED_NORM, FIN_CG_INIT));
      DP_TRY(blas(c, OP_COPY, n, prec, m_out, {&w.p, &w.s}));
    }
    for (int s = 0; s < n; ++s)
      if (start[s]) {
        hs[s].in_inner = 1;
        hs[s].has_inner = 1;
        hs[s].hops += cgnr ? 2 : 0;  // z = Mhat'^+ r
        inner[s] = 1;
      }
    DP_TRY(upload_mask(c, w.mask_inner, inner, 2));
    return DP_OK;
  };

  DP_TRY(outer_step(all));
  while (true) {
    bool any = false;
    for (int s = 0; s < n; ++s) any |= hs[s].in_inner != 0;
    if (!any) break;
    if (!cgnr) {
      DP_TRY(blas(c, OP_BICG_P, n, prec, m_in, {&w.p, &w.r, &w.v}));
      DP_TRY(schur(c, n, prec, 0, w.p, w.to, w.v, m_in, RED_DOT_EXT, FIN_BICG_ALPHA, &w.rh));
      DP_TRY(blas(c, OP_BICG_S, n, prec, m_in, {&w.s, &w.r, &w.v}));
      DP_TRY(schur(c, n, prec, 0, w.s, w.to, w.t, m_in, RED_TS, FIN_BICG_OMEGA));
      DP_TRY(blas(c, OP_BICG_XR, n, prec, m_in, {&w.x, &w.p, &w.s, &w.r, &w.t, &w.rh}, FIN_BICG_RHO));
    } else {
      DP_TRY(schur(c, n, prec, 0, w.p, w.to, w.v, m_in, RED_NORM, FIN_CG_ALPHA));
      DP_TRY(blas(c, OP_CG_XR, n, prec, m_in, {&w.x, &w.p, &w.r, &w.v}, FIN_RR));
      DP_TRY(schur(c, n, prec, 1, w.r, w.to, w.s, m_in, RED_NORM, FIN_CG_BETA));
      DP_TRY(blas(c, OP_CG_P, n, prec, m_in, {&w.p, &w.s}));
    }
    DP_HIP(c, hipMemcpyAsync(hsc, w.sc.p, sizeof(SlotScalars) * n, hipMemcpyDeviceToHost, c->stream));
    DP_HIP(c, hipStreamSynchronize(c->stream));
    std::vector<int> pend(n, 0);
    bool any_pend = false;
    for (int s = 0; s < n; ++s) {
      SlotHost& h = hs[s];
      if (!h.in_inner) continue;
      h.iters++;
      h.hops += 4;
      const double rr = hsc[s].rr;
      bool leave = false;
      if (!std::isfinite(rr) || rr <= h.tol2 || h.iters >= P.max_iter) leave = true;
      if (!cgnr && hsc[s].breakdown) {
        leave = true;
        h.restarts++;
      }
      if (leave) {
        h.in_inner = 0;
        inner[s] = 0;
        pend[s] = 1;
        any_pend = true;
      }
    }
    if (any_pend) {
      DP_TRY(upload_mask(c, w.mask_inner, inner, 2));
      DP_TRY(outer_step(pend));
    }
  }

  // odd sites S'_o = A_oo^-1 (eta'_o - H_oe S'_e), restoration and C_PP
  DP_TRY(hop(c, n, F64, 1, 0, EPI_INV_SUB, 0.0, w.x64, w.to64, &w.eta_o, m_all));
  if (S_dev)
    DP_HIP(c, launch_spinor_export(g, w.x64.ref(), w.to64.ref(), n, w.alpha.as<double>(), S_dev, 2L * g.Vh * 12,
                                   c->stream));
  int rc = DP_OK;
  if (cpp_out) {
    DP_HIP(c, launch_cpp(g, w.x64.ref(), w.to64.ref(), n, w.alpha.as<double>(), w.x0src.as<int>(),
                         w.cpp.as<double>(), c->stream));
    std::vector<double> per(static_cast<size_t>(n) * g.T);
    DP_HIP(c, hipMemcpyAsync(per.data(), w.cpp.p, sizeof(double) * g.T * n, hipMemcpyDeviceToHost, c->stream));
    DP_HIP(c, hipStreamSynchronize(c->stream));
    const int grp = P.ncols_group > 0 ? P.ncols_group : 1;
    for (int k = 0; k < n / grp; ++k)
      for (int t = 0; t < g.T; ++t) {
        double acc = 0.0;
        for (int j = 0; j < grp; ++j) acc += per[(size_t)(k * grp + j) * g.T + t];
        cpp_out[(size_t)k * g.T + t] = acc;
      }
  }
  DP_HIP(c, hipStreamSynchronize(c->stream));
  DP_TRY(timing_harvest(c));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  for (int s = 0; s < n; ++s) {
    if (hs[s].status != DP_OK && rc == DP_OK) rc = hs[s].status;
    if (info) {
      info[s].status = hs[s].status;
      info[s].iters = hs[s].iters;
      info[s].outer = hs[s].outer;
      info[s].hop_calls = hs[s].hops;
      info[s].restarts = hs[s].restarts;
      info[s].true_res = hs[s].eta2 > 0 ? std::sqrt(hs[s].res2 / hs[s].eta2) : 0.0;
      info[s].seconds = secs;
    }
  }
  if (rc != DP_OK) {
    if (rc == DP_ERR_NOT_CONVERGED) c->err = "a right-hand side reached max_iter before the residue r";
    if (rc == DP_ERR_NONFINITE) c->err = "a residual became NaN or Inf";
  }
  return rc;
}

int validate_params(dp_ctx* c, int nrhs, const dp_params* p) {
  if (!p) return fail(c, DP_ERR_INVALID_ARG, "params is NULL");
  if (nrhs <= 0) return fail(c, DP_ERR_INVALID_ARG, "nrhs must be positive");
  if (!(p->r > 0) || !std::isfinite(p->r)) return fail(c, DP_ERR_INVALID_ARG, "r must be positive");
  if (p->solver != DP_SOLVER_BICGSTAB && p->solver != DP_SOLVER_CGNR)
    return fail(c, DP_ERR_INVALID_ARG, "unknown solver");
  if (p->precision < DP_PREC_F64 || p->precision > DP_PREC_F16) return fail(c, DP_ERR_INVALID_ARG, "unknown precision");
  if (p->max_iter <= 0) return fail(c, DP_ERR_INVALID_ARG, "max_iter must be positive");
  if (p->delta < 0 || p->delta >= 1) return fail(c, DP_ERR_INVALID_ARG, "delta must be in [0, 1)");
  if (p->x0_src < 0 || p->x0_src >= c->g.T) return fail(c, DP_ERR_INVALID_ARG, "x0_src outside [0, T)");
  if (p->ncols_group < 0 || (p->ncols_group > 0 && nrhs % p->ncols_group != 0))
    return fail(c, DP_ERR_INVALID_ARG, "nrhs must be a multiple of ncols_group");
  return DP_OK;
}

// Udev == nullptr sets unit links
int set_gauge_common(dp_ctx* c, const double2* Udev, hipStream_t st) {
  const Geom& g = c->g;
  for (int prec = 0; prec < 3; ++prec) {
    for (int p = 0; p < 2; ++p) DP_HIP(c, c->U[prec][p].reserve((size_t)g.Vh * link_site_bytes(prec)));
    void* dst[2] = {c->U[prec][0].p, c->U[prec][1].p};
    DP_HIP(c, launch_gauge_reorder(g, Udev, dst, prec, st));
    c->have_U[prec] = true;
  }
  DP_HIP(c, hipStreamSynchronize(st));
  drop_masses(c);
  c->clover_kind = 0;
  c->csw = 0.0;
  return clover_zero(c);
}

}  // namespace

// ===================================================================== C ABI

extern "C" {

int dp_create(const int dims[4], int bc_t, int device, dp_ctx** out) {
  if (!out || !dims) return DP_ERR_INVALID_ARG;
  *out = nullptr;
  for (int k = 0; k < 4; ++k)
    if (dims[k] < 2 || dims[k] % 2) return DP_ERR_INVALID_ARG;
  if (bc_t != 1 && bc_t != -1) return DP_ERR_INVALID_ARG;
  const long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
  if (V / 2 > (1L << 30) / 12) return DP_ERR_INVALID_ARG;  // 32-bit indexing of the SoA fields
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return DP_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return DP_ERR_DEVICE;
  dp_ctx* c = new (std::nothrow) dp_ctx;
  if (!c) return DP_ERR_OOM;
  c->device = device;
  c->bc_t = bc_t;
  for (int k = 0; k < 4; ++k) c->dims[k] = dims[k];
  Geom& g = c->g;
  g.T = dims[0];
  g.L1 = dims[1];
  g.L2 = dims[2];
  g.L3 = dims[3];
  g.L3h = g.L3 / 2;
  g.Vsh = g.L1 * g.L2 * g.L3 / 2;
  g.Vh = g.T * g.Vsh;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return DP_ERR_DEVICE;
  }
  c->alpha.assign(g.T, 1.0);
  int rc = clover_zero(c);
  if (rc != DP_OK) {
    delete c;
    return rc;
  }
  rc = set_gauge_common(c, nullptr, c->stream);  // unit links
  if (rc != DP_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return DP_OK;
}

void dp_destroy(dp_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

const char* dp_last_error(const dp_ctx* c) { return c ? c->err.c_str() : "null context"; }

int dp_set_gauge(dp_ctx* c, const double* U) {
  if (!c || !U) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  DP_HIP(c, hipSetDevice(c->device));
  const size_t bytes = (size_t)2 * c->g.Vh * 4 * 9 * sizeof(double2);
  DP_HIP(c, c->scratch_aos.reserve(bytes));
  DP_HIP(c, hipMemcpyAsync(c->scratch_aos.p, U, bytes, hipMemcpyHostToDevice, c->stream));
  int rc = set_gauge_common(c, c->scratch_aos.as<double2>(), c->stream);
  c->scratch_aos.release();
  return rc;
}

int dp_set_gauge_dev(dp_ctx* c, const void* U, void* stream) {
  if (!c || !U) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  DP_HIP(c, hipSetDevice(c->device));
  hipStream_t st = stream ? (hipStream_t)stream : c->stream;
  DP_HIP(c, hipStreamSynchronize(st));
  return set_gauge_common(c, static_cast<const double2*>(U), c->stream);
}

int dp_set_clover(dp_ctx* c, double csw) {
  if (!c || !std::isfinite(csw)) return fail(c, DP_ERR_INVALID_ARG, "bad argument");
  DP_HIP(c, hipSetDevice(c->device));
  DP_TRY(check_state(c));
  drop_masses(c);
  if (csw == 0.0) {
    DP_TRY(clover_zero(c));
    c->clover_kind = 0;
  } else {
    const double2* U64[2] = {c->U[F64][0].as<double2>(), c->U[F64][1].as<double2>()};
    double2* C[2] = {c->C64[0].as<double2>(), c->C64[1].as<double2>()};
    DP_HIP(c, launch_clover_build(c->g, U64, csw, C, c->stream));
    DP_TRY(clover_convert_all(c));
    c->clover_kind = 1;
  }
  c->csw = csw;
  DP_HIP(c, hipStreamSynchronize(c->stream));
  return DP_OK;
}

int dp_set_clover_field(dp_ctx* c, const double* Cf) {
  if (!c || !Cf) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  DP_HIP(c, hipSetDevice(c->device));
  const size_t bytes = (size_t)2 * c->g.Vh * 144 * sizeof(double2);
  DP_HIP(c, c->scratch_aos.reserve(bytes));
  DP_HIP(c, hipMemcpyAsync(c->scratch_aos.p, Cf, bytes, hipMemcpyHostToDevice, c->stream));
  DP_HIP(c, c->bad_flag.reserve(sizeof(int)));
  DP_HIP(c, hipMemsetAsync(c->bad_flag.p, 0, sizeof(int), c->stream));
  double2* C[2] = {c->C64[0].as<double2>(), c->C64[1].as<double2>()};
  DP_HIP(c, launch_clover_pack(c->g, c->scratch_aos.as<double2>(), C, c->bad_flag.as<int>(), c->stream));
  int bad = 0;
  DP_HIP(c, hipMemcpyAsync(&bad, c->bad_flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  c->scratch_aos.release();
  drop_masses(c);
  if (bad) {
    clover_zero(c);
    c->clover_kind = 0;
    return fail(c, DP_ERR_INVALID_ARG, "clover field is not Hermitian or mixes the two chiralities");
  }
  DP_TRY(clover_convert_all(c));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  c->clover_kind = 2;
  return DP_OK;
}

int dp_set_mass(dp_ctx* c, double M) {
  if (!c || !std::isfinite(M)) return fail(c, DP_ERR_INVALID_ARG, "mass must be finite");
  c->M = M;
  return DP_OK;
}

int dp_set_kappa(dp_ctx* c, double kappa) {
  if (!c || !(kappa > 0) || !std::isfinite(kappa)) return fail(c, DP_ERR_INVALID_ARG, "kappa must be positive");
  c->M = 1.0 / (2.0 * kappa) - 4.0;
  return DP_OK;
}

int dp_set_alpha(dp_ctx* c, const double* alpha) {
  if (!c || !alpha) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  for (int t = 0; t < c->g.T; ++t)
    if (!(alpha[t] > 0) || !std::isfinite(alpha[t]) || !std::isfinite(1.0 / alpha[t]))
      return fail(c, DP_ERR_INVALID_ARG, "alpha must be finite and positive");
  c->alpha.assign(alpha, alpha + c->g.T);
  return DP_OK;
}

int dp_apply(dp_ctx* c, const double* in, double* out, int flags) {
  if (!c || !in || !out) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  if (flags & ~(DP_PRECOND | DP_DAGGER | DP_HOP_ONLY | DP_APPLY_SCHUR | DP_APPLY_F32 | DP_APPLY_F16))
    return fail(c, DP_ERR_INVALID_ARG, "unknown flag");
  if ((flags & DP_APPLY_F32) && (flags & DP_APPLY_F16)) return fail(c, DP_ERR_INVALID_ARG, "two precisions");
  if ((flags & DP_HOP_ONLY) && (flags & DP_APPLY_SCHUR)) return fail(c, DP_ERR_INVALID_ARG, "hop-only Schur");
  DP_HIP(c, hipSetDevice(c->device));
  DP_TRY(check_state(c));
  const int prec = (flags & DP_APPLY_F32) ? F32 : (flags & DP_APPLY_F16) ? F16 : F64;
  const int dag = (flags & DP_DAGGER) ? 1 : 0;
  DP_TRY(ensure_ws(c, 1, prec));
  MassEntry* me = nullptr;
  DP_TRY(mass_entry(c, c->M, &me));
  std::vector<double> ones(c->g.T, 1.0);
  DP_TRY(upload_slot_tables(c, 1, (flags & DP_PRECOND) ? c->alpha.data() : ones.data(), me, 0));
  Workspace& w = c->ws;
  const Geom& g = c->g;
  std::vector<int> one(1, 1);
  DP_TRY(upload_mask(c, w.mask_all, one, 0));
  const int* m = w.mask_all.as<int>();
  const size_t bytes = (size_t)2 * g.Vh * 12 * sizeof(double2);
  DP_HIP(c, c->scratch_aos.reserve(bytes));
  DP_HIP(c, hipMemcpyAsync(c->scratch_aos.p, in, bytes, hipMemcpyHostToDevice, c->stream));
  DP_HIP(c, launch_spinor_import(g, c->scratch_aos.as<double2>(), 1, 0, 0, w.eta_e.ref(), nullptr, c->stream));
  DP_HIP(c, launch_spinor_import(g, c->scratch_aos.as<double2>(), 1, 0, 1, w.eta_o.ref(), nullptr, c->stream));
  // inputs in the compute precision: even in r, odd in s (Vh sites each)
  const Field* ie = &w.eta_e;
  const Field* io = &w.eta_o;
  const Field* oe = &w.b64;
  const Field* oo = &w.to64;
  if (prec != F64) {
    double one_d = 1.0;
    DP_TRY(h2d(c, w.slot_scale.p, &one_d, sizeof(double)));
    DP_TRY(blas(c, OP_SCALE_COPY, 1, prec, m, {&w.r, &w.eta_e}));
    DP_TRY(blas(c, OP_SCALE_COPY, 1, prec, m, {&w.s, &w.eta_o}));
    ie = &w.r;
    io = &w.s;
    oe = &w.v;
    oo = &w.t;
  }
  if (flags & DP_HOP_ONLY) {
    DP_TRY(hop(c, 1, prec, 0, dag, EPI_HOP, 0.0, *io, *oe, nullptr, m));
    DP_TRY(hop(c, 1, prec, 1, dag, EPI_HOP, 0.0, *ie, *oo, nullptr, m));
  } else if (flags & DP_APPLY_SCHUR) {
    DP_TRY(schur(c, 1, prec, dag, *ie, w.to, *oe, m, RED_NONE, FIN_NONE));
    DP_TRY(blas(c, OP_ZERO, 1, prec, m, {oo}));
  } else {
    DP_TRY(hop(c, 1, prec, 0, dag, EPI_DIAG, 1.0, *io, *oe, ie, m));
    DP_TRY(hop(c, 1, prec, 1, dag, EPI_DIAG, 1.0, *ie, *oo, io, m));
  }
  if (prec != F64) {
    DP_TRY(blas(c, OP_TO64, 1, prec, m, {&w.b64, oe}));
    DP_TRY(blas(c, OP_TO64, 1, prec, m, {&w.to64, oo}));
  }
  DP_HIP(c, launch_spinor_export(g, w.b64.ref(), w.to64.ref(), 1, nullptr, c->scratch_aos.as<double2>(), 0,
                                 c->stream));
  DP_HIP(c, hipMemcpyAsync(out, c->scratch_aos.p, bytes, hipMemcpyDeviceToHost, c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  DP_TRY(timing_harvest(c));
  return DP_OK;
}

int dp_solve(dp_ctx* c, const double* eta, int nrhs, const dp_params* p, double* S, double* cpp, dp_info* info) {
  if (!c || !eta) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  DP_HIP(c, hipSetDevice(c->device));
  DP_TRY(validate_params(c, nrhs, p));
  DP_TRY(check_state(c));
  const size_t bytes = (size_t)nrhs * 2 * c->g.Vh * 12 * sizeof(double2);
  DP_HIP(c, c->scratch_aos.reserve(bytes));
  DP_HIP(c, hipMemcpyAsync(c->scratch_aos.p, eta, bytes, hipMemcpyHostToDevice, c->stream));
  int rc = run_solve(c, c->scratch_aos.as<double2>(), nrhs, *p, S ? c->scratch_aos.as<double2>() : nullptr, cpp, info);
  if (S && (rc == DP_OK || rc == DP_ERR_NOT_CONVERGED)) {
    DP_HIP(c, hipMemcpyAsync(S, c->scratch_aos.p, bytes, hipMemcpyDeviceToHost, c->stream));
    DP_HIP(c, hipStreamSynchronize(c->stream));
  }
  return rc;
}

int dp_solve_dev(dp_ctx* c, const void* eta, int nrhs, const dp_params* p, void* S, double* cpp, dp_info* info,
                 void* stream) {
  if (!c || !eta) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  DP_HIP(c, hipSetDevice(c->device));
  DP_TRY(validate_params(c, nrhs, p));
  DP_TRY(check_state(c));
  if (stream) DP_HIP(c, hipStreamSynchronize((hipStream_t)stream));
  return run_solve(c, static_cast<const double2*>(eta), nrhs, *p, static_cast<double2*>(S), cpp, info);
}

int dp_set_timing(dp_ctx* c, int enable) {
  if (!c) return DP_ERR_INVALID_ARG;
  DP_HIP(c, hipSetDevice(c->device));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  DP_TRY(timing_harvest(c));
  c->kstats.clear();
  c->timing = enable != 0;
  return DP_OK;
}

int dp_get_timing(dp_ctx* c, dp_kernel_stat* out, int max, int* count) {
  if (!c || !count || max < 0 || (max > 0 && !out)) return fail(c, DP_ERR_INVALID_ARG, "bad argument");
  DP_HIP(c, hipSetDevice(c->device));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  DP_TRY(timing_harvest(c));
  int n = 0;
  for (const auto& kv : c->kstats) {
    if (n < max) {
      dp_kernel_stat& o = out[n];
      std::memset(&o, 0, sizeof o);
      std::strncpy(o.name, kv.first.c_str(), sizeof o.name - 1);
      o.launches = kv.second.launches;
      o.ms = kv.second.ms;
      o.bytes = kv.second.bytes;
      o.flops = kv.second.flops;
    }
    ++n;
  }
  *count = n;
  return DP_OK;
}

long long dp_footprint_bytes(const int dims[4], int nrhs, int precision, int new_masses) {
  if (!dims || nrhs < 0 || precision < 0 || precision > 2 || new_masses < 0) return -1;
  long long V = 1;
  for (int k = 0; k < 4; ++k) {
    if (dims[k] < 2 || dims[k] % 2) return -1;
    V *= dims[k];
  }
  const long long Vh = V / 2;
  long long b = 0;
  for (int p = 0; p < 3; ++p) b += 2 * Vh * (long long)link_site_bytes(p);      // links
  for (int p = 0; p < 3; ++p) b += 2 * Vh * (long long)clover_site_bytes(p);    // clover
  b += 2 * Vh * 4;                                                              // FP16 clover scales
  const long long mass = Vh * (long long)(clover_site_bytes(0) + clover_site_bytes(1) + clover_site_bytes(2) + 4);
  b += new_masses * mass;
  const long long f64 = Vh * 192, fin = Vh * (long long)(spinor_site_bytes(precision) + spinor_scale_bytes(precision));
  const long long fx = Vh * (long long)spinor_site_bytes(precision == 2 ? 1 : precision);
  b += nrhs * (7 * f64 + 7 * fin + fx);
  return b;
}

}  // extern "C"
