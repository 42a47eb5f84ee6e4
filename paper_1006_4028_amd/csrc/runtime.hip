// Host runtime of libdp: the context (resident fields, per-mass inverses),
// the launch helpers, dp_apply and the timing statistics.  The solver over
// slots lives in batch.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>

#include "runtime.h"

using namespace dp;

namespace dp {

hipError_t Field::alloc(const Geom& g, int prec_, int nslots_) {
  prec = prec_;
  nslots = nslots_;
  // double2 x12, float4 x6 or uint4 x3 per site
  slot_stride = (long)g.Vp * (prec == F64 ? 12 : prec == F32 ? 6 : 3);
  scale_stride = prec == F16 ? g.Vp : 0;
  hipError_t e = data.reserve((size_t)nslots * g.Vp * spinor_site_bytes(prec));
  if (e != hipSuccess) return e;
  if (prec == F16) e = scale.reserve((size_t)nslots * g.Vp * sizeof(float));
  return e;
}

SpinorRef Field::ref(int s0) const {
  SpinorRef r;
  const size_t unit = prec == F64 ? sizeof(double2) : prec == F32 ? sizeof(float4) : sizeof(uint4);
  r.data = data.p ? static_cast<char*>(data.p) + (size_t)s0 * slot_stride * unit : nullptr;
  r.scale = scale.p ? scale.as<float>() + (size_t)s0 * scale_stride : nullptr;
  r.slot_stride = slot_stride;
  r.scale_stride = scale_stride;
  r.prec = prec;
  return r;
}

size_t Workspace::device_bytes() const {
  const Field* f[] = {&eta_e, &eta_o, &b64, &x64, &r64, &t64, &to64, &r, &rh, &p, &v, &s, &t, &x, &to};
  size_t b = 0;
  for (const Field* q : f) b += q->data.bytes + q->scale.bytes;
  return b;
}

namespace rt {

int fail(dp_ctx* c, int code, const char* msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(dp_ctx* c, hipError_t e, const char* expr, int line) {
  if (c) {
    char b[320];
    snprintf(b, sizeof b, "%s failed: %s (line %d)", expr, hipGetErrorString(e), line);
    c->err = b;
  }
  return e == hipErrorOutOfMemory ? DP_ERR_OOM : DP_ERR_DEVICE;
}

bool env_pad() {
  static const bool v = [] {
    const char* e = getenv("DP_PAD");
    return e && atoi(e) == 1;
  }();
  return v;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ratio tables of the modified time hops for one alpha table:
//   fwd[x0] = s_f alpha(x0)/alpha(x0+1), bwd[x0] = s_b alpha(x0)/alpha(x0-1),
//   fwd_dag, bwd_dag the same for 1/alpha, with the fermion boundary sign s
//   at the wrap-around (the boundary rule eq. redeftbc in ratio form); s = 0
//   is the Dirichlet boundary, the hops across it drop.
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

// The spatial tables of the light-quark factorisation for profiles a[0..2]
// (NULL: ones): variant 0 is all ones, variant 1 the given profiles; each is
// 4 S ratios (fwd, bwd, fwd_dag, bwd_dag per direction, periodic) followed by
// the S profile values, S = L1 + L2 + L3.
int upload_space(dp_ctx* c, const double* const a[3]) {
  const Geom& g = c->g;
  const int Ls[3] = {g.L1, g.L2, g.L3};
  const int S = g.L1 + g.L2 + g.L3;
  std::vector<double> h((size_t)10 * S, 1.0);
  double* r = h.data() + 5 * S;  // variant 1
  int off = 0, poff = 4 * S;
  for (int k = 0; k < 3; ++k) {
    const int L = Ls[k];
    for (int x = 0; x < L; ++x) {
      const double v = a[k] ? a[k][x] : 1.0;
      const double vp = a[k] ? a[k][(x + 1) % L] : 1.0;
      const double vm = a[k] ? a[k][(x - 1 + L) % L] : 1.0;
      r[off + x] = v / vp;
      r[off + L + x] = v / vm;
      r[off + 2 * L + x] = vp / v;
      r[off + 3 * L + x] = vm / v;
      r[poff + x] = v;
    }
    off += 4 * L;
    poff += L;
  }
  DP_HIP(c, c->space.reserve(sizeof(double) * h.size()));
  DP_TRY(h2d(c, c->space.p, h.data(), sizeof(double) * h.size()));
  c->has_space = a[0] || a[1] || a[2];
  return DP_OK;
}

const double* space_ratios(dp_ctx* c, int variant) {
  const Geom& g = c->g;
  return c->space.as<double>() + (size_t)variant * 5 * (g.L1 + g.L2 + g.L3);
}

const double* space_hop_ratios(dp_ctx* c) { return c->has_space ? space_ratios(c, 1) : nullptr; }

const double* space_profile(dp_ctx* c) {
  const Geom& g = c->g;
  return c->has_space ? space_ratios(c, 1) + 4 * (g.L1 + g.L2 + g.L3) : nullptr;
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
  hipError_t e = m->a64.reserve((size_t)g.Vp * clover_site_bytes(F64));
  if (e == hipSuccess) e = m->a32.reserve((size_t)g.Vp * clover_site_bytes(F32));
  if (e == hipSuccess) e = m->a16.reserve((size_t)g.Vp * clover_site_bytes(F16));
  if (e == hipSuccess) e = m->s16.reserve((size_t)g.Vp * sizeof(float));
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

int ensure_ws(dp_ctx* c, Workspace& w, int nslots, int prec) {
  const Geom& g = c->g;
  if (w.nslots >= nslots && w.prec == prec) return DP_OK;
  const int n = std::max(nslots, w.nslots);
  const int px = prec == F16 ? F32 : prec;
  Field* f64s[] = {&w.eta_e, &w.eta_o, &w.b64, &w.x64, &w.r64, &w.t64, &w.to64};
  for (Field* f : f64s) DP_HIP(c, f->alloc(g, F64, n));
  Field* fin[] = {&w.r, &w.p, &w.v, &w.s, &w.t, &w.to};
  for (Field* f : fin) DP_HIP(c, f->alloc(g, prec, n));
  DP_HIP(c, w.rh.alloc(g, rh_prec(prec), n));
  DP_HIP(c, w.x.alloc(g, px, n));
  const int nb = std::max(reduction_blocks(g), hop_blocks(g));
  DP_HIP(c, w.ratio.reserve(sizeof(double) * 4 * g.T * n));
  DP_HIP(c, w.m4.reserve(sizeof(double) * n));
  DP_HIP(c, w.mask_inner.reserve(sizeof(int) * n));
  DP_HIP(c, w.mask_outer.reserve(sizeof(int) * n));
  for (int k = 0; k < 3; ++k) {
    DP_HIP(c, w.ainv_ptr[k].reserve(sizeof(void*) * n));
    w.h_ainv[k].assign(n, nullptr);
  }
  DP_HIP(c, w.ainv_scale_ptr.reserve(sizeof(float*) * n));
  w.h_ainv_scale.assign(n, nullptr);
  DP_HIP(c, w.sc.reserve(sizeof(SlotScalars) * n));
  DP_HIP(c, w.partials.reserve(sizeof(double) * kRedMax * nb * n));
  DP_HIP(c, w.out_sums.reserve(sizeof(double) * 4 * n));
  DP_HIP(c, w.slot_scale.reserve(sizeof(double) * n));
  DP_HIP(c, w.x0src.reserve(sizeof(int) * n));
  DP_HIP(c, w.alpha.reserve(sizeof(double) * g.T * n));
  DP_HIP(c, w.cpp.reserve(sizeof(double) * g.T * n));
  DP_HIP(c, w.h_sc.reserve(sizeof(SlotScalars) * n));
  DP_HIP(c, w.h_sums.reserve(sizeof(double) * 4 * n));
  DP_HIP(c, w.h_mask.reserve(sizeof(int) * 4 * n));
  DP_HIP(c, w.h_scale.reserve(sizeof(double) * (4 * g.T + 8) * n));
  DP_HIP(c, hipMemsetAsync(w.mask_inner.p, 0, sizeof(int) * n, c->stream));
  DP_HIP(c, hipMemsetAsync(w.mask_outer.p, 0, sizeof(int) * n, c->stream));
  DP_HIP(c, hipMemsetAsync(w.sc.p, 0, sizeof(SlotScalars) * n, c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  w.nslots = n;
  w.prec = prec;
  return DP_OK;
}

// host -> device copy on the ctx stream, complete on return
int h2d(dp_ctx* c, void* dst, const void* src, size_t bytes) {
  DP_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  return DP_OK;
}

// Upload a host mask through its own pinned staging row; each row is only
// rewritten after a later stream synchronisation.
int upload_mask(dp_ctx* c, Workspace& w, DevBuf& dst, const std::vector<int>& m, int staging) {
  int cnt = 0;
  for (int v : m) cnt += v != 0;
  c->mask_count[dst.p] = cnt;
  int* h = w.h_mask.as<int>() + (size_t)staging * w.nslots;
  std::memcpy(h, m.data(), sizeof(int) * m.size());
  DP_HIP(c, hipMemcpyAsync(dst.p, h, sizeof(int) * m.size(), hipMemcpyHostToDevice, c->stream));
  return DP_OK;
}

// ----------------------------------------------------------- launch timing

namespace {

const char* prec_name(int p) { return p == F64 ? "f64" : p == F32 ? "f32" : "f16"; }

int active_slots(dp_ctx* c, const int* mask, int n) {
  if (!mask) return n;
  auto it = c->mask_count.find(mask);
  return it == c->mask_count.end() ? n : std::min(n, it->second);
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

// Algorithmic HBM bytes of one hop launch: each link, clover block and input
// spinor once, each output once.  Per output site: 8 links (144 reals, shared by
// the slots), per active slot the input (24) and output (24) spinors, the
// clover block pair (72 reals) for the epilogues that use it, the epilogue
// input (24 per slot) and the dot partner (24 per slot); FP16 adds the 4-byte
// per-site scales.  Flops: 1320 per site and slot for the hop, 552 for a
// clover block pair, 48 for the epilogue axpy and 96 for a fused dot.
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
  if (red == RED_DOT_EXT || red == RED_TS4) {  // the shadow residual, stored in rh_prec(prec)
    const int pw = rh_prec(prec);
    slot += 24 * (pw == F64 ? 8.0 : pw == F32 ? 4.0 : 2.0) + (pw == F16 ? 4.0 : 0.0);
    fl += 96;
  } else if (red != RED_NONE) {
    fl += 96;
  }
  *bytes = Vh * (site + nact * slot);
  *flops = Vh * nact * fl;
}

// reductions of the slots [s0, ...) of a workspace
ReduceRef reduce_ref(Workspace& w, int s0, int red, int fin, int* inner_mask) {
  ReduceRef r;
  r.red = red;
  r.fin = fin;
  r.partials = w.partials.as<double>();  // indexed by the slot within the launch
  r.sc = w.sc.as<SlotScalars>() + s0;
  r.out_sums = w.out_sums.as<double>() + (size_t)4 * s0;
  r.inner_mask = inner_mask ? inner_mask + s0 : nullptr;
  return r;
}

}  // namespace

// per-slot tables of the slots [s0, ...) of a workspace
SlotTable slot_table(Workspace& w, int T, int s0, int prec, const int* mask) {
  SlotTable t;
  t.ratio = w.ratio.as<double>() + (size_t)s0 * 4 * T;
  t.m4 = w.m4.as<double>() + s0;
  t.mask = mask ? mask + s0 : nullptr;
  t.ainv = static_cast<const void* const*>(w.ainv_ptr[prec].p) + s0;
  t.ainv_scale = prec == F16 ? static_cast<const float* const*>(w.ainv_scale_ptr.p) + s0 : nullptr;
  return t;
}

const void* common_ainv(const Workspace& w, int s0, int n, int prec, const float** scale) {
  *scale = nullptr;
  if (n <= 0 || s0 + n > (int)w.h_ainv[prec].size()) return nullptr;
  const void* p0 = w.h_ainv[prec][s0];
  const float* q0 = w.h_ainv_scale[s0];
  for (int s = s0 + 1; s < s0 + n; ++s)
    if (w.h_ainv[prec][s] != p0 || w.h_ainv_scale[s] != q0) return nullptr;
  if (prec == F16) *scale = q0;
  return p0;
}

int timing_harvest(dp_ctx* c) {
  for (auto& q : c->pending) {
    float ms = 0.f;
    DP_HIP(c, hipEventSynchronize(q.b));
    DP_HIP(c, hipEventElapsedTime(&ms, q.a, q.b));
    auto& k = c->kstats[q.name];
    k.launches++;
    k.ms += ms;
    if (k.samples.size() < dp_ctx::kMaxSamples) k.samples.push_back(ms);
    k.bytes += q.bytes;
    k.flops += q.flops;
    c->ev_free.push_back(q.a);
    c->ev_free.push_back(q.b);
  }
  c->pending.clear();
  return DP_OK;
}

int hop(dp_ctx* c, Workspace& w, int s0, int n, int prec, int p, int dag, int epi, double sign, const Field& in,
        const Field& out, const Field* xin, const int* mask, int red, int fin, const Field* wv, int* inner_mask) {
  HopArgs a;
  a.g = c->g;
  a.p = p;
  a.dag = dag;
  a.epi = epi;
  a.sign = sign;
  a.U_out = c->U[prec][p].p;
  a.U_in = c->U[prec][1 - p].p;
  a.link_prec = prec;
  a.in = in.ref(s0);
  a.out = out.ref(s0);
  if (xin) a.xin = xin->ref(s0);
  a.clov.prec = prec;
  a.clov.data = prec == F64 ? c->C64[p].p : prec == F32 ? c->C32[p].p : c->C16[p].p;
  a.clov.scale = prec == F16 ? c->C16s[p].as<float>() : nullptr;
  a.slots = slot_table(w, c->g.T, s0, prec, mask);
  if (epi == EPI_INV || epi == EPI_INV_SUB) a.slots.ainv_common = common_ainv(w, s0, n, prec, &a.slots.ainv_common_scale);
  a.sratio = w.sratio;
  a.red = reduce_ref(w, s0, red, fin, inner_mask);
  if (wv) a.red.w = wv->ref(s0);
  a.nslots = n;
  hipEvent_t ev = nullptr;
  DP_TRY(timing_begin(c, &ev));
  int nparts = 0;
  DP_HIP(c, launch_hop(a, c->stream, &nparts));
  if (c->timing) {
    static const char* epi_names[] = {"hop", "inv", "diag", "sub", "invsub"};
    double bytes, flops;
    hop_cost(c, prec, epi, red, active_slots(c, mask, n), &bytes, &flops);
    std::string name = std::string("hop_") + prec_name(prec) + "_" + epi_names[epi] + (dag ? "_dag" : "");
    DP_TRY(timing_end(c, ev, name, bytes, flops));
  }
  if (red != RED_NONE) {
    const int nv = red_values(red);
    DP_TRY(timing_begin(c, &ev));
    DP_HIP(c, launch_finalize(a.red, nv, nparts, n, a.slots.mask, c->stream));
    DP_TRY(timing_end(c, ev, "finalize", 0.0, 0.0));
  }
  return DP_OK;
}

int blas(dp_ctx* c, Workspace& w, int s0, int n, int op, int prec, const int* mask,
         std::initializer_list<const Field*> v, int fin, int* inner_mask) {
  BlasArgs a;
  a.g = c->g;
  a.nslots = n;
  a.prec = prec;
  a.mask = mask ? mask + s0 : nullptr;
  a.sc = w.sc.as<SlotScalars>() + s0;
  a.slot_scale = w.slot_scale.as<double>() + s0;
  int k = 0;
  for (const Field* f : v) {
    if (f) a.v[k] = f->ref(s0);
    ++k;
  }
  a.red = reduce_ref(w, s0, RED_NONE, fin, inner_mask);
  hipEvent_t ev = nullptr;
  DP_TRY(timing_begin(c, &ev));
  DP_HIP(c, launch_blas(op, a, c->stream));
  if (c->timing) {
    // vectors read + written per site and slot
    static const int nvec[] = {1, 2, 5, 4, 3, 7, 6, 3, 2, 3, 3, 1, 2, 8};
    static_assert(sizeof(nvec) / sizeof(nvec[0]) == OP_BICG_XRP + 1, "one entry per vector op");
    const double b = prec == F64 ? 8.0 : prec == F32 ? 4.0 : 2.0;
    const double bytes = (double)c->g.Vh * active_slots(c, mask, n) * nvec[op] * 24 * b;
    DP_TRY(timing_end(c, ev, std::string("blas_") + prec_name(prec) + "_" + std::to_string(op), bytes, 0.0));
  }
  return DP_OK;
}

int schur(dp_ctx* c, Workspace& w, int s0, int n, int prec, int dag, const Field& in, const Field& to, const Field& out,
          const int* mask, int red, int fin, const Field* wv, int* inner_mask) {
  DP_TRY(hop(c, w, s0, n, prec, 1, dag, EPI_INV, 0.0, in, to, nullptr, mask));
  DP_TRY(hop(c, w, s0, n, prec, 0, dag, EPI_DIAG, -1.0, to, out, &in, mask, red, fin, wv, inner_mask));
  return DP_OK;
}

}  // namespace rt
}  // namespace dp

using namespace dp::rt;

dp_ctx::~dp_ctx() {
  for (auto& q : pending) {
    (void)hipEventDestroy(q.a);
    (void)hipEventDestroy(q.b);
  }
  for (auto e : ev_free) (void)hipEventDestroy(e);
  for (auto* m : masses) delete m;
  dp::sap_free(sap);
  if (stream) (void)hipStreamDestroy(stream);
}

namespace {

int check_state(dp_ctx* c) {
  if (!c->have_U[F64]) return fail(c, DP_ERR_BAD_STATE, "gauge field not set");
  return DP_OK;
}

// the cached inverses depend on links and clover; a batch holds pointers to them
int drop_masses(dp_ctx* c) {
  if (c->solve_batch) {  // the batch dp_solve keeps between calls
    dp_batch_close(c->solve_batch);
    c->solve_batch = nullptr;
  }
  if (c->open_batches > 0) return fail(c, DP_ERR_BAD_STATE, "a batch is open on this context");
  for (auto* m : c->masses) delete m;
  c->masses.clear();
  c->apply_key.clear();
  return DP_OK;
}

// zero clover (c_sw = 0) in every precision
int clover_zero(dp_ctx* c) {
  const Geom& g = c->g;
  for (int p = 0; p < 2; ++p) {
    DP_HIP(c, c->C64[p].reserve((size_t)g.Vp * clover_site_bytes(F64)));
    DP_HIP(c, c->C32[p].reserve((size_t)g.Vp * clover_site_bytes(F32)));
    DP_HIP(c, c->C16[p].reserve((size_t)g.Vp * clover_site_bytes(F16)));
    DP_HIP(c, c->C16s[p].reserve((size_t)g.Vp * sizeof(float)));
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

// Udev == nullptr sets unit links
int set_gauge_common(dp_ctx* c, const double2* Udev, hipStream_t st) {
  DP_TRY(drop_masses(c));
  c->sf = false;
  c->ct_tilde = 1.0;
  const Geom& g = c->g;
  for (int prec = 0; prec < 3; ++prec) {
    for (int p = 0; p < 2; ++p) DP_HIP(c, c->U[prec][p].reserve((size_t)g.Vp * link_site_bytes(prec)));
    void* dst[2] = {c->U[prec][0].p, c->U[prec][1].p};
    DP_HIP(c, launch_gauge_reorder(g, Udev, dst, prec, st));
    c->have_U[prec] = true;
  }
  DP_HIP(c, hipStreamSynchronize(st));
  c->clover_kind = 0;
  c->csw = 0.0;
  return clover_zero(c);
}

// Schroedinger functional: the clover term of the interior built on the
// padded lattice (the boundary links in its first and last timeslices), plus
// (ct_tilde - 1) on the diagonal next to the boundaries; csw = 0 gives the
// counterterm alone.
int clover_sf(dp_ctx* c, double csw) {
  const Geom& g = c->g;
  Geom gp = g;
  gp.T = g.T + 2;
  gp.Vh = gp.T * gp.Vsh;
  gp.Vp = gp.Vh;
  DevBuf Up[2], Cp[2];
  for (int p = 0; p < 2; ++p) {
    DP_HIP(c, Up[p].reserve((size_t)gp.Vp * link_site_bytes(F64)));
    DP_HIP(c, Cp[p].reserve((size_t)gp.Vp * clover_site_bytes(F64)));
  }
  void* up[2] = {Up[0].p, Up[1].p};
  DP_HIP(c, launch_gauge_reorder(gp, c->sf_ext.as<double2>(), up, F64, c->stream));
  double2* cp[2] = {Cp[0].as<double2>(), Cp[1].as<double2>()};
  if (csw != 0.0) {
    const double2* u64[2] = {Up[0].as<double2>(), Up[1].as<double2>()};
    DP_HIP(c, launch_clover_build(gp, u64, csw, cp, c->stream));
  } else {
    for (int p = 0; p < 2; ++p) DP_HIP(c, hipMemsetAsync(Cp[p].p, 0, Cp[p].bytes, c->stream));
  }
  const double2* cpc[2] = {cp[0], cp[1]};
  double2* C[2] = {c->C64[0].as<double2>(), c->C64[1].as<double2>()};
  DP_HIP(c, launch_clover_sf_interior(g, gp, cpc, c->ct_tilde - 1.0, C, c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));  // the temporaries are freed on return
  return DP_OK;
}

}  // namespace

namespace {
int scratch_setup(dp_ctx* c);
}  // namespace

// ===================================================================== C ABI

extern "C" {

int dp_create(const int dims[4], int bc_t, int device, dp_ctx** out) {
  if (!out || !dims) return DP_ERR_INVALID_ARG;
  *out = nullptr;
  for (int k = 0; k < 4; ++k)
    if (dims[k] < 2 || dims[k] % 2) return DP_ERR_INVALID_ARG;
  if (bc_t != 1 && bc_t != -1 && bc_t != 0) return DP_ERR_INVALID_ARG;
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
  // Component stride of the structure-of-arrays fields.  With a stride of Vh
  // the arrays of one site start at the same address modulo a large power of
  // two (24^3x48: 81 x 64 KB); padding it by an odd multiple of 32 sites was
  // measured on MI355X to change nothing (the caches hash the address), so it
  // stays Vh.  Tuning knob: DP_PAD = 1 pads.
  g.Vp = env_pad() ? ((g.Vh + 63) / 64) * 64 + 32 : g.Vh;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return DP_ERR_DEVICE;
  }
  c->alpha.assign(g.T, 1.0);
  // dp_apply_dev_noalloc: this device's scratch address and the host staging
  // of its per-slot tables (ratio tables, T ones, masses, unit scales, pointers)
  c->na_host.assign((size_t)(4 * g.T + 2 + 4) * DP_NOALLOC_MAX_RHS + g.T, 0.0);
  for (int q = 0; q < 3; ++q) c->ws_noalloc.h_ainv[q].assign(DP_NOALLOC_MAX_RHS, nullptr);
  c->ws_noalloc.h_ainv_scale.assign(DP_NOALLOC_MAX_RHS, nullptr);
  const double* none[3] = {nullptr, nullptr, nullptr};
  int rc = scratch_setup(c);
  if (rc == DP_OK) rc = upload_space(c, none);
  if (rc == DP_OK) rc = set_gauge_common(c, nullptr, c->stream);  // unit links, no clover
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
  if (c->solve_batch) {
    dp_batch_close(c->solve_batch);
    c->solve_batch = nullptr;
  }
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
  if (stream) DP_HIP(c, hipStreamSynchronize((hipStream_t)stream));
  return set_gauge_common(c, static_cast<const double2*>(U), c->stream);
}

int dp_set_gauge_sf(dp_ctx* c, const double* U_ext, double ct_tilde) {
  if (!c || !U_ext || !std::isfinite(ct_tilde)) return fail(c, DP_ERR_INVALID_ARG, "bad argument");
  if (c->bc_t != 0) return fail(c, DP_ERR_BAD_STATE, "the Schroedinger functional needs a ctx with bc_t = 0");
  DP_HIP(c, hipSetDevice(c->device));
  const Geom& g = c->g;
  const size_t per_t = (size_t)2 * g.Vsh * 4 * 9;  // double2 per timeslice
  DP_HIP(c, c->sf_ext.reserve(sizeof(double2) * per_t * (g.T + 2)));
  DP_HIP(c, hipMemcpyAsync(c->sf_ext.p, U_ext, sizeof(double2) * per_t * (g.T + 2), hipMemcpyHostToDevice,
                           c->stream));
  // the interior links, as dp_set_gauge (which clears the SF state: set it after)
  DP_TRY(set_gauge_common(c, c->sf_ext.as<double2>() + per_t, c->stream));
  c->sf = true;
  c->ct_tilde = ct_tilde;
  // the counterterm applies from now on (with c_sw = 0 until dp_set_clover)
  DP_TRY(clover_sf(c, 0.0));
  DP_TRY(clover_convert_all(c));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  c->clover_kind = ct_tilde != 1.0 ? 1 : 0;
  return DP_OK;
}

int dp_sf_wall_sources(dp_ctx* c, int side, int c0, int ncols, void* eta, void* stream) {
  if (!c || !eta) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  if (side != 0 && side != 1) return fail(c, DP_ERR_INVALID_ARG, "side must be 0 (x0 = 0) or 1 (x0 = T + 1)");
  if (c0 < 0 || ncols < 1 || c0 + ncols > 12) return fail(c, DP_ERR_INVALID_ARG, "need 0 <= c0 and c0 + ncols <= 12");
  if (!c->sf) return fail(c, DP_ERR_BAD_STATE, "no Schroedinger-functional links set (dp_set_gauge_sf)");
  DP_HIP(c, hipSetDevice(c->device));
  if (stream) DP_HIP(c, hipStreamSynchronize((hipStream_t)stream));
  // the padded timeslice next to the boundary: x0 = 0 or x0 = T
  const size_t per_t = (size_t)2 * c->g.Vsh * 4 * 9;
  const double2* Ut = c->sf_ext.as<double2>() + (side == 0 ? 0 : per_t * c->g.T);
  DP_HIP(c, launch_sf_wall_sources(c->g, Ut, side, c0, ncols, static_cast<double2*>(eta), c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  return DP_OK;
}

int dp_set_clover(dp_ctx* c, double csw) {
  if (!c || !std::isfinite(csw)) return fail(c, DP_ERR_INVALID_ARG, "bad argument");
  DP_HIP(c, hipSetDevice(c->device));
  DP_TRY(check_state(c));
  DP_TRY(drop_masses(c));
  if (c->sf) {
    DP_TRY(clover_sf(c, csw));
    DP_TRY(clover_convert_all(c));
    c->clover_kind = 1;
  } else if (csw == 0.0) {
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
  DP_TRY(drop_masses(c));
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

int dp_set_alpha_space(dp_ctx* c, const double* a1, const double* a2, const double* a3) {
  if (!c) return DP_ERR_INVALID_ARG;
  const double* a[3] = {a1, a2, a3};
  const int Ls[3] = {c->g.L1, c->g.L2, c->g.L3};
  for (int k = 0; k < 3; ++k)
    if (a[k])
      for (int x = 0; x < Ls[k]; ++x)
        if (!(a[k][x] > 0) || !std::isfinite(a[k][x]) || !std::isfinite(1.0 / a[k][x]))
          return fail(c, DP_ERR_INVALID_ARG, "spatial profiles must be finite and positive");
  DP_HIP(c, hipSetDevice(c->device));
  if (c->solve_batch) {  // the batch dp_solve keeps between calls
    dp_batch_close(c->solve_batch);
    c->solve_batch = nullptr;
  }
  if (c->open_batches > 0) return fail(c, DP_ERR_BAD_STATE, "a batch is open on this context");
  return upload_space(c, a);
}

}  // extern "C"

namespace {

int check_apply_flags(dp_ctx* c, int flags) {
  if (flags & ~(DP_PRECOND | DP_DAGGER | DP_HOP_ONLY | DP_APPLY_SCHUR | DP_APPLY_F32 | DP_APPLY_F16))
    return fail(c, DP_ERR_INVALID_ARG, "unknown flag");
  if ((flags & DP_APPLY_F32) && (flags & DP_APPLY_F16)) return fail(c, DP_ERR_INVALID_ARG, "two precisions");
  if ((flags & DP_HOP_ONLY) && (flags & DP_APPLY_SCHUR)) return fail(c, DP_ERR_INVALID_ARG, "hop-only Schur");
  return DP_OK;
}

int apply_run(dp_ctx* c, Workspace& w, const double2* in, double2* out, int n, int flags);

// The operator on n device spinors in host layout (in and out may not alias),
// enqueued on the ctx stream.  Slot k has the mass Ms[k] and the time profile
// alphas[k * T ..] (null: the ctx's for every slot).  The per-slot tables are
// uploaded only when the masses, the profiles, the precondition flag or the
// slot count changed.
int apply_core(dp_ctx* c, const double2* in, double2* out, int n, int flags, const double* Ms = nullptr,
               const double* alphas = nullptr) {
  const int prec = (flags & DP_APPLY_F32) ? F32 : (flags & DP_APPLY_F16) ? F16 : F64;
  Workspace& w = c->ws_apply;
  DP_TRY(ensure_ws(c, w, n, prec));
  w.sratio = (flags & DP_PRECOND) && c->has_space ? space_ratios(c, 1) : nullptr;
  const Geom& g = c->g;
  std::vector<MassEntry*> me(n, nullptr);
  for (int k = 0; k < n; ++k) DP_TRY(mass_entry(c, Ms ? Ms[k] : c->M, &me[k]));
  std::vector<double> key;
  key.push_back((double)n);
  key.push_back((flags & DP_PRECOND) ? 1.0 : 0.0);
  key.push_back((double)(uintptr_t)w.ratio.p);
  for (int k = 0; k < n; ++k) {
    key.push_back(me[k]->M);
    key.push_back((double)(uintptr_t)me[k]);
  }
  if (flags & DP_PRECOND) {
    if (alphas) key.insert(key.end(), alphas, alphas + (size_t)n * g.T);
    else key.insert(key.end(), c->alpha.begin(), c->alpha.end());
  }
  if (key != c->apply_key) {
    std::vector<double> ones(g.T, 1.0), all((size_t)4 * g.T * n), m4(n), one(n, 1.0);
    for (int k = 0; k < n; ++k) {
      const double* a = !(flags & DP_PRECOND) ? ones.data() : alphas ? alphas + (size_t)k * g.T : c->alpha.data();
      ratio_tables(g.T, c->bc_t, a, all.data() + (size_t)4 * g.T * k);
      m4[k] = 4.0 + me[k]->M;
    }
    DP_TRY(h2d(c, w.ratio.p, all.data(), sizeof(double) * all.size()));
    DP_TRY(h2d(c, w.m4.p, m4.data(), sizeof(double) * n));
    DP_TRY(h2d(c, w.slot_scale.p, one.data(), sizeof(double) * n));
    for (int q = 0; q < 3; ++q) {
      std::vector<const void*> v(n);
      for (int k = 0; k < n; ++k) v[k] = q == 0 ? me[k]->a64.p : q == 1 ? me[k]->a32.p : me[k]->a16.p;
      DP_TRY(h2d(c, w.ainv_ptr[q].p, v.data(), sizeof(void*) * n));
      std::copy(v.begin(), v.end(), w.h_ainv[q].begin());
    }
    std::vector<const float*> s16(n);
    for (int k = 0; k < n; ++k) s16[k] = me[k]->s16.as<float>();
    DP_TRY(h2d(c, w.ainv_scale_ptr.p, s16.data(), sizeof(float*) * n));
    std::copy(s16.begin(), s16.end(), w.h_ainv_scale.begin());
    c->apply_key = key;
  }
  return apply_run(c, w, in, out, n, flags);
}

// The launches of the operator on n device spinors (host layout) with the
// per-slot tables of w already in place: import into parity fields, the
// inner-precision copies, the hop kernels (full, Schur or hop-only operator),
// the FP64 copies and the export.
int apply_run(dp_ctx* c, Workspace& w, const double2* in, double2* out, int n, int flags) {
  const int prec = (flags & DP_APPLY_F32) ? F32 : (flags & DP_APPLY_F16) ? F16 : F64;
  const int dag = (flags & DP_DAGGER) ? 1 : 0;
  const Geom& g = c->g;
  const long col = 2L * g.Vh * 12;  // double2 per column
  DP_HIP(c, launch_spinor_import(g, in, n, col, 0, w.eta_e.ref(), nullptr, nullptr, c->stream));
  DP_HIP(c, launch_spinor_import(g, in, n, col, 1, w.eta_o.ref(), nullptr, nullptr, c->stream));
  // inputs in the compute precision: even in r, odd in s (Vh sites each)
  const Field* ie = &w.eta_e;
  const Field* io = &w.eta_o;
  const Field* oe = &w.b64;
  const Field* oo = &w.to64;
  if (prec != F64) {
    DP_TRY(blas(c, w, 0, n, OP_SCALE_COPY, prec, nullptr, {&w.r, &w.eta_e}));
    DP_TRY(blas(c, w, 0, n, OP_SCALE_COPY, prec, nullptr, {&w.s, &w.eta_o}));
    ie = &w.r;
    io = &w.s;
    oe = &w.v;
    oo = &w.t;
  }
  if (flags & DP_HOP_ONLY) {
    DP_TRY(hop(c, w, 0, n, prec, 0, dag, EPI_HOP, 0.0, *io, *oe, nullptr, nullptr));
    DP_TRY(hop(c, w, 0, n, prec, 1, dag, EPI_HOP, 0.0, *ie, *oo, nullptr, nullptr));
  } else if (flags & DP_APPLY_SCHUR) {
    DP_TRY(schur(c, w, 0, n, prec, dag, *ie, w.to, *oe, nullptr, RED_NONE, FIN_NONE));
    DP_TRY(blas(c, w, 0, n, OP_ZERO, prec, nullptr, {oo}));
  } else {
    DP_TRY(hop(c, w, 0, n, prec, 0, dag, EPI_DIAG, 1.0, *io, *oe, ie, nullptr));
    DP_TRY(hop(c, w, 0, n, prec, 1, dag, EPI_DIAG, 1.0, *ie, *oo, io, nullptr));
  }
  if (prec != F64) {
    DP_TRY(blas(c, w, 0, n, OP_TO64, prec, nullptr, {&w.b64, oe}));
    DP_TRY(blas(c, w, 0, n, OP_TO64, prec, nullptr, {&w.to64, oo}));
  }
  DP_HIP(c, launch_spinor_export(g, w.b64.ref(), w.to64.ref(), n, nullptr, nullptr, out, col, c->stream));
  return DP_OK;
}

// ------------------------------------------------------------ no-alloc apply
//
// dp_apply_dev_noalloc keeps every temporary of dp_apply_dev (the parity
// fields, their inner-precision copies and the per-slot tables) in `scratch`,
// a static device array the loader places on every GPU the library runs on.
// Host code never passes the array's name anywhere: it is a host-side
// stand-in for the symbol.  The device address comes from
// hipGetSymbolAddress, once per device with that device current (at
// dp_create), and only that address is used.

__device__ __align__(256) unsigned char scratch[DP_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;  // device -> address of its copy of `scratch`

int scratch_setup(dp_ctx* c) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(c->device);
  if (it == g_scratch_addr.end()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)", __LINE__);
    if (!ptr) return fail(c, DP_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned a null address");
    it = g_scratch_addr.emplace(c->device, ptr).first;
  }
  c->scratch_dev = it->second;
  return DP_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets in the scratch for n right-hand sides at precision prec.
struct NoallocLayout {
  size_t f64[5];  // eta_e, eta_o, b64, to64, to (to: FP64 only)
  size_t in[5], in_scale[5];  // r, s, v, t, to in the inner precision (and FP16 scales)
  size_t ratio, m4, sscale, ainv[3], ainv_scale, end;
};

NoallocLayout noalloc_layout(const Geom& g, int n, int prec) {
  NoallocLayout L{};
  size_t off = 0;
  const size_t f64 = align256((size_t)n * g.Vp * spinor_site_bytes(F64));
  for (int k = 0; k < 5; ++k) {
    L.f64[k] = off;
    if (k < 4 || prec == F64) off += f64;
  }
  if (prec != F64) {
    const size_t fin = align256((size_t)n * g.Vp * spinor_site_bytes(prec));
    const size_t fsc = prec == F16 ? align256((size_t)n * g.Vp * sizeof(float)) : 0;
    for (int k = 0; k < 5; ++k) {
      L.in[k] = off;
      off += fin;
      L.in_scale[k] = off;
      off += fsc;
    }
  }
  L.ratio = off;
  off += align256(sizeof(double) * 4 * g.T * n);
  L.m4 = off;
  off += align256(sizeof(double) * n);
  L.sscale = off;
  off += align256(sizeof(double) * n);
  for (int q = 0; q < 3; ++q) {
    L.ainv[q] = off;
    off += align256(sizeof(void*) * n);
  }
  L.ainv_scale = off;
  off += align256(sizeof(float*) * n);
  L.end = off;
  return L;
}

void field_view(Field& f, const Geom& g, int prec, int n, char* data, char* scale) {
  f.prec = prec;
  f.nslots = n;
  f.slot_stride = (long)g.Vp * (prec == F64 ? 12 : prec == F32 ? 6 : 3);
  f.scale_stride = prec == F16 ? g.Vp : 0;
  f.data.view(data, (size_t)n * g.Vp * spinor_site_bytes(prec));
  if (prec == F16) f.scale.view(scale, (size_t)n * g.Vp * sizeof(float));
  else f.scale.view(nullptr, 0);
}

}  // namespace

extern "C" {

int dp_apply_dev_noalloc(dp_ctx* c, const void* in, void* out, int nrhs, int flags, void* stream) {
  if (!c || !in || !out) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  if (nrhs <= 0 || nrhs > DP_NOALLOC_MAX_RHS) return fail(c, DP_ERR_INVALID_ARG, "nrhs must be in [1, DP_NOALLOC_MAX_RHS]");
  DP_TRY(check_apply_flags(c, flags));
  const Geom& g = c->g;
  const size_t bytes = (size_t)nrhs * 2 * g.Vh * 12 * sizeof(double2);
  const char* a = static_cast<const char*>(in);
  const char* b = static_cast<const char*>(out);
  if (a < b + bytes && b < a + bytes) return fail(c, DP_ERR_INVALID_ARG, "in and out overlap");
  if (!c->scratch_dev) return fail(c, DP_ERR_BAD_STATE, "no scratch address for this device");
  const int prec = (flags & DP_APPLY_F32) ? F32 : (flags & DP_APPLY_F16) ? F16 : F64;
  const NoallocLayout lay = noalloc_layout(g, nrhs, prec);
  if (lay.end > (size_t)DP_NOALLOC_SCRATCH_BYTES) {
    char msg[200];
    snprintf(msg, sizeof msg, "%d right-hand sides of this lattice need %zu bytes of scratch; it holds %zu", nrhs,
             lay.end, (size_t)DP_NOALLOC_SCRATCH_BYTES);
    return fail(c, DP_ERR_INVALID_ARG, msg);
  }
  DP_HIP(c, hipSetDevice(c->device));
  DP_TRY(check_state(c));
  // the inverse clover of the current mass is only looked up, never built
  MassEntry* me = nullptr;
  for (auto* m : c->masses)
    if (m->M == c->M) me = m;
  if (!me && (flags & DP_APPLY_SCHUR))
    return fail(c, DP_ERR_BAD_STATE,
                "the inverse clover of the current mass is not built: call dp_apply_dev (or a solve) with this "
                "mass once before");
  if (stream) DP_HIP(c, hipStreamSynchronize((hipStream_t)stream));
  // views into the scratch
  Workspace& w = c->ws_noalloc;
  char* base = static_cast<char*>(c->scratch_dev);
  Field* f64[5] = {&w.eta_e, &w.eta_o, &w.b64, &w.to64, &w.to};
  for (int k = 0; k < 5; ++k)
    if (k < 4 || prec == F64) field_view(*f64[k], g, F64, nrhs, base + lay.f64[k], nullptr);
  if (prec != F64) {
    Field* fin[5] = {&w.r, &w.s, &w.v, &w.t, &w.to};
    for (int k = 0; k < 5; ++k) field_view(*fin[k], g, prec, nrhs, base + lay.in[k], base + lay.in_scale[k]);
  }
  w.ratio.view(base + lay.ratio, sizeof(double) * 4 * g.T * nrhs);
  w.m4.view(base + lay.m4, sizeof(double) * nrhs);
  w.slot_scale.view(base + lay.sscale, sizeof(double) * nrhs);
  for (int q = 0; q < 3; ++q) w.ainv_ptr[q].view(base + lay.ainv[q], sizeof(void*) * nrhs);
  w.ainv_scale_ptr.view(base + lay.ainv_scale, sizeof(float*) * nrhs);
  w.nslots = nrhs;
  w.prec = prec;
  w.sratio = (flags & DP_PRECOND) && c->has_space ? space_ratios(c, 1) : nullptr;
  // per-slot tables, staged in the host area sized at dp_create
  double* h = c->na_host.data();
  const double* alpha = (flags & DP_PRECOND) ? c->alpha.data() : nullptr;
  for (int k = 0; k < nrhs; ++k) {
    double* rt = h + (size_t)4 * g.T * k;
    if (alpha) {
      ratio_tables(g.T, c->bc_t, alpha, rt);
    } else {
      double* ones = h + (size_t)4 * g.T * nrhs;  // T ones after the tables
      for (int t = 0; t < g.T; ++t) ones[t] = 1.0;
      ratio_tables(g.T, c->bc_t, ones, rt);
    }
  }
  double* m4 = h + (size_t)4 * g.T * nrhs + g.T;
  double* one = m4 + nrhs;
  const void** ptrs = reinterpret_cast<const void**>(one + nrhs);  // 4 nrhs pointers
  for (int k = 0; k < nrhs; ++k) {
    m4[k] = 4.0 + c->M;
    one[k] = 1.0;
    ptrs[k] = me ? me->a64.p : nullptr;
    ptrs[nrhs + k] = me ? me->a32.p : nullptr;
    ptrs[2 * nrhs + k] = me ? me->a16.p : nullptr;
    ptrs[3 * nrhs + k] = me ? me->s16.p : nullptr;
    for (int q = 0; q < 3; ++q) w.h_ainv[q][k] = ptrs[q * nrhs + k];
    w.h_ainv_scale[k] = static_cast<const float*>(ptrs[3 * nrhs + k]);
  }
  for (int k = nrhs; k < (int)w.h_ainv_scale.size(); ++k) {  // entries beyond this call's slots
    for (int q = 0; q < 3; ++q) w.h_ainv[q][k] = nullptr;
    w.h_ainv_scale[k] = nullptr;
  }
  DP_HIP(c, hipMemcpyAsync(w.ratio.p, h, sizeof(double) * 4 * g.T * nrhs, hipMemcpyHostToDevice, c->stream));
  DP_HIP(c, hipMemcpyAsync(w.m4.p, m4, sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
  DP_HIP(c, hipMemcpyAsync(w.slot_scale.p, one, sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
  for (int q = 0; q < 3; ++q)
    DP_HIP(c, hipMemcpyAsync(w.ainv_ptr[q].p, ptrs + q * nrhs, sizeof(void*) * nrhs, hipMemcpyHostToDevice,
                             c->stream));
  DP_HIP(c, hipMemcpyAsync(w.ainv_scale_ptr.p, ptrs + 3 * nrhs, sizeof(float*) * nrhs, hipMemcpyHostToDevice,
                           c->stream));
  // no launch timing here (it creates events and records into host maps)
  const bool timing = c->timing;
  c->timing = false;
  const int rc = apply_run(c, w, static_cast<const double2*>(in), static_cast<double2*>(out), nrhs, flags);
  c->timing = timing;
  DP_TRY(rc);
  DP_HIP(c, hipStreamSynchronize(c->stream));
  return DP_OK;
}

int dp_apply(dp_ctx* c, const double* in, double* out, int flags) {
  TraceRange tr("dp_apply");
  if (!c || !in || !out) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  DP_TRY(check_apply_flags(c, flags));
  DP_HIP(c, hipSetDevice(c->device));
  DP_TRY(check_state(c));
  const Geom& g = c->g;
  const size_t bytes = (size_t)2 * g.Vh * 12 * sizeof(double2);
  DP_HIP(c, c->scratch_aos.reserve(2 * bytes));
  double2* din = c->scratch_aos.as<double2>();
  double2* dout = din + (size_t)2 * g.Vh * 12;
  DP_HIP(c, hipMemcpyAsync(din, in, bytes, hipMemcpyHostToDevice, c->stream));
  DP_TRY(apply_core(c, din, dout, 1, flags));
  DP_HIP(c, hipMemcpyAsync(out, dout, bytes, hipMemcpyDeviceToHost, c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  DP_TRY(timing_harvest(c));
  return DP_OK;
}

int dp_apply_dev(dp_ctx* c, const void* in, void* out, int nrhs, int flags, void* stream) {
  TraceRange tr("dp_apply_dev");
  if (!c || !in || !out) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  if (nrhs <= 0) return fail(c, DP_ERR_INVALID_ARG, "nrhs must be positive");
  DP_TRY(check_apply_flags(c, flags));
  const Geom& g = c->g;
  const size_t bytes = (size_t)nrhs * 2 * g.Vh * 12 * sizeof(double2);
  const char* a = static_cast<const char*>(in);
  const char* b = static_cast<const char*>(out);
  if (a < b + bytes && b < a + bytes) return fail(c, DP_ERR_INVALID_ARG, "in and out overlap");
  DP_HIP(c, hipSetDevice(c->device));
  DP_TRY(check_state(c));
  if (stream) DP_HIP(c, hipStreamSynchronize((hipStream_t)stream));
  DP_TRY(apply_core(c, static_cast<const double2*>(in), static_cast<double2*>(out), nrhs, flags));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  DP_TRY(timing_harvest(c));
  return DP_OK;
}

int dp_apply_dev_slots(dp_ctx* c, const void* in, void* out, int nrhs, int flags, const double* M,
                       const double* alpha, void* stream) {
  if (!c || !in || !out) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  if (nrhs <= 0) return fail(c, DP_ERR_INVALID_ARG, "nrhs must be positive");
  DP_TRY(check_apply_flags(c, flags));
  const Geom& g = c->g;
  if (M)
    for (int k = 0; k < nrhs; ++k)
      if (!std::isfinite(M[k])) return fail(c, DP_ERR_INVALID_ARG, "masses must be finite");
  if (alpha)
    for (long k = 0; k < (long)nrhs * g.T; ++k)
      if (!(alpha[k] > 0) || !std::isfinite(alpha[k]) || !std::isfinite(1.0 / alpha[k]))
        return fail(c, DP_ERR_INVALID_ARG, "alpha must be finite and positive");
  const size_t bytes = (size_t)nrhs * 2 * g.Vh * 12 * sizeof(double2);
  const char* a = static_cast<const char*>(in);
  const char* b = static_cast<const char*>(out);
  if (a < b + bytes && b < a + bytes) return fail(c, DP_ERR_INVALID_ARG, "in and out overlap");
  DP_HIP(c, hipSetDevice(c->device));
  DP_TRY(check_state(c));
  if (stream) DP_HIP(c, hipStreamSynchronize((hipStream_t)stream));
  DP_TRY(apply_core(c, static_cast<const double2*>(in), static_cast<double2*>(out), nrhs, flags, M, alpha));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  DP_TRY(timing_harvest(c));
  return DP_OK;
}

int dp_point_sources(dp_ctx* c, const int site[4], int c0, int ncols, void* eta, void* stream) {
  if (!c || !site || !eta) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  if (c0 < 0 || ncols < 1 || c0 + ncols > 12) return fail(c, DP_ERR_INVALID_ARG, "need 0 <= c0 and c0 + ncols <= 12");
  for (int k = 0; k < 4; ++k)
    if (site[k] < 0 || site[k] >= c->dims[k]) return fail(c, DP_ERR_INVALID_ARG, "site outside the lattice");
  DP_HIP(c, hipSetDevice(c->device));
  if (stream) DP_HIP(c, hipStreamSynchronize((hipStream_t)stream));
  DP_HIP(c, launch_point_sources(c->g, site, c0, ncols, static_cast<double2*>(eta), c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  return DP_OK;
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

int dp_get_timing_samples(dp_ctx* c, const char* name, float* ms, int max, int* count) {
  if (!c || !name || !count || max < 0 || (max > 0 && !ms)) return fail(c, DP_ERR_INVALID_ARG, "bad argument");
  DP_HIP(c, hipSetDevice(c->device));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  DP_TRY(timing_harvest(c));
  auto it = c->kstats.find(name);
  const int n = it == c->kstats.end() ? 0 : (int)it->second.samples.size();
  for (int k = 0; k < std::min(n, max); ++k) ms[k] = it->second.samples[k];
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
  for (int p = 0; p < 3; ++p) b += 2 * Vh * (long long)link_site_bytes(p);    // links
  for (int p = 0; p < 3; ++p) b += 2 * Vh * (long long)clover_site_bytes(p);  // clover
  b += 2 * Vh * 4;                                                            // FP16 clover scales
  const long long mass = Vh * (long long)(clover_site_bytes(0) + clover_site_bytes(1) + clover_site_bytes(2) + 4);
  b += new_masses * mass;
  const long long f64 = Vh * 192;
  const long long fin = Vh * (long long)(spinor_site_bytes(precision) + spinor_scale_bytes(precision));
  const long long fx = Vh * (long long)spinor_site_bytes(precision == 2 ? 1 : precision);
  b += nrhs * (7 * f64 + 7 * fin + fx);
  return b;
}

}  // extern "C"
