// The batch of slots: the solve of the paper's preconditioned system
// (eq. linsysprec) for many right-hand sides at once, each slot with its own
// source, mass, alpha profile and residue, entering and leaving on its own
// (continuous batching).  dp_solve is one batch filled with the columns of a
// request.
//
// Per slot:
//   admit   eta' = alpha eta (eq. redeft), b = eta'_e - H_eo A_oo^-1 eta'_o,
//           x = 0, then an outer step;
//   outer   x += |r| e (when an inner result exists), r = b - Mhat' x in FP64,
//           the stopping rule |r| <= r_target |eta'| (eq. stopping); else a new
//           inner solve on r/|r| in the inner precision, to relative tolerance
//           max(delta, r_target |eta'| / 2|r|);
//   inner   BiCGStab or CGNR iterations on all slots of the inner mask; a slot
//           leaves the mask on the device (converged, breakdown, max_iter,
//           non-finite), so k iterations run without host round trips and are
//           replayed from a captured hipGraph;
//   finish  S'_o = A_oo^-1 (eta'_o - H_oe S'_e), S = S'/alpha and
//           C_PP = -sum |S|^2 per timeslice (restoration, eq. backcorrection).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "runtime.h"

using namespace dp;
using namespace dp::rt;

dp_batch::~dp_batch() {
  if (graph) (void)hipGraphExecDestroy(graph);
}

namespace {

int upload_slot(dp_batch* b, int s) {
  dp_ctx* c = b->c;
  Workspace& w = b->w;
  dp_batch::Slot& sl = b->slots[s];
  const int T = c->g.T;
  std::vector<double> rt(4 * T);
  ratio_tables(T, c->bc_t, sl.alpha.data(), rt.data());
  DP_TRY(h2d(c, w.ratio.as<double>() + (size_t)s * 4 * T, rt.data(), sizeof(double) * 4 * T));
  DP_TRY(h2d(c, w.alpha.as<double>() + (size_t)s * T, sl.alpha.data(), sizeof(double) * T));
  const double m4 = 4.0 + sl.me->M;
  DP_TRY(h2d(c, w.m4.as<double>() + s, &m4, sizeof(double)));
  const void* p3[3] = {sl.me->a64.p, sl.me->a32.p, sl.me->a16.p};
  for (int k = 0; k < 3; ++k) {
    DP_TRY(h2d(c, static_cast<const void**>(w.ainv_ptr[k].p) + s, &p3[k], sizeof(void*)));
    w.h_ainv[k][s] = p3[k];
  }
  const float* s16 = sl.me->s16.as<float>();
  DP_TRY(h2d(c, static_cast<const float**>(w.ainv_scale_ptr.p) + s, &s16, sizeof(float*)));
  w.h_ainv_scale[s] = s16;
  DP_TRY(h2d(c, w.x0src.as<int>() + s, &sl.x0, sizeof(int)));
  return DP_OK;
}

// FP64 residual, stopping test and (re)start of the inner solve for the slots
// in `pend`; slots that stop are finished.
int outer_step(dp_batch* b, const std::vector<int>& pend, std::vector<int>& finished) {
  dp_ctx* c = b->c;
  Workspace& w = b->w;
  const int n = b->nslots, prec = b->prec;
  const bool cgnr = b->solver == DP_SOLVER_CGNR;
  const int* m_out = w.mask_outer.as<int>();
  double* hscale = w.h_scale.as<double>();
  double* sums = w.h_sums.as<double>();
  b->m_outer = pend;
  DP_TRY(upload_mask(c, w, w.mask_outer, b->m_outer, 1));
  bool any_prev = false;
  for (int s = 0; s < n; ++s) {
    const bool use = pend[s] && b->slots[s].has_inner;
    hscale[s] = use ? b->slots[s].scale : 0.0;
    any_prev |= use;
  }
  if (any_prev) {
    // slots without an inner result get scale 0; their x is finite (zeroed at every inner start)
    DP_HIP(c, hipMemcpyAsync(w.slot_scale.p, hscale, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    DP_TRY(blas(c, w, 0, n, OP_AXPY_SCALED, prec, m_out, {&w.x64, &w.x}));
  }
  DP_TRY(schur(c, w, 0, n, F64, 0, w.x64, w.to64, w.t64, m_out, RED_NONE, FIN_NONE));
  DP_TRY(blas(c, w, 0, n, OP_SUB64, F64, m_out, {&w.r64, &w.b64, &w.t64}, FIN_STORE));
  DP_HIP(c, hipMemcpyAsync(sums, w.out_sums.p, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  std::vector<int> start(n, 0);
  bool any_start = false;
  SlotScalars* hsc = w.h_sc.as<SlotScalars>();
  for (int s = 0; s < n; ++s) {
    if (!pend[s]) continue;
    dp_batch::Slot& h = b->slots[s];
    h.outer++;
    h.hops += 2;
    const double prev = h.res2;
    h.res2 = sums[4 * s];
    // a breakdown that left the residual where it was counts towards giving up
    if (h.has_inner && h.last_left == 2) h.stall = h.res2 < 0.99 * prev ? 0 : h.stall + 1;
    else h.stall = 0;
    if (!std::isfinite(h.res2)) {
      h.status = DP_ERR_NONFINITE;
      finished.push_back(s);
    } else if (h.res2 <= h.r * h.r * h.eta2) {
      h.status = DP_OK;
      finished.push_back(s);
    } else if (b->single && h.has_inner) {
      // one inner solve only: its own stopping rule decides; true_res reports
      // the FP64 residual of what it returned
      h.status = h.last_left == 1 ? DP_OK
                 : h.last_left == 2 ? DP_ERR_BREAKDOWN
                 : h.last_left == 4 ? DP_ERR_NONFINITE
                                    : DP_ERR_NOT_CONVERGED;
      finished.push_back(s);
    } else if (h.iters >= h.max_iter) {
      h.status = DP_ERR_NOT_CONVERGED;
      finished.push_back(s);
    } else if (h.stall >= 3) {
      h.status = DP_ERR_BREAKDOWN;
      finished.push_back(s);
    } else {
      start[s] = 1;
      any_start = true;
      h.scale = std::sqrt(h.res2);
      const double need = (b->single ? 1.0 : 0.5) * h.r * std::sqrt(h.eta2 / h.res2);
      double tol = prec == F64 || b->single ? need : std::max(need, h.delta);
      tol = std::min(tol, 0.5);
      SlotScalars& q = hsc[s];
      std::memset(&q, 0, sizeof q);
      q.tol2 = tol * tol;
      q.iters = h.iters;
      q.max_iter = h.max_iter;
      q.shadow = h.has_inner && h.last_left == 2 ? 1 : 0;
      DP_HIP(c, hipMemcpyAsync(w.sc.as<SlotScalars>() + s, &q, sizeof q, hipMemcpyHostToDevice, c->stream));
    }
  }
  if (!any_start) return DP_OK;
  for (int s = 0; s < n; ++s) hscale[s] = start[s] ? 1.0 / b->slots[s].scale : 0.0;
  DP_HIP(c, hipMemcpyAsync(w.slot_scale.p, hscale, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
  b->m_outer = start;
  DP_TRY(upload_mask(c, w, w.mask_outer, b->m_outer, 2));
  DP_TRY(blas(c, w, 0, n, OP_SCALE_COPY, prec, m_out, {&w.r, &w.r64}));
  DP_TRY(blas(c, w, 0, n, OP_BICG_INIT, prec, m_out, {&w.rh, &w.r, &w.p, &w.v, &w.x}, FIN_BICG_INIT));
  if (cgnr) {
    DP_TRY(schur(c, w, 0, n, prec, 1, w.r, w.to, w.s, m_out, RED_NORM, FIN_CG_INIT));
    DP_TRY(blas(c, w, 0, n, OP_COPY, prec, m_out, {&w.p, &w.s}));
  }
  for (int s = 0; s < n; ++s)
    if (start[s]) {
      b->slots[s].in_inner = true;
      b->slots[s].has_inner = true;
      b->slots[s].hops += cgnr ? 2 : 0;
      b->m_inner[s] = 1;
    }
  DP_TRY(upload_mask(c, w, w.mask_inner, b->m_inner, 0));
  DP_HIP(c, hipStreamSynchronize(c->stream));  // staging rows and scalars are reused next
  return DP_OK;
}

// one inner iteration for every slot in the inner mask
int inner_iteration(dp_batch* b) {
  dp_ctx* c = b->c;
  Workspace& w = b->w;
  const int n = b->nslots, prec = b->prec;
  int* mi = w.mask_inner.as<int>();
  // tuning knob: DP_BICG_FUSED = 0 takes rho from the stored residual and
  // updates the search direction in a kernel of its own (one vector sweep
  // more per iteration)
  static const bool fused = [] {
    const char* e = getenv("DP_BICG_FUSED");
    return !(e && atoi(e) == 0);
  }();
  if (b->solver == DP_SOLVER_BICGSTAB && fused) {
    // p enters as r after the start (and as the previous iteration's update)
    DP_TRY(schur(c, w, 0, n, prec, 0, w.p, w.to, w.v, mi, RED_DOT_EXT, FIN_BICG_ALPHA, &w.rh, mi));
    DP_TRY(blas(c, w, 0, n, OP_BICG_S, prec, mi, {&w.s, &w.r, &w.v}));
    DP_TRY(schur(c, w, 0, n, prec, 0, w.s, w.to, w.t, mi, RED_TS4, FIN_BICG_OMEGA_RHO, &w.rh));
    DP_TRY(blas(c, w, 0, n, OP_BICG_XRP, prec, mi, {&w.x, &w.p, &w.s, &w.r, &w.t, &w.v}, FIN_BICG_RR, mi));
  } else if (b->solver == DP_SOLVER_BICGSTAB) {
    DP_TRY(blas(c, w, 0, n, OP_BICG_P, prec, mi, {&w.p, &w.r, &w.v}));
    DP_TRY(schur(c, w, 0, n, prec, 0, w.p, w.to, w.v, mi, RED_DOT_EXT, FIN_BICG_ALPHA, &w.rh, mi));
    DP_TRY(blas(c, w, 0, n, OP_BICG_S, prec, mi, {&w.s, &w.r, &w.v}));
    DP_TRY(schur(c, w, 0, n, prec, 0, w.s, w.to, w.t, mi, RED_TS, FIN_BICG_OMEGA));
    DP_TRY(blas(c, w, 0, n, OP_BICG_XR, prec, mi, {&w.x, &w.p, &w.s, &w.r, &w.t, &w.rh}, FIN_BICG_RHO, mi));
  } else {
    DP_TRY(schur(c, w, 0, n, prec, 0, w.p, w.to, w.v, mi, RED_NORM, FIN_CG_ALPHA));
    DP_TRY(blas(c, w, 0, n, OP_CG_XR, prec, mi, {&w.x, &w.p, &w.r, &w.v}, FIN_RR));
    DP_TRY(schur(c, w, 0, n, prec, 1, w.r, w.to, w.s, mi, RED_NORM, FIN_CG_BETA, nullptr, mi));
    DP_TRY(blas(c, w, 0, n, OP_CG_P, prec, mi, {&w.p, &w.s}));
  }
  return DP_OK;
}

// k inner iterations: replayed from a captured graph unless launches are timed
int inner_iterations(dp_batch* b, int k) {
  dp_ctx* c = b->c;
  if (c->timing || !c->use_graphs) {
    for (int j = 0; j < k; ++j) DP_TRY(inner_iteration(b));
    return DP_OK;
  }
  // the launches capture whether all slots share one mass (and its A_oo^-1)
  const float* unused = nullptr;
  const void* ainv = common_ainv(b->w, 0, b->nslots, b->prec, &unused);
  if (!b->graph || b->graph_k != k || b->graph_ainv != ainv) {
    if (b->graph) {
      DP_HIP(c, hipGraphExecDestroy(b->graph));
      b->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    DP_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    int rc = DP_OK;
    for (int j = 0; j < k && rc == DP_OK; ++j) rc = inner_iteration(b);
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc != DP_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    DP_HIP(c, e);
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    DP_HIP(c, e);
    b->graph_k = k;
    b->graph_ainv = ainv;
  }
  DP_HIP(c, hipGraphLaunch(b->graph, c->stream));
  return DP_OK;
}

// odd reconstruction, restoration, C_PP and the optional S export of finished slots
int finish(dp_batch* b, const std::vector<int>& fin) {
  if (fin.empty()) return DP_OK;
  dp_ctx* c = b->c;
  Workspace& w = b->w;
  const Geom& g = c->g;
  const int n = b->nslots;
  std::vector<int> m(n, 0);
  for (int s : fin) m[s] = 1;
  b->m_outer = m;
  DP_TRY(upload_mask(c, w, w.mask_outer, b->m_outer, 3));
  DP_TRY(hop(c, w, 0, n, F64, 1, 0, EPI_INV_SUB, 0.0, w.x64, w.to64, &w.eta_o, w.mask_outer.as<int>()));
  for (int s : fin) {
    dp_batch::Slot& h = b->slots[s];
    h.hops += 1;
    DP_HIP(c, launch_cpp(g, w.x64.ref(s), w.to64.ref(s), 1, w.alpha.as<double>() + (size_t)s * g.T,
                         space_profile(c), w.x0src.as<int>() + s, w.cpp.as<double>() + (size_t)s * g.T,
                         c->stream));
    if (h.S_dev)
      DP_HIP(c, launch_spinor_export(g, w.x64.ref(s), w.to64.ref(s), 1, w.alpha.as<double>() + (size_t)s * g.T,
                                     space_profile(c), static_cast<double2*>(h.S_dev), 0, c->stream));
  }
  std::vector<double> all((size_t)n * g.T);
  DP_HIP(c, hipMemcpyAsync(all.data(), w.cpp.p, sizeof(double) * g.T * n, hipMemcpyDeviceToHost, c->stream));
  DP_HIP(c, hipStreamSynchronize(c->stream));
  const double t = now_s();
  for (int s : fin) {
    dp_batch::Slot& h = b->slots[s];
    h.cpp.assign(all.begin() + (size_t)s * g.T, all.begin() + (size_t)(s + 1) * g.T);
    h.state = dp_batch::DONE;
    h.in_inner = false;
    h.t_done = t;
    b->done_order.push_back(s);
  }
  return DP_OK;
}

}  // namespace

// ===================================================================== C ABI

extern "C" {

int dp_batch_open(dp_ctx* c, int nslots, int precision, int solver, dp_batch** out) {
  if (!c || !out) return DP_ERR_INVALID_ARG;
  *out = nullptr;
  if (nslots <= 0 || nslots > 4096) return fail(c, DP_ERR_INVALID_ARG, "nslots must be in [1, 4096]");
  if (precision < DP_PREC_F64 || precision > DP_PREC_F32_SINGLE)
    return fail(c, DP_ERR_INVALID_ARG, "unknown precision");
  if (solver != DP_SOLVER_BICGSTAB && solver != DP_SOLVER_CGNR) return fail(c, DP_ERR_INVALID_ARG, "unknown solver");
  DP_HIP(c, hipSetDevice(c->device));
  dp_batch* b = new (std::nothrow) dp_batch;
  if (!b) return fail(c, DP_ERR_OOM, "host allocation failed");
  b->c = c;
  b->nslots = nslots;
  b->api_prec = precision;
  b->single = precision == DP_PREC_F32_SINGLE;
  b->prec = b->single ? F32 : precision;
  b->solver = solver;
  int rc = ensure_ws(c, b->w, nslots, b->prec);
  b->w.sratio = space_hop_ratios(c);  // fixed while the batch is open
  if (rc != DP_OK) {
    delete b;
    return rc;
  }
  b->slots.resize(nslots);
  b->m_inner.assign(nslots, 0);
  b->m_outer.assign(nslots, 0);
  rc = upload_mask(c, b->w, b->w.mask_inner, b->m_inner, 0);
  if (rc == DP_OK) rc = upload_mask(c, b->w, b->w.mask_outer, b->m_outer, 1);
  if (rc == DP_OK) rc = hipStreamSynchronize(c->stream) == hipSuccess ? DP_OK : DP_ERR_DEVICE;
  if (rc != DP_OK) {
    delete b;
    return rc;
  }
  c->open_batches++;
  *out = b;
  return DP_OK;
}

void dp_batch_close(dp_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->c->device);
  (void)hipStreamSynchronize(b->c->stream);
  b->c->mask_count.erase(b->w.mask_inner.p);
  b->c->mask_count.erase(b->w.mask_outer.p);
  b->c->open_batches--;
  delete b;
}

int dp_batch_admit(dp_batch* b, int ncols, const void* eta_dev, void* S_dev, double M, const double* alpha, double r,
                   int max_iter, double delta, int x0_src, long long tag, int* slots_out) {
  if (!b) return DP_ERR_INVALID_ARG;
  dp_ctx* c = b->c;
  if (ncols <= 0 || !eta_dev) return fail(c, DP_ERR_INVALID_ARG, "need ncols > 0 and a source");
  if (!(r > 0) || !std::isfinite(r) || max_iter <= 0 || delta < 0 || delta >= 1 || !std::isfinite(M))
    return fail(c, DP_ERR_INVALID_ARG, "bad residue, max_iter, delta or mass");
  const Geom& g = c->g;
  if (x0_src < 0 || x0_src >= g.T) return fail(c, DP_ERR_INVALID_ARG, "x0_src outside [0, T)");
  if (alpha)
    for (int t = 0; t < g.T; ++t)
      if (!(alpha[t] > 0) || !std::isfinite(alpha[t]) || !std::isfinite(1.0 / alpha[t]))
        return fail(c, DP_ERR_INVALID_ARG, "alpha must be finite and positive");
  DP_HIP(c, hipSetDevice(c->device));
  std::vector<int> fr;
  for (int s = 0; s < b->nslots && (int)fr.size() < ncols; ++s)
    if (b->slots[s].state == dp_batch::FREE) fr.push_back(s);
  if ((int)fr.size() < ncols) return fail(c, DP_ERR_FULL, "not enough free slots in the batch");
  MassEntry* me = nullptr;
  DP_TRY(mass_entry(c, M, &me));
  Workspace& w = b->w;
  const long col = 2L * g.Vh * 12;  // double2 per column
  const double t0 = now_s();
  std::vector<int> pend(b->nslots, 0);
  for (int j = 0; j < ncols; ++j) {
    const int s = fr[j];
    dp_batch::Slot& h = b->slots[s];
    h = dp_batch::Slot();
    h.state = dp_batch::RUNNING;
    h.tag = tag;
    h.S_dev = S_dev ? static_cast<double2*>(S_dev) + (size_t)j * col : nullptr;
    h.me = me;
    h.alpha.assign(alpha ? alpha : c->alpha.data(), (alpha ? alpha : c->alpha.data()) + g.T);
    h.r = r;
    h.delta = delta > 0 ? delta : (b->prec == F16 ? 5e-3 : 1e-5);
    h.max_iter = max_iter;
    h.x0 = x0_src;
    h.t_admit = t0;
    DP_TRY(upload_slot(b, s));
    const double2* src = static_cast<const double2*>(eta_dev) + (size_t)j * col;
    const double* am = w.alpha.as<double>() + (size_t)s * g.T;
    DP_HIP(c, launch_spinor_import(g, src, 1, 0, 0, w.eta_e.ref(s), am, space_profile(c), c->stream));
    DP_HIP(c, launch_spinor_import(g, src, 1, 0, 1, w.eta_o.ref(s), am, space_profile(c), c->stream));
    pend[s] = 1;
    if (slots_out) slots_out[j] = s;
  }
  const int n = b->nslots;
  b->m_outer = pend;
  DP_TRY(upload_mask(c, w, w.mask_outer, b->m_outer, 1));
  const int* m_out = w.mask_outer.as<int>();
  // |eta'|^2 over both parities
  double* sums = w.h_sums.as<double>();
  for (int par = 0; par < 2; ++par) {
    DP_TRY(blas(c, w, 0, n, OP_NORM, F64, m_out, {nullptr, par ? &w.eta_o : &w.eta_e}, FIN_STORE));
    DP_HIP(c, hipMemcpyAsync(sums, w.out_sums.p, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, c->stream));
    DP_HIP(c, hipStreamSynchronize(c->stream));
    for (int s = 0; s < n; ++s)
      if (pend[s]) b->slots[s].eta2 += sums[4 * s];
  }
  for (int s = 0; s < n; ++s)
    if (pend[s] && !std::isfinite(b->slots[s].eta2)) {
      for (int t = 0; t < n; ++t)
        if (pend[t]) b->slots[t].state = dp_batch::FREE;
      return fail(c, DP_ERR_NONFINITE, "source contains NaN or Inf");
    }
  // Schur right-hand side and x = 0
  DP_HIP(c, launch_clover_apply(g, slot_table(w, g.T, 0, F64, m_out), w.eta_o.ref(), w.to64.ref(), n, c->stream));
  DP_TRY(hop(c, w, 0, n, F64, 0, 0, EPI_SUB, 0.0, w.to64, w.b64, &w.eta_e, m_out));
  DP_TRY(blas(c, w, 0, n, OP_ZERO, F64, m_out, {&w.x64}));
  for (int s = 0; s < n; ++s)
    if (pend[s]) b->slots[s].hops = 1;
  std::vector<int> fin;
  DP_TRY(outer_step(b, pend, fin));
  DP_TRY(finish(b, fin));
  return DP_OK;
}

int dp_batch_step(dp_batch* b, int k, int* ndone) {
  if (!b || k <= 0) return DP_ERR_INVALID_ARG;
  TraceRange tr("dp_batch_step");
  dp_ctx* c = b->c;
  DP_HIP(c, hipSetDevice(c->device));
  Workspace& w = b->w;
  const int n = b->nslots;
  bool any = false;
  for (int s = 0; s < n; ++s) any |= b->slots[s].in_inner;
  if (any) {
    {
      TraceRange ti("inner_iterations");
      DP_TRY(inner_iterations(b, k));
    }
    SlotScalars* hsc = w.h_sc.as<SlotScalars>();
    int* hm = w.h_mask.as<int>() + (size_t)3 * w.nslots;
    DP_HIP(c, hipMemcpyAsync(hsc, w.sc.p, sizeof(SlotScalars) * n, hipMemcpyDeviceToHost, c->stream));
    DP_HIP(c, hipMemcpyAsync(hm, w.mask_inner.p, sizeof(int) * n, hipMemcpyDeviceToHost, c->stream));
    DP_HIP(c, hipStreamSynchronize(c->stream));
    DP_TRY(timing_harvest(c));
    std::vector<int> pend(n, 0);
    bool any_pend = false;
    for (int s = 0; s < n; ++s) {
      dp_batch::Slot& h = b->slots[s];
      if (!h.in_inner) continue;
      h.hops += 4 * (hsc[s].iters - h.iters);
      h.iters = hsc[s].iters;
      if (!hm[s]) {
        if (hsc[s].left == 2) h.restarts++;
        h.last_left = hsc[s].left;
        h.in_inner = false;
        b->m_inner[s] = 0;
        pend[s] = 1;
        any_pend = true;
      }
    }
    c->mask_count[w.mask_inner.p] = (int)std::count(b->m_inner.begin(), b->m_inner.end(), 1);
    if (any_pend) {
      TraceRange to("outer_step");
      std::vector<int> fin;
      DP_TRY(outer_step(b, pend, fin));
      DP_TRY(finish(b, fin));
    }
  }
  if (ndone) *ndone = (int)b->done_order.size();
  return DP_OK;
}

int dp_batch_harvest(dp_batch* b, dp_batch_result* out, double* cpp, int max, int* count) {
  if (!b || !count || max < 0 || (max > 0 && !out)) return DP_ERR_INVALID_ARG;
  const int T = b->c->g.T;
  int k = 0;
  while (k < max && !b->done_order.empty()) {
    const int s = b->done_order.front();
    b->done_order.erase(b->done_order.begin());
    dp_batch::Slot& h = b->slots[s];
    dp_batch_result& o = out[k];
    std::memset(&o, 0, sizeof o);
    o.tag = h.tag;
    o.slot = s;
    o.info.status = h.status;
    o.info.iters = h.iters;
    o.info.outer = h.outer;
    o.info.hop_calls = h.hops;
    o.info.restarts = h.restarts;
    o.info.true_res = h.eta2 > 0 ? std::sqrt(h.res2 / h.eta2) : 0.0;
    o.info.seconds = h.t_done - h.t_admit;
    if (cpp) std::memcpy(cpp + (size_t)k * T, h.cpp.data(), sizeof(double) * T);
    h.state = dp_batch::FREE;
    ++k;
  }
  *count = k;
  return DP_OK;
}

int dp_batch_status(const dp_batch* b, int* free_slots, int* running, int* done) {
  if (!b) return DP_ERR_INVALID_ARG;
  int f = 0, r = 0, d = 0;
  for (const auto& s : b->slots) {
    f += s.state == dp_batch::FREE;
    r += s.state == dp_batch::RUNNING;
    d += s.state == dp_batch::DONE;
  }
  if (free_slots) *free_slots = f;
  if (running) *running = r;
  if (done) *done = d;
  return DP_OK;
}

long long dp_batch_device_bytes(const dp_batch* b) { return b ? (long long)b->w.device_bytes() : -1; }

// ------------------------------------------------------------ dp_solve

static int validate_params(dp_ctx* c, int nrhs, const dp_params* p) {
  if (!p) return fail(c, DP_ERR_INVALID_ARG, "params is NULL");
  if (nrhs <= 0) return fail(c, DP_ERR_INVALID_ARG, "nrhs must be positive");
  if (!(p->r > 0) || !std::isfinite(p->r)) return fail(c, DP_ERR_INVALID_ARG, "r must be positive");
  if (p->solver != DP_SOLVER_BICGSTAB && p->solver != DP_SOLVER_CGNR)
    return fail(c, DP_ERR_INVALID_ARG, "unknown solver");
  if (p->precision < DP_PREC_F64 || p->precision > DP_PREC_F32_SINGLE)
    return fail(c, DP_ERR_INVALID_ARG, "unknown precision");
  if (p->max_iter <= 0) return fail(c, DP_ERR_INVALID_ARG, "max_iter must be positive");
  if (p->delta < 0 || p->delta >= 1) return fail(c, DP_ERR_INVALID_ARG, "delta must be in [0, 1)");
  if (p->x0_src < 0 || p->x0_src >= c->g.T) return fail(c, DP_ERR_INVALID_ARG, "x0_src outside [0, T)");
  if (p->ncols_group < 0 || (p->ncols_group > 0 && nrhs % p->ncols_group != 0))
    return fail(c, DP_ERR_INVALID_ARG, "nrhs must be a multiple of ncols_group");
  return DP_OK;
}

static int solve_batch(dp_ctx* c, const double2* eta, int n, const dp_params& P, double2* S, double* cpp_out,
                       dp_info* info);

// One batch filled with the columns of the request; after a failure other than
// a column stopping at max_iter or going non-finite (both finish their slots)
// the kept batch may hold slots that never finish, so it is dropped.
static int solve_common(dp_ctx* c, const double2* eta, int n, const dp_params& P, double2* S, double* cpp_out,
                        dp_info* info) {
  const int T = c->g.T;
  const int grp = P.ncols_group > 0 ? P.ncols_group : 1;
  std::vector<dp_info> inf(n);
  std::vector<double> per((size_t)n * T);
  dp_params Pc = P;
  Pc.ncols_group = 0;  // per column here; grouped below
  int rc = solve_batch(c, eta, n, Pc, S, per.data(), inf.data());
  if (rc != DP_OK && rc != DP_ERR_NOT_CONVERGED && rc != DP_ERR_NONFINITE && rc != DP_ERR_BREAKDOWN) {
    if (c->solve_batch) {
      const std::string err = c->err;
      dp_batch_close(c->solve_batch);
      c->solve_batch = nullptr;
      c->err = err;
    }
    return rc;
  }
  // A column whose FP32 / FP16 inner solve went non-finite is solved again in
  // FP64, which the inner precision's range does not limit.
  if (rc == DP_ERR_NONFINITE && P.precision != DP_PREC_F64) {
    dp_params P64 = Pc;
    P64.precision = DP_PREC_F64;
    const size_t col = (size_t)2 * c->g.Vh * 12;  // double2 per column
    for (int j = 0; j < n; ++j) {
      if (inf[j].status != DP_ERR_NONFINITE) continue;
      dp_info one{};
      const int r1 = solve_batch(c, eta + j * col, 1, P64, S ? S + j * col : nullptr, per.data() + (size_t)j * T, &one);
      if (r1 != DP_OK && r1 != DP_ERR_NOT_CONVERGED && r1 != DP_ERR_NONFINITE && r1 != DP_ERR_BREAKDOWN) return r1;
      one.restarts += inf[j].restarts;
      one.iters += inf[j].iters;
      one.outer += inf[j].outer;
      one.hop_calls += inf[j].hop_calls;
      one.fallback = 1;
      inf[j] = one;
    }
    rc = DP_OK;
    for (int j = 0; j < n; ++j)
      if (inf[j].status != DP_OK && rc == DP_OK) rc = inf[j].status;
  }
  if (info) std::copy(inf.begin(), inf.end(), info);
  if (cpp_out)
    for (int k = 0; k < n / grp; ++k)
      for (int t = 0; t < T; ++t) {
        double acc = 0.0;
        for (int j = 0; j < grp; ++j) acc += per[(size_t)(k * grp + j) * T + t];
        cpp_out[(size_t)k * T + t] = acc;
      }
  if (rc == DP_ERR_NOT_CONVERGED) c->err = "a right-hand side reached max_iter before the residue r";
  if (rc == DP_ERR_NONFINITE) c->err = "a residual became NaN or Inf";
  if (rc == DP_ERR_BREAKDOWN) c->err = "BiCGStab broke down three times in a row without progress";
  return rc;
}

static int solve_batch(dp_ctx* c, const double2* eta, int n, const dp_params& P, double2* S, double* cpp_out,
                       dp_info* info) {
  dp_batch*& b = c->solve_batch;
  if (b && (b->nslots < n || b->api_prec != P.precision || b->solver != P.solver)) {
    dp_batch_close(b);
    b = nullptr;
  }
  if (!b) DP_TRY(dp_batch_open(c, n, P.precision, P.solver, &b));
  const double t0 = now_s();
  std::vector<int> slot(n);
  int rc = dp_batch_admit(b, n, eta, S, c->M, c->alpha.data(), P.r, P.max_iter, P.delta, P.x0_src, 0, slot.data());
  if (rc != DP_OK) return rc;
  int done = 0;
  while (done < n) {
    int running = 0;
    DP_TRY(dp_batch_step(b, 4, &done));
    DP_TRY(dp_batch_status(b, nullptr, &running, nullptr));
    bool inner = false;
    for (const auto& sl : b->slots) inner |= sl.in_inner;
    if (done < n && !inner) return fail(c, DP_ERR_BAD_STATE, "slots neither running nor finished");
  }
  std::vector<dp_batch_result> res(n);
  std::vector<double> cpp((size_t)n * c->g.T);
  int cnt = 0;
  DP_TRY(dp_batch_harvest(b, res.data(), cpp.data(), n, &cnt));
  const double secs = now_s() - t0;
  // results come in completion order; map them back to the columns
  std::vector<int> col_of_slot(b->nslots, -1);
  for (int j = 0; j < n; ++j) col_of_slot[slot[j]] = j;
  std::vector<double> per((size_t)n * c->g.T);
  int status = DP_OK;
  for (int k = 0; k < cnt; ++k) {
    const int j = col_of_slot[res[k].slot];
    std::memcpy(per.data() + (size_t)j * c->g.T, cpp.data() + (size_t)k * c->g.T, sizeof(double) * c->g.T);
    if (info) {
      info[j] = res[k].info;
      info[j].seconds = secs;
    }
    if (res[k].info.status != DP_OK && status == DP_OK) status = res[k].info.status;
  }
  if (cpp_out) std::copy(per.begin(), per.end(), cpp_out);  // per column (ncols_group is applied by the caller)
  return status;
}

int dp_solve(dp_ctx* c, const double* eta, int nrhs, const dp_params* p, double* S, double* cpp, dp_info* info) {
  TraceRange tr("dp_solve");
  if (!c || !eta) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  DP_HIP(c, hipSetDevice(c->device));
  DP_TRY(validate_params(c, nrhs, p));
  const size_t bytes = (size_t)nrhs * 2 * c->g.Vh * 12 * sizeof(double2);
  // sources and solutions in separate halves (an FP64 retry reads a source again)
  DP_HIP(c, c->scratch_aos.reserve(S ? 2 * bytes : bytes));
  double2* deta = c->scratch_aos.as<double2>();
  double2* dS = S ? deta + bytes / sizeof(double2) : nullptr;
  DP_HIP(c, hipMemcpyAsync(deta, eta, bytes, hipMemcpyHostToDevice, c->stream));
  int rc = solve_common(c, deta, nrhs, *p, dS, cpp, info);
  if (S && (rc == DP_OK || rc == DP_ERR_NOT_CONVERGED || rc == DP_ERR_BREAKDOWN || rc == DP_ERR_NONFINITE)) {
    DP_HIP(c, hipMemcpyAsync(S, dS, bytes, hipMemcpyDeviceToHost, c->stream));
    DP_HIP(c, hipStreamSynchronize(c->stream));
  }
  return rc;
}

int dp_solve_dev(dp_ctx* c, const void* eta, int nrhs, const dp_params* p, void* S, double* cpp, dp_info* info,
                 void* stream) {
  TraceRange tr("dp_solve_dev");
  if (!c || !eta) return fail(c, DP_ERR_INVALID_ARG, "null argument");
  DP_HIP(c, hipSetDevice(c->device));
  DP_TRY(validate_params(c, nrhs, p));
  const size_t bytes = (size_t)nrhs * 2 * c->g.Vh * 12 * sizeof(double2);
  const char* e0 = static_cast<const char*>(eta);
  const char* s0 = static_cast<const char*>(S);
  if (S && e0 < s0 + bytes && s0 < e0 + bytes) return fail(c, DP_ERR_INVALID_ARG, "eta and S overlap");
  if (stream) DP_HIP(c, hipStreamSynchronize((hipStream_t)stream));
  return solve_common(c, static_cast<const double2*>(eta), nrhs, *p, static_cast<double2*>(S), cpp, info);
}

}  // extern "C"
