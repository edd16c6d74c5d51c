// Host runtime behind the C ABI of include/ch.h: validation, workspace
// planning, table generation, kernel dispatch.  The library allocates no
// device memory: all tables and scratch live in the caller's workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/ch.h"
#include "ch_internal.h"

using chk::InstDev;
using chk::WorkItem;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Sub-allocation plan of the workspace (byte offsets).
struct Block {
  size_t off = 0, bytes = 0;
};

struct ClassPlan {      // all instances sharing (dim, n, fine kind, precision)
  int dim = 2, n = 0, fine_kind = 0, precision = 0;
  int waves = 0;        // fine-kernel variant (0 = default), set by the autotuner
  std::vector<WorkItem> items;   // every slice of every instance in the class
  std::vector<int32_t> insts;    // instance indices
  Block items_blk, insts_blk;
  Block sine_blk;                // 2D: Se | So | lam ; 1D: S | lam
  int chain_groups = 1;          // workgroups per instance in the coarse chain
  int fine_groups = 1;           // workgroups per work item in the fine sweep
  Block sync_blk;                // barrier words of the multi-workgroup kernels
};

}  // namespace

struct ch_ctx {
  std::vector<ch_problem> probs;
  std::vector<InstDev> inst;        // host copy (device pointers filled at bind)
  std::vector<int64_t> slice_off, iter_off;
  int64_t slice_total = 0, iter_total = 0;
  std::vector<ClassPlan> classes;
  Block inst_blk, active_blk, status_blk, k_blk;
  Block iters_blk;                  // solver iteration counts, two per slice
  std::vector<Block> rsig_fine_blk, rsig_stab_blk, tab_blk, work_blk;
  // learned coarse propagator
  Block nn_blk, nn_out_blk, nn_part_blk;
  // its judge (instances created with the learned propagator): the instance
  // list (host-initialised), JudgeDev records, live and refresh flags (one
  // per instance), ratios (one per iteration), the plain propagator's
  // results and the two per-slice distances
  std::vector<int32_t> judge_insts;
  std::vector<int32_t> judge_enabled;
  int judge_rstride = 0;
  Block jinsts_blk, jdev_blk, jlive_blk, jrefresh_blk, jratio_blk, jgp_blk, jdist_blk, jgate_blk;
  Block nn_gbase_blk;               // G_plain(u) under a learned propagator with a plain base
  bool capturing = false;           // a graph of one iteration is being recorded
  // pipelined iterations (one 2D n = 128 instance): fine inputs (2 N n^2),
  // odd-iteration fine results (N n^2), hand-off counters
  bool pipe = false;
  Block pipe_blk, pipe_sync_blk;
  size_t nn_floats = 0;
  const uint16_t* nn_w = nullptr;
  bool nn_planned = false;
  size_t ws_bytes = 0;
  size_t host_init_bytes = 0;       // leading part of the workspace uploaded at bind
  char* ws = nullptr;               // bound workspace
  std::string err;
  // side streams that run the sequential coarse sweeps of the grid-size
  // classes concurrently (each sweep alone fills few CUs), created on first
  // use; forked from and joined to the caller's stream with events
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> side_done;
  hipEvent_t fork_ev = nullptr;
  ~ch_ctx() {
    for (hipEvent_t e : side_done) (void)hipEventDestroy(e);
    for (hipStream_t q : side) (void)hipStreamDestroy(q);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
  }
};

namespace {

ch_status fail(ch_ctx* c, ch_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

ch_status hip_check(ch_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return CH_OK;
  return fail(c, CH_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// sin(j k pi / (n+1)) with the integer product reduced modulo 2(n+1) first,
// so the argument stays in [0, 2 pi) and carries no large-argument error.
double sine_entry(long j, long k, long n) {
  const long period = 2 * (n + 1);
  const long m = (j * k) % period;
  const long double ang = (long double)m * 3.14159265358979323846264338327950288L / (long double)(n + 1);
  return (double)(std::sqrt(2.0L / (long double)(n + 1)) * sinl(ang));
}
// Eigenvalues of the Dirichlet difference Laplacian (1-based p):
// lam_p = (2/h^2)(cos(p pi/(n+1)) - 1) = -(4/h^2) sin^2(p pi / (2(n+1))).
double lap_eig(long p, long n) {
  const long double h = 1.0L / (long double)(n + 1);
  const long double sn = sinl((long double)p * 3.14159265358979323846264338327950288L /
                              (2.0L * (long double)(n + 1)));
  return (double)(-4.0L / (h * h) * sn * sn);
}

bool supported_2d(int n) { return n == 32 || n == 64 || n == 128 || n == 256; }

}  // namespace

extern "C" {

// side streams of the per-class coarse sweeps (defined with coarse_all)
static ch_status make_sides(ch_ctx* c, size_t count);

const char* ch_status_str(ch_status s) {
  switch (s) {
    case CH_OK: return "CH_OK";
    case CH_ERR_ARG: return "CH_ERR_ARG";
    case CH_ERR_HIP: return "CH_ERR_HIP";
    case CH_ERR_UNSUPPORTED: return "CH_ERR_UNSUPPORTED";
    case CH_ERR_NOCONV: return "CH_ERR_NOCONV";
    case CH_ERR_STATE: return "CH_ERR_STATE";
    case CH_ERR_TIMEOUT: return "CH_ERR_TIMEOUT";
  }
  return "CH_ERR_UNKNOWN";
}

const char* ch_last_error(const ch_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// Subdomains of the direct 1D (2.4) solve: the divisor N0 <= 64 of n + 1
// (at least two intervals each) with the shortest elimination chains, about
// 2 (n+1)/N0 (a subdomain's factorisation and solve) + 2 N0 (the interface
// elimination, forward and back); 1 when n + 1 has none.
static int direct_sub(int n) {
  int best = 1;
  double cost = 2.0 * (n + 1) + 2.0;
  for (int k = 2; k <= 64 && 2 * k <= n + 1; ++k) {
    if ((n + 1) % k) continue;
    const double c = 2.0 * (n + 1) / k + 2.0 * k;
    if (c < cost) { cost = c; best = k; }
  }
  return best;
}

// Neumann-Neumann parameters with their defaults (0 selects the default)
static int dd_sub(const ch_problem& p) { return p.dd_subdomains > 0 ? p.dd_subdomains : 8; }

ch_status ch_create(const ch_problem* probs, int32_t n_inst, ch_ctx** out) {
  if (!out) return CH_ERR_ARG;
  *out = nullptr;
  if (!probs || n_inst <= 0) return CH_ERR_ARG;
  ch_ctx* c = new ch_ctx();
  c->probs.assign(probs, probs + n_inst);
  for (int i = 0; i < n_inst; ++i) {
    const ch_problem& p = probs[i];
    ch_status bad = CH_OK;
    if (p.dim != 1 && p.dim != 2) bad = fail(c, CH_ERR_UNSUPPORTED, "instance %d: dim %d", i, p.dim);
    else if (p.n < 2) bad = fail(c, CH_ERR_ARG, "instance %d: n = %d", i, p.n);
    else if (!(p.eps > 0) || !(p.T > 0) || !(p.s_fine >= 0))
      bad = fail(c, CH_ERR_ARG, "instance %d: eps, T must be > 0 and s >= 0", i);
    else if (p.n_slices < 1 || p.j_fine < 1 || p.m_coarse < 1)
      bad = fail(c, CH_ERR_ARG, "instance %d: n_slices, j_fine, m_coarse must be >= 1", i);
    else if (p.krylov_max < 1 || !(p.krylov_rtol >= 0))
      bad = fail(c, CH_ERR_ARG, "instance %d: krylov_max >= 1 and krylov_rtol >= 0 needed", i);
    else if (p.fine_kind < CH_FINE_LINEAR || p.fine_kind > CH_FINE_APPROX2_DD)
      bad = fail(c, CH_ERR_ARG, "instance %d: fine_kind %d", i, p.fine_kind);
    else if (p.fine_kind == CH_FINE_APPROX2_DD && (p.dim != 1 || p.f_zero))
      bad = fail(c, CH_ERR_UNSUPPORTED,
                 "instance %d: the Neumann-Neumann fine step is 1D and has no f == 0 form", i);
    else if (p.fine_kind == CH_FINE_APPROX2_DD &&
             (p.dd_subdomains < 0 || p.dd_max < 0 || !(p.dd_tol >= 0) ||
              !(p.dd_theta >= 0 && p.dd_theta < 1) ||
              (p.n + 1) % dd_sub(p) != 0 || (p.n + 1) / dd_sub(p) < 2))
      bad = fail(c, CH_ERR_ARG,
                 "instance %d: Neumann-Neumann parameters (n + 1 = %d must split into N0 = %d "
                 "pieces of >= 2 intervals; 0 <= theta < 1, tol >= 0, max >= 0)",
                 i, p.n + 1, dd_sub(p));
    else if (p.coarse_kind < CH_COARSE_APPROX2 || p.coarse_kind > CH_COARSE_EYRE)
      bad = fail(c, CH_ERR_ARG, "instance %d: coarse_kind %d", i, p.coarse_kind);
    else if (p.precision != CH_PREC_FP64 && p.precision != CH_PREC_SPLIT_BF16)
      bad = fail(c, CH_ERR_ARG, "instance %d: precision %d", i, p.precision);
    else if ((p.fine_kind == CH_FINE_NONLINEAR || p.coarse_kind == CH_COARSE_EYRE) &&
             (p.nl_variant < CH_NL_EYRE || p.nl_variant > CH_NL_FULL_BE || p.newton_max < 1 ||
              !(p.newton_tol > 0) || !(p.nl_krylov_rtol > 0)))
      bad = fail(c, CH_ERR_ARG, "instance %d: Newton parameters", i);
    else if (p.nn_base != 0 && p.nn_base != 1)
      bad = fail(c, CH_ERR_ARG, "instance %d: nn_base %d", i, p.nn_base);
    else if (p.coarse_kind == CH_COARSE_NEURAL && (p.dim != 2 || p.n % 8 != 0))
      bad = fail(c, CH_ERR_UNSUPPORTED,
                 "instance %d: the learned coarse propagator needs 2D with n divisible by 8", i);
    else if (p.precision == CH_PREC_SPLIT_BF16 &&
             (p.dim != 2 || p.fine_kind != CH_FINE_LINEAR || (p.n != 64 && p.n != 128)))
      bad = fail(c, CH_ERR_UNSUPPORTED,
                 "instance %d: split-bf16 covers the 2D linear step with n = 64, 128", i);
    else if (p.dim == 2 && !supported_2d(p.n))
      bad = fail(c, CH_ERR_UNSUPPORTED, "instance %d: 2D n = %d (kernels cover 32, 64, 128, 256)", i, p.n);
    else if (p.dim == 1 && p.n > 128)
      bad = fail(c, CH_ERR_UNSUPPORTED, "instance %d: 1D n = %d (n <= 128)", i, p.n);
    if (bad != CH_OK) {
      ch_status s = bad;
      // keep the message for the caller: the context is not returned, so
      // print it to stderr as well.
      fprintf(stderr, "ch_create: %s\n", c->err.c_str());
      delete c;
      return s;
    }
  }
  // layouts
  c->slice_off.resize(n_inst);
  c->iter_off.resize(n_inst);
  int64_t so = 0, io = 0, slice_base = 0;
  c->inst.resize(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    const ch_problem& p = probs[i];
    const int64_t P = p.dim == 2 ? (int64_t)p.n * p.n : p.n;
    c->slice_off[i] = so;
    c->iter_off[i] = io;
    InstDev& d = c->inst[i];
    memset(&d, 0, sizeof d);
    d.dim = p.dim; d.n = p.n; d.n_slices = p.n_slices; d.j_fine = p.j_fine;
    d.m_coarse = p.m_coarse; d.coarse_kind = p.coarse_kind; d.fine_kind = p.fine_kind;
    d.nl_variant = p.nl_variant; d.f_zero = p.f_zero; d.krylov_max = p.krylov_max;
    d.newton_max = p.newton_max; d.precision = p.precision;
    d.eps = p.eps; d.dT = p.T / p.n_slices; d.dt = d.dT / p.j_fine; d.s_fine = p.s_fine;
    // CG target of the (2.4) solves: 0 picks the default, 1e-12 with the
    // linear fine step and 1e-13 otherwise (measured: at 1e-12 the implicit
    // and PA-I runs at n = 128 miss the 1e-11 bar, the linear ones keep it)
    const double rtol = p.krylov_rtol > 0 ? p.krylov_rtol
                                          : (p.fine_kind == CH_FINE_LINEAR ? 1e-12 : 1e-13);
    d.h = 1.0 / (p.n + 1); d.newton_tol = p.newton_tol; d.krylov_rtol = rtol;
    d.nl_krylov_rtol = p.nl_krylov_rtol;
    // streamed Newton solves (n = 256) carry two more vectors
    d.work_vecs = (p.dim == 2 && p.n == 256 &&
                   (p.fine_kind == CH_FINE_NONLINEAR || p.coarse_kind == CH_COARSE_EYRE))
                      ? 9 : chk::WORK_VECS;
    d.nn_base = p.nn_base;
    d.dd_sub = dd_sub(p);
    d.direct_sub = direct_sub(p.n);
    d.dd_max = p.dd_max > 0 ? p.dd_max : 100;
    d.dd_theta = p.dd_theta > 0 ? p.dd_theta : 0.25;
    d.dd_tol = p.dd_tol > 0 ? p.dd_tol : 1e-10;
    d.wait_ticks = chk::WAIT_TICKS_DEFAULT;
    d.pipe_wait_ticks = chk::PIPE_WAIT_TICKS_DEFAULT;
    d.off_slices = so; d.off_iter = io; d.slice_base = slice_base;
    so += (int64_t)p.n_slices * P;
    io += (int64_t)(p.n_slices + 1) * P;
    slice_base += p.n_slices;
  }
  c->slice_total = so;
  c->iter_total = io;
  // classes
  std::map<std::tuple<int, int, int, int>, int> cls;
  for (int i = 0; i < n_inst; ++i) {
    auto key = std::make_tuple(probs[i].dim, probs[i].n, probs[i].fine_kind, probs[i].precision);
    if (!cls.count(key)) {
      cls[key] = (int)c->classes.size();
      ClassPlan cp;
      cp.dim = probs[i].dim;
      cp.n = probs[i].n;
      cp.fine_kind = probs[i].fine_kind;
      cp.precision = probs[i].precision;
      c->classes.push_back(cp);
    }
    ClassPlan& cp = c->classes[cls[key]];
    cp.insts.push_back(i);
    for (int s = 0; s < probs[i].n_slices; ++s) cp.items.push_back(WorkItem{i, s});
  }
  // workspace plan
  size_t off = 0;
  auto take = [&](size_t bytes) { Block b; b.off = off; b.bytes = bytes; off = align_up(off + bytes); return b; };
  c->inst_blk = take(sizeof(InstDev) * n_inst);
  c->active_blk = take(sizeof(int32_t) * n_inst);
  c->status_blk = take(sizeof(int32_t) * n_inst);
  c->k_blk = take(sizeof(int32_t));
  for (int i = 0; i < n_inst; ++i)
    if (probs[i].coarse_kind == CH_COARSE_NEURAL) {
      c->judge_insts.push_back(i);
      c->judge_enabled.push_back(1);
      c->judge_rstride = std::max(c->judge_rstride, probs[i].n_slices);
    }
  if (!c->judge_insts.empty()) {
    c->jinsts_blk = take(sizeof(int32_t) * c->judge_insts.size());
    c->jdev_blk = take(sizeof(chk::JudgeDev) * c->judge_insts.size());
  }
  for (auto& cp : c->classes) {
    cp.items_blk = take(sizeof(WorkItem) * cp.items.size());
    cp.insts_blk = take(sizeof(int32_t) * cp.insts.size());
    const size_t n = cp.n;
    cp.sine_blk = cp.dim == 2 ? take(sizeof(double) * (2 * (n + 1) + n))
                              : take(sizeof(double) * (n * n + n));
  }
  // blocks initialised from the host image first, device-only blocks after
  c->rsig_fine_blk.resize(n_inst);
  c->rsig_stab_blk.resize(n_inst);
  c->tab_blk.resize(n_inst);
  c->work_blk.resize(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    const size_t P = probs[i].dim == 2 ? (size_t)probs[i].n * probs[i].n : probs[i].n;
    c->rsig_fine_blk[i] = take(sizeof(double) * P);
    c->rsig_stab_blk[i] = take(sizeof(double) * P);
  }
  // solver iteration counts of the fine sweeps, two per slice (zeroed with
  // the host image)
  c->iters_blk = take(sizeof(int32_t) * 2 * (size_t)slice_base);
  c->host_init_bytes = off;
  for (auto& cp : c->classes) {
    if (cp.dim != 2) continue;
    // coarse sweep: groups of eight while 8 x instances fit on a 256-CU
    // device, else groups of four (the launch falls back to one workgroup per
    // instance on a smaller device)
    const int cap = chk::chain_coop_capacity(cp.n);
    if (cap > 0 && (int)cp.insts.size() <= cap / 2) cp.chain_groups = 8;
    else if (cap > 0 && (int)cp.insts.size() <= cap) cp.chain_groups = 4;
    const int fcap = chk::fine_group_capacity(cp.n);
    if (fcap > 0 && (int)cp.items.size() <= fcap && cp.fine_kind == CH_FINE_LINEAR &&
        cp.precision == CH_PREC_FP64)
      cp.fine_groups = chk::fine_group_default(cp.n);
    // implicit step: groups of 16 at n = 256 always; groups of 8 at n = 128
    // while the groups of the class fit on the device at once
    if (cp.fine_kind == CH_FINE_NONLINEAR && cp.n == 256) cp.fine_groups = 16;
    if (cp.fine_kind == CH_FINE_NONLINEAR && cp.n == 128 && cp.items.size() <= 32)
      cp.fine_groups = 8;
    const size_t units = std::max(cp.insts.size(), cp.items.size());
    cp.sync_blk = take(sizeof(int32_t) * 64 * 8 * ((units + 7) / 8));
  }
  for (int i = 0; i < n_inst; ++i) {
    const size_t P = probs[i].dim == 2 ? (size_t)probs[i].n * probs[i].n : probs[i].n;
    if (probs[i].dim == 2) {
      c->tab_blk[i] = take(sizeof(double) * P * chk::TAB_VECS);
      c->work_blk[i] = take(sizeof(double) * P * (size_t)c->inst[i].work_vecs * (size_t)probs[i].n_slices);
    }
  }
  // pipelined iterations: one instance of a class the pipelined kernel covers
  if (n_inst == 1 && probs[0].dim == 2 && chk::pipe_supported(probs[0].n) &&
      probs[0].fine_kind == CH_FINE_LINEAR && probs[0].precision == CH_PREC_FP64 &&
      probs[0].coarse_kind == CH_COARSE_APPROX2 && probs[0].n_slices >= 2) {
    const size_t SN = (size_t)probs[0].n_slices * probs[0].n * probs[0].n;
    c->pipe = true;
    c->pipe_blk = take(sizeof(double) * 3 * SN);
    c->pipe_sync_blk = take(sizeof(int32_t) * chk::pipe_sync_words(probs[0].n_slices));
  }
  // learned coarse propagator workspace: activations for a batch of all
  // slices of the largest neural instance, FP64 outputs, norm partials
  {
    size_t fl = 0, outd = 0, partd = 0;
    for (int i = 0; i < n_inst; ++i) {
      if (probs[i].coarse_kind != CH_COARSE_NEURAL) continue;
      c->nn_planned = true;
      const size_t P = (size_t)probs[i].n * probs[i].n;
      fl = std::max(fl, chk::nn_plan(probs[i].n_slices, probs[i].n).floats);
      outd = std::max(outd, (size_t)probs[i].n_slices * P);
      partd = std::max(partd, (size_t)probs[i].n_slices * ((P + 255) / 256));
    }
    if (c->nn_planned) {
      c->nn_floats = fl;
      c->nn_blk = take(fl * sizeof(float));
      c->nn_out_blk = take(outd * sizeof(double));
      c->nn_part_blk = take(partd * sizeof(double));
      int64_t n_slices_all = 0;
      for (int i = 0; i < n_inst; ++i) n_slices_all += probs[i].n_slices;
      c->jlive_blk = take(sizeof(int32_t) * n_inst);
      c->jrefresh_blk = take(sizeof(int32_t) * n_inst);
      c->jratio_blk = take(sizeof(double) * c->judge_insts.size() * (size_t)c->judge_rstride);
      c->jgp_blk = take(sizeof(double) * (size_t)c->slice_total);
      c->jdist_blk = take(sizeof(double) * 2 * (size_t)n_slices_all);
      c->jgate_blk = take(sizeof(int32_t) * (size_t)n_slices_all);
      bool base = false;
      for (int i = 0; i < n_inst; ++i)
        base = base || (probs[i].coarse_kind == CH_COARSE_NEURAL && probs[i].nn_base);
      if (base) c->nn_gbase_blk = take(sizeof(double) * (size_t)c->slice_total);
    }
  }
  c->ws_bytes = off;
  *out = c;
  return CH_OK;
}

ch_status ch_destroy(ch_ctx* ctx) {
  delete ctx;
  return CH_OK;
}

ch_status ch_workspace_size(const ch_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return CH_ERR_ARG;
  *bytes = ctx->ws_bytes;
  return CH_OK;
}

ch_status ch_layout(const ch_ctx* ctx, int32_t inst, int64_t* slice_total, int64_t* iter_total,
                    int64_t* slice_off, int64_t* iter_off) {
  if (!ctx) return CH_ERR_ARG;
  if (inst < 0 || inst >= (int32_t)ctx->probs.size()) return CH_ERR_ARG;
  if (slice_total) *slice_total = ctx->slice_total;
  if (iter_total) *iter_total = ctx->iter_total;
  if (slice_off) *slice_off = ctx->slice_off[inst];
  if (iter_off) *iter_off = ctx->iter_off[inst];
  return CH_OK;
}

ch_status ch_bind_workspace(ch_ctx* c, void* dptr, size_t bytes, ch_stream stream) {
  if (!c) return CH_ERR_ARG;
  if (!dptr || (reinterpret_cast<uintptr_t>(dptr) % kAlign) != 0)
    return fail(c, CH_ERR_ARG, "workspace must be a non-null 256-byte aligned device pointer");
  if (bytes < c->ws_bytes)
    return fail(c, CH_ERR_ARG, "workspace too small: %zu < %zu bytes", bytes, c->ws_bytes);
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)dptr;
  c->ws = ws;
  const int n_inst = (int)c->probs.size();
  // host images of everything, copied in one pass
  std::vector<char> img(c->host_init_bytes, 0);
  for (int i = 0; i < n_inst; ++i) {
    InstDev& d = c->inst[i];
    const ch_problem& p = c->probs[i];
    d.rsig_fine = (const double*)(ws + c->rsig_fine_blk[i].off);
    d.rsig_stab = (const double*)(ws + c->rsig_stab_blk[i].off);
    d.tab = p.dim == 2 ? (double*)(ws + c->tab_blk[i].off) : nullptr;
    d.work = p.dim == 2 ? (double*)(ws + c->work_blk[i].off) : nullptr;
    d.status = (int32_t*)(ws + c->status_blk.off) + i;
    d.iters = (int32_t*)(ws + c->iters_blk.off) + 2 * d.slice_base;
    // inverse symbols 1/(1 + tau eps^2 Lam^2 - s tau Lam) of the linear step
    const int n = p.n;
    std::vector<double> lam(n);
    for (int k = 0; k < n; ++k) lam[k] = lap_eig(k + 1, n);
    auto fill = [&](Block b, double tau) {
      double* t = (double*)(img.data() + b.off);
      if (p.dim == 2) {
        for (int r = 0; r < n; ++r)
          for (int q = 0; q < n; ++q) {
            const double L = lam[r] + lam[q];
            t[r * n + q] = 1.0 / (1.0 + tau * p.eps * p.eps * L * L - p.s_fine * tau * L);
          }
      } else {
        for (int r = 0; r < n; ++r) {
          const double L = lam[r];
          t[r] = 1.0 / (1.0 + tau * p.eps * p.eps * L * L - p.s_fine * tau * L);
        }
      }
    };
    fill(c->rsig_fine_blk[i], d.dt);
    fill(c->rsig_stab_blk[i], d.dT / p.m_coarse);
  }
  memcpy(img.data() + c->inst_blk.off, c->inst.data(), sizeof(InstDev) * n_inst);
  if (!c->judge_insts.empty()) {
    memcpy(img.data() + c->jinsts_blk.off, c->judge_insts.data(),
           sizeof(int32_t) * c->judge_insts.size());
    chk::JudgeDev* jd = (chk::JudgeDev*)(img.data() + c->jdev_blk.off);
    for (size_t t = 0; t < c->judge_insts.size(); ++t) {
      jd[t].delta_prev = 0.0;
      jd[t].fallback_at = -1;
      jd[t].enabled = 1;
    }
  }
  for (auto& cp : c->classes) {
    memcpy(img.data() + cp.items_blk.off, cp.items.data(), sizeof(WorkItem) * cp.items.size());
    memcpy(img.data() + cp.insts_blk.off, cp.insts.data(), sizeof(int32_t) * cp.insts.size());
    const int n = cp.n;
    double* t = (double*)(img.data() + cp.sine_blk.off);
    if (cp.dim == 2) {
      // T[m] = sqrt(2/(n+1)) sin(m pi/(n+1)), m < 2(n+1), then lam
      for (int m = 0; m < 2 * (n + 1); ++m) t[m] = sine_entry(m, 1, n);
      for (int k = 0; k < n; ++k) t[2 * (n + 1) + k] = lap_eig(k + 1, n);
    } else {
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) t[a * n + b] = sine_entry(a + 1, b + 1, n);
      for (int k = 0; k < n; ++k) t[n * n + k] = lap_eig(k + 1, n);
    }
  }
  ch_status st = hip_check(c, hipMemcpyAsync(ws, img.data(), c->host_init_bytes,
                                             hipMemcpyHostToDevice, s),
                           "workspace upload");
  if (st != CH_OK) return st;
  for (auto& cp : c->classes) {
    if (cp.dim != 2) continue;
    const double* lam = (const double*)(ws + cp.sine_blk.off) + 2 * (cp.n + 1);
    st = hip_check(c, chk::launch_cg_tables(cp.n, 2, (const int32_t*)(ws + cp.insts_blk.off),
                                            (int)cp.insts.size(),
                                            (const InstDev*)(ws + c->inst_blk.off), lam, s),
                   "cg tables");
    if (st != CH_OK) return st;
  }
  // side streams of the per-class coarse sweeps, made here so that no stream
  // is created while a caller captures
  if (c->classes.size() > 1) {
    st = make_sides(c, c->classes.size() - 1);
    if (st != CH_OK) return st;
  }
  // the host image must outlive the copy
  return hip_check(c, hipStreamSynchronize(s), "bind synchronize");
}

static ch_status require_bound(ch_ctx* c) {
  if (!c) return CH_ERR_ARG;
  if (!c->ws) return fail(c, CH_ERR_STATE, "workspace not bound");
  return CH_OK;
}

// The workspace status words collect the flags the kernels of one call
// raise (bit 1 solver cap, 2 non-finite, 4 group wait timed out); every call
// that launches fine or coarse kernels of its own clears them first.
static int32_t* ws_status(ch_ctx* c) { return (int32_t*)(c->ws + c->status_blk.off); }
static ch_status clear_ws_status(ch_ctx* c, hipStream_t s) {
  return hip_check(c, chk::launch_zero_i32(ws_status(c), (int)c->probs.size(), s), "status clear");
}

static const double* class_sine(const ch_ctx* c, const ClassPlan& cp) {
  return (const double*)(c->ws + cp.sine_blk.off);
}

static ch_status fine_all(ch_ctx* c, const double* U_in, double* F_out, const uint8_t* mask,
                          const int32_t* active, const int32_t* k_min, int in_iter, hipStream_t s) {
  const InstDev* inst = (const InstDev*)(c->ws + c->inst_blk.off);
  for (auto& cp : c->classes) {
    const WorkItem* items = (const WorkItem*)(c->ws + cp.items_blk.off);
    const double* tab = class_sine(c, cp);
    hipError_t e;
    if (cp.dim == 2 && cp.fine_kind == CH_FINE_NONLINEAR) {
      e = hipErrorNotSupported;
      if (cp.fine_groups > 1) {
        e = chk::launch_fine_newton_group(cp.n, cp.fine_groups, items, (int)cp.items.size(), inst,
                                          tab, U_in, F_out, mask, active, k_min, in_iter,
                                          (int32_t*)(c->ws + cp.sync_blk.off), s);
        if (e == hipErrorCooperativeLaunchTooLarge) cp.fine_groups = 1;
      }
      if (cp.fine_groups == 1)
        e = chk::launch_fine_newton_2d(cp.n, items, (int)cp.items.size(), inst, tab, U_in, F_out,
                                       mask, active, k_min, in_iter, s);
    } else if (cp.dim == 2 && cp.fine_kind == CH_FINE_APPROX2) {
      e = chk::launch_fine_approx2_2d(cp.n, items, (int)cp.items.size(), inst, tab, U_in, F_out,
                                      mask, active, k_min, in_iter, s);
    } else if (cp.dim == 2 && cp.precision == CH_PREC_SPLIT_BF16) {
      e = chk::launch_fine_split_2d(cp.n, items, (int)cp.items.size(), inst, tab, U_in, F_out,
                                    mask, active, k_min, in_iter, s);
    } else if (cp.dim == 2) {
      e = hipErrorNotSupported;
      if (cp.fine_groups > 1) {
        e = chk::launch_fine_group(cp.n, cp.fine_groups, items, (int)cp.items.size(), inst, tab,
                                   U_in, F_out, mask, active, k_min, in_iter,
                                   (int32_t*)(c->ws + cp.sync_blk.off), s);
        // a device that cannot hold every workgroup of the group launch at
        // once takes the one-workgroup-per-item kernel
        if (e == hipErrorCooperativeLaunchTooLarge) cp.fine_groups = 1;
      }
      if (cp.fine_groups == 1)
        e = chk::launch_fine_2d(cp.n, items, (int)cp.items.size(), inst, tab, U_in, F_out,
                                mask, active, k_min, in_iter, s, cp.waves);
    } else if (cp.fine_kind == CH_FINE_APPROX2_DD) {
      e = chk::launch_fine_dd_1d(cp.n, items, (int)cp.items.size(), inst, U_in, F_out, mask,
                                 active, k_min, in_iter, s);
    } else {
      e = chk::launch_fine_1d(cp.n, items, (int)cp.items.size(), inst, tab, U_in, F_out,
                              mask, active, k_min, in_iter, s, cp.fine_kind != CH_FINE_APPROX2);
    }
    ch_status st = hip_check(c, e, "fine sweep launch");
    if (st != CH_OK) return st;
  }
  return CH_OK;
}

ch_status ch_fine_propagate(ch_ctx* c, const double* U_in, double* F_out, const uint8_t* mask,
                            ch_stream stream) {
  ch_status st = require_bound(c);
  if (st != CH_OK) return st;
  if (!U_in || !F_out) return fail(c, CH_ERR_ARG, "null state pointer");
  const size_t bytes = sizeof(double) * c->slice_total;
  const char *a = (const char*)U_in, *b = (const char*)F_out;
  if (a < b + bytes && b < a + bytes) return fail(c, CH_ERR_ARG, "U_in and F_out overlap");
  st = clear_ws_status(c, (hipStream_t)stream);
  if (st != CH_OK) return st;
  return fine_all(c, U_in, F_out, mask, nullptr, nullptr, 0, (hipStream_t)stream);
}

// Fork the caller's stream into one side stream per class after the first
// (default priority, non-blocking), so the classes' sequential coarse sweeps
// run side by side; join_sides makes the caller's stream wait for all of them.
// Both work inside a stream capture (the side streams join the capture).
static ch_status make_sides(ch_ctx* c, size_t count) {
  ch_status r;
  if (!c->fork_ev) {
    r = hip_check(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming), "fork event");
    if (r != CH_OK) return r;
  }
  while (c->side.size() < count) {
    hipStream_t q = nullptr;
    hipEvent_t e = nullptr;
    r = hip_check(c, hipStreamCreateWithFlags(&q, hipStreamNonBlocking), "side stream");
    if (r != CH_OK) return r;
    c->side.push_back(q);
    r = hip_check(c, hipEventCreateWithFlags(&e, hipEventDisableTiming), "side event");
    if (r != CH_OK) return r;
    c->side_done.push_back(e);
  }
  return CH_OK;
}
static ch_status fork_sides(ch_ctx* c, size_t count, hipStream_t s) {
  ch_status r = make_sides(c, count);
  if (r != CH_OK) return r;
  r = hip_check(c, hipEventRecord(c->fork_ev, s), "fork record");
  for (size_t i = 0; i < count && r == CH_OK; ++i)
    r = hip_check(c, hipStreamWaitEvent(c->side[i], c->fork_ev, 0), "fork wait");
  return r;
}
static ch_status join_sides(ch_ctx* c, size_t count, hipStream_t s) {
  ch_status r = CH_OK;
  for (size_t i = 0; i < count && r == CH_OK; ++i) {
    r = hip_check(c, hipEventRecord(c->side_done[i], c->side[i]), "join record");
    if (r == CH_OK) r = hip_check(c, hipStreamWaitEvent(s, c->side_done[i], 0), "join wait");
  }
  return r;
}

static ch_status coarse_all(ch_ctx* c, int mode, const double* U_in, double* G_out,
                            const uint8_t* mask, ch_pr_state* st, int k, hipStream_t s0) {
  const InstDev* inst = (const InstDev*)(c->ws + c->inst_blk.off);
  const int32_t* active = mode == 0 ? nullptr : (const int32_t*)(c->ws + c->active_blk.off);
  const int32_t* kdev = mode == 2 ? (const int32_t*)(c->ws + c->k_blk.off) : nullptr;
  double* U = st ? st->U : nullptr;
  const double* F = st ? st->F : nullptr;
  double* Gold = st ? st->G_old : nullptr;
  double* delta = st ? st->delta : nullptr;
  int32_t* status = st ? st->status : nullptr;
  // Phase 1: the sequential sweeps (modes 1, 2) that run on a group of
  // workgroups per instance.  Their members meet at device-memory barriers,
  // so each such launch needs every workgroup resident at once: they run on
  // the caller's stream, one class after another, with nothing of this call
  // beside them.
  std::vector<size_t> rest;
  for (size_t ci = 0; ci < c->classes.size(); ++ci) {
    auto& cp = c->classes[ci];
    bool coop = cp.dim == 2 && mode != 0 && cp.chain_groups > 1;
    for (int32_t i : cp.insts)
      coop = coop && c->inst[i].coarse_kind != CH_COARSE_STAB &&
             c->inst[i].coarse_kind != CH_COARSE_EYRE;
    if (!coop) { rest.push_back(ci); continue; }
    const int32_t* insts = (const int32_t*)(c->ws + cp.insts_blk.off);
    hipError_t e = chk::launch_chain_coop(cp.n, cp.chain_groups, mode, insts, (int)cp.insts.size(),
                                          inst, class_sine(c, cp), U, F, Gold, delta, status,
                                          active, k, kdev, (int32_t*)(c->ws + cp.sync_blk.off), s0);
    // a device that cannot hold every workgroup at once takes one per instance
    if (e == hipErrorCooperativeLaunchTooLarge) {
      cp.chain_groups = 1;
      rest.push_back(ci);
      continue;
    }
    ch_status r = hip_check(c, e, "coarse launch");
    if (r != CH_OK) return r;
  }
  // Phase 2: one workgroup per instance (no inter-workgroup waits).  The
  // sequential sweeps of several classes run side by side, one stream each.
  const size_t n_side = (mode != 0 && rest.size() > 1) ? rest.size() - 1 : 0;
  if (n_side) {
    ch_status r = fork_sides(c, n_side, s0);
    if (r != CH_OK) return r;
  }
  for (size_t ri = 0; ri < rest.size(); ++ri) {
    auto& cp = c->classes[rest[ri]];
    hipStream_t s = (n_side && ri > 0) ? c->side[ri - 1] : s0;
    const WorkItem* items = (const WorkItem*)(c->ws + cp.items_blk.off);
    const int32_t* insts = (const int32_t*)(c->ws + cp.insts_blk.off);
    const double* tab = class_sine(c, cp);
    hipError_t e;
    if (cp.dim == 2) {
      e = chk::launch_coarse_2d(cp.n, mode, insts, (int)cp.insts.size(), items, (int)cp.items.size(),
                                inst, tab, U_in, G_out, mask, U, F, Gold, delta, status,
                                active, k, kdev, s);
    } else {
      e = chk::launch_coarse_1d(cp.n, mode, insts, (int)cp.insts.size(), items, (int)cp.items.size(),
                                inst, tab, U_in, G_out, mask, U, F, Gold, delta, status, active, k,
                                kdev, s);
    }
    ch_status r = hip_check(c, e, "coarse launch");
    if (r != CH_OK) return r;
  }
  if (n_side) {
    ch_status r = join_sides(c, n_side, s0);
    if (r != CH_OK) return r;
  }
  hipStream_t s = s0;
  // learned coarse propagator: a sequence of network passes per instance,
  // each gated on the device by the instance's live flag (it still uses the
  // learned propagator, and is active), so that a fallback taken on the
  // device switches them off also inside a captured graph
  int32_t* jlive = nullptr;
  if (!c->judge_insts.empty()) {
    jlive = (int32_t*)(c->ws + c->jlive_blk.off);
    ch_status r = hip_check(
        c, chk::launch_judge(1, (const int32_t*)(c->ws + c->jinsts_blk.off),
                             (int)c->judge_insts.size(), (InstDev*)(c->ws + c->inst_blk.off),
                             active, jlive, nullptr, nullptr, 0, nullptr, nullptr, nullptr,
                             nullptr, 0.0, nullptr, s),
        "live flags");
    if (r != CH_OK) return r;
  }
  for (int i = 0; i < (int)c->probs.size(); ++i) {
    const InstDev& d = c->inst[i];
    if (d.coarse_kind != CH_COARSE_NEURAL) continue;
    if (!c->nn_w) return fail(c, CH_ERR_STATE, "instance %d: no surrogate weights bound", i);
    const int32_t* live = jlive + i;
    // with a plain base: G_plain of slice sl (iterate layout) into gbase,
    // gated by *gate, before the network pass of that slice
    const ClassPlan* cpi = nullptr;
    int item0 = 0;
    for (const auto& cp : c->classes) {
      int acc = 0;
      for (int32_t j : cp.insts) {
        if (j == i) { cpi = &cp; item0 = acc; }
        acc += c->probs[j].n_slices;
      }
    }
    double* gbase = d.nn_base ? (double*)(c->ws + c->nn_gbase_blk.off) + d.off_slices : nullptr;
    auto plain = [&](int mode3, int first, int count, const double* src, const int32_t* gate) {
      return chk::launch_coarse_2d(d.n, mode3, nullptr, 0,
                                   (const WorkItem*)(c->ws + cpi->items_blk.off) + item0 + first,
                                   count, inst, class_sine(c, *cpi), src,
                                   (double*)(c->ws + c->nn_gbase_blk.off), nullptr, nullptr,
                                   nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr, s, gate);
    };
    const int n = d.n, N = d.n_slices;
    const int64_t P = (int64_t)n * n;
    float* nws = (float*)(c->ws + c->nn_blk.off);
    double* g = (double*)(c->ws + c->nn_out_blk.off);
    double* part = (double*)(c->ws + c->nn_part_blk.off);
    const int nb = (int)((P + 255) / 256);
    hipError_t e = hipSuccess;
    if (mode == 0) {
      const chk::NNPlan pl = chk::nn_plan(N, n);
      if (gbase) e = plain(5, 0, N, U_in, jlive);
      if (e == hipSuccess)
        e = chk::nn_forward(c->nn_w, U_in + d.off_slices, N, n, nws, pl, g, s, live, gbase);
      if (e == hipSuccess)
        e = chk::masked_copy(G_out + d.off_slices, g, mask, P, N, d.slice_base, s, live);
    } else {
      const chk::NNPlan pl = chk::nn_plan(1, n);
      const int32_t* act = live;
      double* Ui = st->U + d.off_iter;
      const double* Fi = st->F + d.off_slices;
      double* Gi = st->G_old + d.off_slices;
      // the weights in the forward layout once for the whole sweep
      e = chk::nn_pack_forward(c->nn_w, nws, pl, s, act);
      if (mode == 1) {
        for (int sl = 0; sl < N && e == hipSuccess; ++sl) {
          if (gbase) e = plain(4, sl, 1, st->U, act);
          if (e == hipSuccess)
            e = chk::nn_forward(c->nn_w, Ui + sl * P, 1, n, nws, pl, g, s, act,
                                gbase ? gbase + sl * P : nullptr, false);
          if (e == hipSuccess) e = chk::pr_correct(Ui + (sl + 1) * P, nullptr, Gi + sl * P, g, P, part, 1, act, s);
        }
      } else {
        // the correction sweep from slice k + 1, k = the device iteration
        // counter: U_{k+1} = F_k (its G terms cancel), then for sl > k
        // U_{sl+1} = F_sl + (G(U_sl) - G_old_sl); every launch is gated on
        // the device (sl > k and the live flag), so a captured sweep serves
        // every iteration.  Eagerly, the slices up to the host's k are not
        // launched at all.  Row sl of part holds the change of U_{sl+1}.
        int32_t* gates = (int32_t*)(c->ws + c->jgate_blk.off) + d.slice_base;
        e = chk::slice_gates(act, kdev, N, gates, s);
        if (e == hipSuccess) e = chk::pr_first(Ui, Fi, P, N, part, nb, kdev, act, s);
        const int first = c->capturing ? 1 : k + 1;
        for (int sl = first; sl < N && e == hipSuccess; ++sl) {
          if (gbase) e = plain(4, sl, 1, st->U, gates + sl);
          if (e == hipSuccess)
            e = chk::nn_forward(c->nn_w, Ui + sl * P, 1, n, nws, pl, g, s, gates + sl,
                                gbase ? gbase + sl * P : nullptr, false);
          if (e == hipSuccess)
            e = chk::pr_correct(Ui + (sl + 1) * P, Fi + sl * P, Gi + sl * P, g, P,
                                part + (int64_t)sl * nb, 0, gates + sl, s);
        }
        if (e == hipSuccess)
          e = chk::pr_delta(part, nb, N, d.h * d.h, st->delta + i, st->status + i, act, s, kdev);
      }
    }
    ch_status r = hip_check(c, e, "learned coarse propagator");
    if (r != CH_OK) return r;
  }
  return CH_OK;
}

ch_status ch_coarse_propagate(ch_ctx* c, const double* U_in, double* G_out, const uint8_t* mask,
                              ch_stream stream) {
  ch_status st = require_bound(c);
  if (st != CH_OK) return st;
  if (!U_in || !G_out) return fail(c, CH_ERR_ARG, "null state pointer");
  const size_t bytes = sizeof(double) * c->slice_total;
  const char *a = (const char*)U_in, *b = (const char*)G_out;
  if (a < b + bytes && b < a + bytes) return fail(c, CH_ERR_ARG, "U_in and G_out overlap");
  st = clear_ws_status(c, (hipStream_t)stream);
  if (st != CH_OK) return st;
  return coarse_all(c, 0, U_in, G_out, mask, nullptr, 0, (hipStream_t)stream);
}

static ch_status pr_check(ch_ctx* c, ch_pr_state* st) {
  ch_status r = require_bound(c);
  if (r != CH_OK) return r;
  if (!st || !st->U || !st->F || !st->G_old || !st->delta || !st->status)
    return fail(c, CH_ERR_ARG, "incomplete ch_pr_state");
  if (st->k < 0) return fail(c, CH_ERR_ARG, "negative iteration counter");
  return CH_OK;
}

// The judge of the learned propagator, every step on the device (no host
// decision, so a captured iteration replays it):
//  what = 0 (new run): the learned propagator again for every instance
//    created with it (unless switched on the host), no fallback yet;
//  what = 1 (before the correction): the plain propagator (2.4) at the
//    current iterate, G_plain(U_n^k), per-slice distances of it and of
//    G_old_n = G(U_n^k) from F_n, and their ratio (k_judge_ratio);
//  what = 2 (after the correction): the fallback decision (k_judge_decide)
//    and, for an instance that fell back, G_old_n = G_plain(U_n^{k+1}).
static ch_status judge_step(ch_ctx* c, int what, ch_pr_state* st, double tol, hipStream_t s) {
  if (c->judge_insts.empty()) return CH_OK;
  const int32_t* jl = (const int32_t*)(c->ws + c->jinsts_blk.off);
  const int nj = (int)c->judge_insts.size();
  InstDev* inst = (InstDev*)(c->ws + c->inst_blk.off);
  int32_t* active = (int32_t*)(c->ws + c->active_blk.off);
  int32_t* kdev = (int32_t*)(c->ws + c->k_blk.off);
  int32_t* live = (int32_t*)(c->ws + c->jlive_blk.off);
  int32_t* refresh = (int32_t*)(c->ws + c->jrefresh_blk.off);
  chk::JudgeDev* J = (chk::JudgeDev*)(c->ws + c->jdev_blk.off);
  double* ratios = (double*)(c->ws + c->jratio_blk.off);
  double* gp = (double*)(c->ws + c->jgp_blk.off);
  int64_t n_slices_all = 0;
  for (const auto& p : c->probs) n_slices_all += p.n_slices;
  double* d0 = (double*)(c->ws + c->jdist_blk.off);
  double* d1 = d0 + n_slices_all;
  const int rs = c->judge_rstride;
  auto judge = [&](int k, const int32_t* act) {
    return hip_check(c, chk::launch_judge(k, jl, nj, inst, act, live, J, ratios, rs, refresh, d0,
                                          d1, st->delta, tol, kdev, s), "judge");
  };
  // the plain propagator (2.4) on every slice of the gated instances, inputs
  // from the iterate layout (mode 3), in each class holding such instances
  auto plain_all = [&](double* out, const int32_t* gate) {
    for (auto& cp : c->classes) {
      bool has = false;
      for (int32_t i : cp.insts) has = has || c->probs[i].coarse_kind == CH_COARSE_NEURAL;
      if (!has) continue;
      ch_status r = hip_check(
          c, chk::launch_coarse_2d(cp.n, 3, (const int32_t*)(c->ws + cp.insts_blk.off),
                                   (int)cp.insts.size(), (const WorkItem*)(c->ws + cp.items_blk.off),
                                   (int)cp.items.size(), inst, class_sine(c, cp), st->U, out,
                                   nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                                   nullptr, s, gate),
          "plain propagator");
      if (r != CH_OK) return r;
    }
    return CH_OK;
  };
  ch_status r = CH_OK;
  if (what == 0) return judge(0, nullptr);
  if (what == 1) {
    r = judge(1, active);
    if (r == CH_OK) r = plain_all(gp, live);
    for (auto& cp : c->classes) {
      bool has = false;
      for (int32_t i : cp.insts) has = has || c->probs[i].coarse_kind == CH_COARSE_NEURAL;
      if (!has || r != CH_OK) continue;
      const WorkItem* items = (const WorkItem*)(c->ws + cp.items_blk.off);
      r = hip_check(c, chk::launch_slice_dist(items, (int)cp.items.size(), inst, st->G_old, st->F,
                                              d0, s), "judge distances");
      if (r == CH_OK)
        r = hip_check(c, chk::launch_slice_dist(items, (int)cp.items.size(), inst, gp, st->F, d1,
                                                s), "judge distances");
    }
    if (r == CH_OK) r = judge(2, active);
    return r;
  }
  r = judge(3, active);
  if (r == CH_OK) r = plain_all(st->G_old, refresh);
  return r;
}

// One step of the iteration.  The iteration index the kernels use lives in
// device memory (k_blk) and is advanced by a kernel, so a captured step can
// be replayed for successive iterations; st->k mirrors it on the host
// (host_k = false while capturing: the replays advance only the device copy).
static ch_status pr_step(ch_ctx* c, ch_pr_state* st, double tol, hipStream_t s, int with_fine,
                         bool host_k = true) {
  int32_t* active = (int32_t*)(c->ws + c->active_blk.off);
  int32_t* kdev = (int32_t*)(c->ws + c->k_blk.off);
  const int n_inst = (int)c->probs.size();
  ch_status r;
  if (!st->predicted) {
    // a new run: st->status starts from zero and collects the flags of every
    // later call of the run
    r = hip_check(c, chk::launch_counter(kdev, 0, 0, s), "iteration counter");
    if (r == CH_OK) r = hip_check(c, chk::launch_zero_i32(st->status, n_inst, s), "status clear");
    if (r == CH_OK) r = clear_ws_status(c, s);
    if (r != CH_OK) return r;
    r = hip_check(c, chk::launch_flag_active(st->delta, active, n_inst, tol, 1, kdev, s), "flags");
    if (r == CH_OK) r = judge_step(c, 0, st, tol, s);
    if (r != CH_OK) return r;
    r = coarse_all(c, 1, nullptr, nullptr, nullptr, st, 0, s);
    if (r == CH_OK)
      r = hip_check(c, chk::launch_status_merge(st->status, ws_status(c), n_inst, s), "status");
    if (r != CH_OK) return r;
    st->predicted = 1;
    st->k = 0;
    return CH_OK;
  }
  r = hip_check(c, chk::launch_flag_active(st->delta, active, n_inst, tol, 0, kdev, s), "flags");
  if (r != CH_OK) return r;
  if (with_fine) {
    // the correction alone (with_fine == 0) keeps the flags of the caller's
    // preceding ch_fine_propagate
    r = clear_ws_status(c, s);
    if (r == CH_OK) r = fine_all(c, st->U, st->F, nullptr, active, kdev, 1, s);
    if (r != CH_OK) return r;
  }
  r = judge_step(c, 1, st, tol, s);
  if (r == CH_OK) r = coarse_all(c, 2, nullptr, nullptr, nullptr, st, st->k, s);
  if (r == CH_OK) r = judge_step(c, 2, st, tol, s);
  if (r == CH_OK)
    r = hip_check(c, chk::launch_status_merge(st->status, ws_status(c), n_inst, s), "status");
  if (r != CH_OK) return r;
  r = hip_check(c, chk::launch_counter(kdev, 1, 1, s), "iteration counter");
  if (r != CH_OK) return r;
  if (host_k) st->k += 1;
  return CH_OK;
}

ch_status ch_parareal_iterate(ch_ctx* c, ch_pr_state* st, double tol, ch_stream stream) {
  ch_status r = pr_check(c, st);
  if (r != CH_OK) return r;
  return pr_step(c, st, tol, (hipStream_t)stream, 1);
}

ch_status ch_parareal_run(ch_ctx* c, ch_pr_state* st, double tol, int32_t max_iters,
                          int32_t flags, ch_stream stream) {
  if (!c) return CH_ERR_ARG;
  // what the context covers is known on the host, before any binding
  if (!c->pipe)
    return fail(c, CH_ERR_UNSUPPORTED,
                "pipelined iterations need one 2D n = 128 instance, linear FP64 fine step, "
                "coarse scheme (2.4), N >= 2");
  const InstDev& d = c->inst[0];
  if (d.coarse_kind != CH_COARSE_APPROX2)
    return fail(c, CH_ERR_UNSUPPORTED, "pipelined iterations need the coarse scheme (2.4)");
  if (max_iters < 0) return fail(c, CH_ERR_ARG, "max_iters = %d", max_iters);
  if (flags & ~CH_RUN_SWEEP_ALL) return fail(c, CH_ERR_ARG, "unknown flags 0x%x", flags);
  ch_status r = pr_check(c, st);
  if (r != CH_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  if (!st->predicted) {
    r = pr_step(c, st, tol, s, 1);
    if (r != CH_OK) return r;
  }
  if (max_iters == 0) return CH_OK;
  int32_t* active = (int32_t*)(c->ws + c->active_blk.off);
  int32_t* kdev = (int32_t*)(c->ws + c->k_blk.off);
  r = hip_check(c, chk::launch_flag_active(st->delta, active, 1, tol, 0, kdev, s), "flags");
  if (r == CH_OK) r = clear_ws_status(c, s);
  if (r != CH_OK) return r;
  const size_t SN = (size_t)d.n_slices * d.n * d.n;
  double* F1 = (double*)(c->ws + c->pipe_blk.off);
  double* Uin = F1 + SN;
  const ClassPlan& cp = c->classes[0];
  hipError_t e = chk::launch_parareal_pipe(
      d.n, (const InstDev*)(c->ws + c->inst_blk.off), 0, d.n_slices, class_sine(c, cp), st->U,
      st->F, F1, Uin, st->G_old, st->delta, st->status, active, kdev, max_iters,
      (flags & CH_RUN_SWEEP_ALL) ? 1 : 0, tol, (int32_t*)(c->ws + c->pipe_sync_blk.off), s);
  if (e == hipErrorCooperativeLaunchTooLarge)
    return fail(c, CH_ERR_UNSUPPORTED, "the device cannot hold the pipelined launch at once");
  r = hip_check(c, e, "pipelined iterations");
  if (r != CH_OK) return r;
  return hip_check(c, chk::launch_status_merge(st->status, ws_status(c), 1, s), "status");
}

ch_status ch_parareal_correct(ch_ctx* c, ch_pr_state* st, double tol, ch_stream stream) {
  ch_status r = pr_check(c, st);
  if (r != CH_OK) return r;
  if (!st->predicted) return fail(c, CH_ERR_STATE, "the coarse prediction has not been formed");
  return pr_step(c, st, tol, (hipStream_t)stream, 0);
}

static bool tunable(const ClassPlan& cp) {
  return cp.dim == 2 && cp.fine_kind == CH_FINE_LINEAR && cp.precision == CH_PREC_FP64;
}

// Launch configurations of a class's linear fine sweep, timed by the
// autotuner: one workgroup per slice with each wave count, and groups of G
// workgroups per slice with each group size.
ch_status ch_autotune(ch_ctx* c, const double* U_in, double* F_out, int32_t steps, ch_stream stream) {
  ch_status r = require_bound(c);
  if (r != CH_OK) return r;
  if (!U_in || !F_out || steps < 1) return fail(c, CH_ERR_ARG, "autotune arguments");
  hipStream_t s = (hipStream_t)stream;
  const InstDev* inst = (const InstDev*)(c->ws + c->inst_blk.off);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(c, CH_ERR_HIP, "event create");
  for (auto& cp : c->classes) {
    if (!tunable(cp)) continue;
    int wopt[8], gopt[8];
    const int nw = chk::fine_wave_options(cp.n, wopt);
    const int ng = chk::fine_group_options(cp.n, gopt);
    float best = 1e30f;
    int best_w = wopt[0], best_g = 1;
    const WorkItem* items = (const WorkItem*)(c->ws + cp.items_blk.off);
    const int n_items = (int)cp.items.size();
    int32_t* sync = (int32_t*)(c->ws + cp.sync_blk.off);
    for (int o = 0; o < nw + ng; ++o) {
      const bool grp = o >= nw;
      auto launch = [&](int j) {
        return grp ? chk::launch_fine_group(cp.n, gopt[o - nw], items, n_items, inst,
                                            class_sine(c, cp), U_in, F_out, nullptr, nullptr,
                                            nullptr, 0, sync, s, j)
                   : chk::launch_fine_2d(cp.n, items, n_items, inst, class_sine(c, cp), U_in,
                                         F_out, nullptr, nullptr, nullptr, 0, s, wopt[o], j);
      };
      // warm-up then timed launch of `steps` fine steps over the class
      hipError_t e = launch(1);
      if (grp && (e == hipErrorCooperativeLaunchTooLarge || e == hipErrorNotSupported)) {
        (void)hipGetLastError();
        continue;             // this group size does not fit on the device
      }
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      if (e == hipSuccess) e = launch(steps);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return hip_check(c, e, "autotune run");
      }
      if (ms < best) {
        best = ms;
        best_w = grp ? wopt[0] : wopt[o];
        best_g = grp ? gopt[o - nw] : 1;
      }
    }
    cp.waves = best_w;
    cp.fine_groups = best_g;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return CH_OK;
}

ch_status ch_fine_variant(ch_ctx* c, int32_t n, int32_t* waves, int32_t set) {
  if (!c || !waves) return CH_ERR_ARG;
  bool found = false;
  for (auto& cp : c->classes) {
    if (!tunable(cp) || cp.n != n) continue;
    found = true;
    if (set) {
      int opts[8];
      const int no = chk::fine_wave_options(n, opts);
      bool ok = false;
      for (int o = 0; o < no; ++o) ok = ok || opts[o] == *waves;
      if (!ok) return fail(c, CH_ERR_ARG, "n = %d has no %d-wave variant", n, *waves);
      cp.waves = *waves;
    } else {
      int opts[8];
      chk::fine_wave_options(n, opts);
      *waves = cp.waves ? cp.waves : opts[0];
    }
  }
  return found ? CH_OK : fail(c, CH_ERR_ARG, "no tunable class with n = %d", n);
}

ch_status ch_fine_groups(ch_ctx* c, int32_t n, int32_t fine_kind, int32_t* groups, int32_t set) {
  if (!c || !groups) return CH_ERR_ARG;
  if (fine_kind < CH_FINE_LINEAR || fine_kind > CH_FINE_APPROX2)
    return fail(c, CH_ERR_ARG, "fine kind %d", fine_kind);
  bool found = false;
  for (auto& cp : c->classes) {
    if (cp.dim != 2 || cp.precision != CH_PREC_FP64 || cp.n != n || cp.fine_kind != fine_kind)
      continue;
    found = true;
    if (set) {
      const bool lin = cp.fine_kind == CH_FINE_LINEAR;
      const bool nl = cp.fine_kind == CH_FINE_NONLINEAR;
      const bool ok = *groups == 1 ||
                      (lin && n == 128 && (*groups == 4 || *groups == 8)) ||
                      (lin && n == 256 && *groups == 8) ||
                      (nl && n == 128 && *groups == 8) || (nl && n == 256 && *groups == 16);
      if (*groups != 1 && *groups != 4 && *groups != 8 && *groups != 16)
        return fail(c, CH_ERR_ARG, "fine groups must be 1, 4, 8 or 16, got %d", *groups);
      if (!ok)
        return fail(c, CH_ERR_UNSUPPORTED, "no %d-workgroup fine sweep for this class (n = %d)",
                    *groups, n);
      cp.fine_groups = *groups;
    } else {
      *groups = cp.fine_groups;
    }
  }
  return found ? CH_OK
               : fail(c, CH_ERR_ARG, "no FP64 2D class with n = %d and fine kind %d", n, fine_kind);
}

ch_status ch_chain_variant(ch_ctx* c, int32_t n, int32_t* groups, int32_t set) {
  if (!c || !groups) return CH_ERR_ARG;
  bool found = false;
  for (auto& cp : c->classes) {
    if (cp.dim != 2 || cp.n != n) continue;
    found = true;
    if (set) {
      if (*groups != 1 && *groups != 4 && *groups != 8)
        return fail(c, CH_ERR_ARG, "chain groups must be 1, 4 or 8, got %d", *groups);
      const int cap = chk::chain_coop_capacity(n);
      if (*groups > 1 && (cap == 0 || (int)cp.insts.size() * *groups > 4 * cap))
        return fail(c, CH_ERR_UNSUPPORTED, "no multi-workgroup chain for n = %d with %zu instances",
                    n, cp.insts.size());
      cp.chain_groups = *groups;
    } else {
      *groups = cp.chain_groups;
    }
  }
  return found ? CH_OK : fail(c, CH_ERR_ARG, "no 2D class with n = %d", n);
}

ch_status ch_parareal_graph_create(ch_ctx* c, ch_pr_state* st, double tol, ch_stream stream,
                                   void** graph_exec) {
  ch_status r = pr_check(c, st);
  if (r != CH_OK) return r;
  if (!graph_exec) return fail(c, CH_ERR_ARG, "null graph handle");
  if (!st->predicted) return fail(c, CH_ERR_STATE, "form the coarse prediction first");
  if (!stream) return fail(c, CH_ERR_ARG, "capture needs a non-default stream");
  hipStream_t s = (hipStream_t)stream;
  hipGraph_t g = nullptr;
  r = hip_check(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
  if (r != CH_OK) return r;
  c->capturing = true;
  ch_status inner = pr_step(c, st, tol, s, 1, false);
  c->capturing = false;
  r = hip_check(c, hipStreamEndCapture(s, &g), "end capture");
  if (inner != CH_OK) return inner;
  if (r != CH_OK) return r;
  hipGraphExec_t ex = nullptr;
  r = hip_check(c, hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "instantiate");
  (void)hipGraphDestroy(g);
  if (r != CH_OK) return r;
  *graph_exec = (void*)ex;
  return CH_OK;
}

ch_status ch_graph_launch(void* graph_exec, ch_stream stream) {
  if (!graph_exec) return CH_ERR_ARG;
  return hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream) == hipSuccess ? CH_OK
                                                                                      : CH_ERR_HIP;
}

ch_status ch_graph_destroy(void* graph_exec) {
  if (!graph_exec) return CH_ERR_ARG;
  return hipGraphExecDestroy((hipGraphExec_t)graph_exec) == hipSuccess ? CH_OK : CH_ERR_HIP;
}

ch_status ch_iteration_count(ch_ctx* c, ch_pr_state* st, ch_stream stream) {
  ch_status r = require_bound(c);
  if (r != CH_OK) return r;
  if (!st) return fail(c, CH_ERR_ARG, "null state");
  int32_t k = 0;
  hipStream_t s = (hipStream_t)stream;
  r = hip_check(c, hipMemcpyAsync(&k, c->ws + c->k_blk.off, sizeof k, hipMemcpyDeviceToHost, s),
                "counter read");
  if (r != CH_OK) return r;
  r = hip_check(c, hipStreamSynchronize(s), "counter sync");
  if (r != CH_OK) return r;
  st->k = k;
  return CH_OK;
}

ch_status ch_set_iteration(ch_ctx* c, ch_pr_state* st, int32_t k, ch_stream stream) {
  ch_status r = require_bound(c);
  if (r != CH_OK) return r;
  if (!st || k < 0) return fail(c, CH_ERR_ARG, "set iteration arguments");
  r = hip_check(c, chk::launch_counter((int32_t*)(c->ws + c->k_blk.off), k, 0, (hipStream_t)stream),
                "iteration counter");
  if (r == CH_OK) st->k = k;
  return r;
}

ch_status ch_check_status(ch_ctx* c, const ch_pr_state* st, int32_t* bits, ch_stream stream) {
  ch_status r = require_bound(c);
  if (r != CH_OK) return r;
  const int n_inst = (int)c->probs.size();
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> a(n_inst, 0), b(n_inst, 0);
  r = hip_check(c, hipMemcpyAsync(a.data(), ws_status(c), sizeof(int32_t) * n_inst,
                                  hipMemcpyDeviceToHost, s), "status read");
  if (r == CH_OK && st && st->status)
    r = hip_check(c, hipMemcpyAsync(b.data(), st->status, sizeof(int32_t) * n_inst,
                                    hipMemcpyDeviceToHost, s), "status read");
  if (r == CH_OK) r = hip_check(c, hipStreamSynchronize(s), "status sync");
  if (r != CH_OK) return r;
  int32_t all = 0, first = -1;
  for (int i = 0; i < n_inst; ++i) {
    const int32_t v = a[i] | b[i];
    if (bits) bits[i] = v;
    if (v && first < 0) first = i;
    all |= v;
  }
  if (all & 4)
    return fail(c, CH_ERR_TIMEOUT,
                "instance %d: a workgroup of a group launch waited past its limit (status 0x%x); "
                "the states of that launch are invalid", first, all);
  if (all & 3)
    return fail(c, CH_ERR_NOCONV, "instance %d: %s (status 0x%x)", first,
                (all & 2) ? "non-finite update norm" : "Newton or Krylov iteration cap reached", all);
  return CH_OK;
}

ch_status ch_set_wait_limit(ch_ctx* c, double group_seconds, double pipe_seconds,
                            ch_stream stream) {
  ch_status r = require_bound(c);
  if (r != CH_OK) return r;
  if (!(group_seconds >= 0 && group_seconds <= 60) || !(pipe_seconds >= 0 && pipe_seconds <= 60))
    return fail(c, CH_ERR_ARG, "wait limits must lie in [0, 60] s");
  for (auto& d : c->inst) {
    d.wait_ticks = (uint64_t)(group_seconds * 1e8);
    d.pipe_wait_ticks = (uint64_t)(pipe_seconds * 1e8);
  }
  hipStream_t s = (hipStream_t)stream;
  r = hip_check(c, hipMemcpyAsync(c->ws + c->inst_blk.off, c->inst.data(),
                                  sizeof(InstDev) * c->inst.size(), hipMemcpyHostToDevice, s),
                "limit upload");
  if (r != CH_OK) return r;
  return hip_check(c, hipStreamSynchronize(s), "limit sync");
}

ch_status ch_linear_bound(int32_t dim, int32_t n, double eps, double dT, int32_t J,
                          int32_t m_coarse, double i_fine, double i_coarse, double* alpha,
                          double* beta) {
  if ((dim != 1 && dim != 2) || n < 1 || !(eps > 0) || !(dT > 0) || J < 1 || m_coarse < 1 ||
      !alpha || !beta)
    return CH_ERR_ARG;
  // symbol of (I - i tau D + eps^2 tau D^2)^{-1} (I - i tau D) on the sine
  // mode with D_h eigenvalue L (D_h symmetric: the 2-norm of a polynomial in
  // it is the largest modulus over its spectrum)
  auto g = [&](double L, double tau, double i) {
    return (1.0 - i * tau * L) / (1.0 - i * tau * L + eps * eps * tau * L * L);
  };
  std::vector<double> lam(n);
  for (int k = 0; k < n; ++k) lam[k] = lap_eig(k + 1, n);
  double a = 0.0, b = 0.0;
  const int nq = dim == 2 ? n : 1;
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < nq; ++q) {
      const double L = lam[p] + (dim == 2 ? lam[q] : 0.0);
      const double gc = std::pow(g(L, dT / m_coarse, i_coarse), m_coarse);
      const double gf = std::pow(g(L, dT / J, i_fine), J);
      a = std::max(a, std::fabs(gf - gc));
      b = std::max(b, std::fabs(gc));
    }
  *alpha = a;
  *beta = b;
  return CH_OK;
}

int64_t ch_nn_param_count(void) { return chk::nn_param_count(); }

ch_status ch_nn_layer(int32_t layer, int32_t* c_in, int32_t* c_out, int32_t* k, int32_t* stride,
                      int32_t* act, int32_t* cat) {
  if (layer < 0 || layer >= chk::NN_LAYERS) return CH_ERR_ARG;
  const chk::NNLayer& L = chk::kNNLayers[layer];
  if (c_in) *c_in = L.c_in;
  if (c_out) *c_out = L.c_out;
  if (k) *k = L.k;
  if (stride) *stride = L.stride;
  if (act) *act = L.act;
  if (cat) *cat = L.cat;
  return CH_OK;
}

size_t ch_nn_workspace_bytes(int32_t batch, int32_t n) {
  if (batch < 1 || n < 8 || n % 8) return 0;
  return chk::nn_plan(batch, n).floats * sizeof(float);
}

ch_status ch_nn_forward(const uint16_t* w, const double* u, int32_t batch, int32_t n, void* ws,
                        double* out, ch_stream stream) {
  if (!w || !u || !ws || !out || batch < 1 || n < 8 || n % 8) return CH_ERR_ARG;
  const chk::NNPlan pl = chk::nn_plan(batch, n);
  return chk::nn_forward(w, u, batch, n, (float*)ws, pl, out, (hipStream_t)stream) == hipSuccess
             ? CH_OK : CH_ERR_HIP;
}

ch_status ch_nn_forward_static(const uint16_t* w, const double* u, int32_t batch, int32_t n,
                               double* out, ch_stream stream) {
  if (!w || !u || !out || batch < 1 || n < 8 || n % 8) return CH_ERR_ARG;
  const size_t need = chk::nn_forward_floats(batch, n);
  if (need > chk::NN_STATIC_FLOATS) {
    fprintf(stderr, "ch_nn_forward_static: batch %d at n = %d needs %zu floats of activations and weights, "
            "more than the %zu of the static scratch\n", batch, n, need, chk::NN_STATIC_FLOATS);
    return CH_ERR_ARG;
  }
  float* ws = nullptr;
  if (chk::nn_static_scratch(&ws) != hipSuccess) return CH_ERR_HIP;
  const chk::NNPlan pl = chk::nn_plan(batch, n);
  return chk::nn_forward(w, u, batch, n, ws, pl, out, (hipStream_t)stream) == hipSuccess
             ? CH_OK : CH_ERR_HIP;
}

ch_status ch_nn_train_step(const uint16_t* w, const double* u, const double* target, int32_t batch,
                           int32_t n, void* ws, float* grad, float* loss, ch_stream stream) {
  if (!w || !u || !target || !ws || !grad || !loss || batch < 1 || n < 8 || n % 8) return CH_ERR_ARG;
  if ((int64_t)batch * n * n > 4096 * 256) return CH_ERR_ARG;
  const chk::NNPlan pl = chk::nn_plan(batch, n);
  return chk::nn_train_step(w, u, target, batch, n, (float*)ws, pl, grad, loss,
                            (hipStream_t)stream) == hipSuccess ? CH_OK : CH_ERR_HIP;
}

ch_status ch_nn_adam(float* w_master, uint16_t* w_bf16, float* m, float* v, const float* grad,
                     int64_t count, float lr, float beta1, float beta2, float eps, int32_t step,
                     ch_stream stream) {
  if (!w_master || !w_bf16 || !m || !v || !grad || count < 1 || step < 1) return CH_ERR_ARG;
  return chk::nn_adam(w_master, w_bf16, m, v, grad, count, lr, beta1, beta2, eps, step,
                      (hipStream_t)stream) == hipSuccess ? CH_OK : CH_ERR_HIP;
}

ch_status ch_nn_to_bf16(const float* w_master, uint16_t* w_bf16, int64_t count, ch_stream stream) {
  if (!w_master || !w_bf16 || count < 1) return CH_ERR_ARG;
  return chk::nn_to_bf16(w_master, w_bf16, count, (hipStream_t)stream) == hipSuccess ? CH_OK
                                                                                      : CH_ERR_HIP;
}

ch_status ch_nn_bind(ch_ctx* c, const uint16_t* w_bf16) {
  if (!c) return CH_ERR_ARG;
  c->nn_w = w_bf16;
  return CH_OK;
}

ch_status ch_set_coarse_kind(ch_ctx* c, int32_t inst, int32_t kind, ch_stream stream) {
  ch_status r = require_bound(c);
  if (r != CH_OK) return r;
  if (inst < 0 || inst >= (int32_t)c->probs.size()) return fail(c, CH_ERR_ARG, "instance index");
  if (kind < CH_COARSE_APPROX2 || kind > CH_COARSE_EYRE) return fail(c, CH_ERR_ARG, "kind");
  if ((kind == CH_COARSE_EYRE) != (c->probs[inst].coarse_kind == CH_COARSE_EYRE))
    return fail(c, CH_ERR_UNSUPPORTED,
                "the (2.3) coarse step is chosen at creation (its Newton workspace)");
  if (c->probs[inst].dim != 2 && kind == CH_COARSE_NEURAL)
    return fail(c, CH_ERR_UNSUPPORTED, "learned coarse propagator needs 2D");
  if (kind == CH_COARSE_NEURAL && !c->nn_planned)
    return fail(c, CH_ERR_STATE, "context was created without a learned-propagator workspace");
  c->inst[inst].coarse_kind = kind;
  for (size_t t = 0; t < c->judge_insts.size(); ++t)
    if (c->judge_insts[t] == inst) {
      // the judge restores the learned propagator at a new run only while
      // the host keeps the instance on it
      c->judge_enabled[t] = kind == CH_COARSE_NEURAL;
      chk::JudgeDev* jd = (chk::JudgeDev*)(c->ws + c->jdev_blk.off) + t;
      r = hip_check(c, hipMemcpyAsync(&jd->enabled, &c->judge_enabled[t], sizeof(int32_t),
                                      hipMemcpyHostToDevice, (hipStream_t)stream),
                    "judge flag update");
      if (r != CH_OK) return r;
    }
  InstDev* dev = (InstDev*)(c->ws + c->inst_blk.off) + inst;
  return hip_check(c, hipMemcpyAsync(&dev->coarse_kind, &c->inst[inst].coarse_kind, sizeof(int32_t),
                                     hipMemcpyHostToDevice, (hipStream_t)stream),
                   "coarse kind update");
}

ch_status ch_judge_read(ch_ctx* c, int32_t inst, double* ratios, int32_t* fallback_at,
                        int32_t* learned_now, ch_stream stream) {
  ch_status r = require_bound(c);
  if (r != CH_OK) return r;
  if (inst < 0 || inst >= (int32_t)c->probs.size()) return fail(c, CH_ERR_ARG, "instance index");
  int t = -1;
  for (size_t q = 0; q < c->judge_insts.size(); ++q)
    if (c->judge_insts[q] == inst) t = (int)q;
  if (t < 0) return fail(c, CH_ERR_ARG, "instance %d was not created with the learned propagator", inst);
  hipStream_t s = (hipStream_t)stream;
  const int N = c->probs[inst].n_slices;
  chk::JudgeDev jd;
  int32_t kind = 0;
  r = hip_check(c, hipMemcpyAsync(&jd, (chk::JudgeDev*)(c->ws + c->jdev_blk.off) + t, sizeof jd,
                                  hipMemcpyDeviceToHost, s), "judge read");
  if (r == CH_OK)
    r = hip_check(c, hipMemcpyAsync(&kind, &((InstDev*)(c->ws + c->inst_blk.off) + inst)->coarse_kind,
                                    sizeof kind, hipMemcpyDeviceToHost, s), "judge read");
  if (r == CH_OK && ratios)
    r = hip_check(c, hipMemcpyAsync(ratios, (double*)(c->ws + c->jratio_blk.off) +
                                                (int64_t)t * c->judge_rstride,
                                    sizeof(double) * N, hipMemcpyDeviceToHost, s), "judge read");
  if (r == CH_OK) r = hip_check(c, hipStreamSynchronize(s), "judge sync");
  if (r != CH_OK) return r;
  if (fallback_at) *fallback_at = jd.fallback_at;
  if (learned_now) *learned_now = kind == CH_COARSE_NEURAL;
  return CH_OK;
}

// Both counts of every slice of instance inst (host, synchronous).
static ch_status read_iters(ch_ctx* c, int32_t inst, int32_t* outer, int32_t* inner,
                            ch_stream stream) {
  const int N = c->probs[inst].n_slices;
  std::vector<int32_t> v(2 * (size_t)N);
  hipStream_t s = (hipStream_t)stream;
  ch_status r = hip_check(c, hipMemcpyAsync(v.data(), (int32_t*)(c->ws + c->iters_blk.off) +
                                                          2 * c->inst[inst].slice_base,
                                            sizeof(int32_t) * 2 * N, hipMemcpyDeviceToHost, s),
                          "iteration count read");
  if (r == CH_OK) r = hip_check(c, hipStreamSynchronize(s), "iteration count sync");
  if (r != CH_OK) return r;
  for (int k = 0; k < N; ++k) {
    if (outer) outer[k] = v[2 * k];
    if (inner) inner[k] = v[2 * k + 1];
  }
  return CH_OK;
}

ch_status ch_dd_iterations(ch_ctx* c, int32_t inst, int32_t* iters, ch_stream stream) {
  ch_status r = require_bound(c);
  if (r != CH_OK) return r;
  if (inst < 0 || inst >= (int32_t)c->probs.size()) return fail(c, CH_ERR_ARG, "instance index");
  if (!iters) return fail(c, CH_ERR_ARG, "null pointer");
  if (c->probs[inst].fine_kind != CH_FINE_APPROX2_DD)
    return fail(c, CH_ERR_ARG, "instance %d does not use the Neumann-Neumann fine step", inst);
  return read_iters(c, inst, iters, nullptr, stream);
}

ch_status ch_solver_counts(ch_ctx* c, int32_t inst, int32_t* newton, int32_t* krylov,
                           ch_stream stream) {
  ch_status r = require_bound(c);
  if (r != CH_OK) return r;
  if (inst < 0 || inst >= (int32_t)c->probs.size()) return fail(c, CH_ERR_ARG, "instance index");
  if (!newton || !krylov) return fail(c, CH_ERR_ARG, "null pointer");
  const ch_problem& p = c->probs[inst];
  if (p.fine_kind != CH_FINE_NONLINEAR || p.dim != 2)
    return fail(c, CH_ERR_ARG, "instance %d does not use the 2D implicit fine step", inst);
  for (auto& cp : c->classes)
    if (cp.dim == 2 && cp.n == p.n && cp.fine_kind == p.fine_kind && cp.precision == p.precision &&
        cp.fine_groups <= 1)
      return fail(c, CH_ERR_UNSUPPORTED,
                  "instance %d runs on one workgroup per slice, which does not count", inst);
  return read_iters(c, inst, newton, krylov, stream);
}

ch_status ch_slice_distance(ch_ctx* c, const double* A, const double* B, double* out,
                            ch_stream stream) {
  ch_status st = require_bound(c);
  if (st != CH_OK) return st;
  if (!A || !B || !out) return fail(c, CH_ERR_ARG, "null pointer");
  const InstDev* inst = (const InstDev*)(c->ws + c->inst_blk.off);
  for (auto& cp : c->classes) {
    st = hip_check(c, chk::launch_slice_dist((const WorkItem*)(c->ws + cp.items_blk.off),
                                             (int)cp.items.size(), inst, A, B, out,
                                             (hipStream_t)stream),
                   "slice distance");
    if (st != CH_OK) return st;
  }
  return CH_OK;
}

ch_status ch_energy(ch_ctx* c, int32_t inst, const double* u, int32_t count, double* E_out,
                    ch_stream stream) {
  ch_status st = require_bound(c);
  if (st != CH_OK) return st;
  if (inst < 0 || inst >= (int32_t)c->probs.size()) return fail(c, CH_ERR_ARG, "instance index");
  if (count < 0 || (count > 0 && (!u || !E_out))) return fail(c, CH_ERR_ARG, "energy arguments");
  const ch_problem& p = c->probs[inst];
  return hip_check(c, chk::launch_energy(p.n, p.dim, u, count, p.eps, E_out, (hipStream_t)stream),
                   "energy launch");
}

}  // extern "C"
