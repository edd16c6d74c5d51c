// Internal declarations shared by the host runtime (ch_api.cpp) and the
// device code (ch_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <algorithm>
#include <cstdint>

namespace chk {

// Per-instance parameters, one record per instance in device memory.
struct InstDev {
  int32_t dim, n, n_slices, j_fine;
  int32_t m_coarse, coarse_kind, fine_kind, nl_variant;
  int32_t f_zero, krylov_max, newton_max, precision;
  double eps, dt, dT, s_fine, h;
  double newton_tol, krylov_rtol;
  int64_t off_slices;        // element offset of slice 0 in the slice layout
  int64_t off_iter;          // element offset of U_0 in the iterate layout
  int64_t slice_base;        // index of slice 0 among all slices (mask index)
  const double* rsig_fine;   // [n^d] 1/sigma, sigma = 1 + dt eps^2 Lam^2 - s dt Lam
  const double* rsig_stab;   // [n^d] same with tau = dT/m_coarse
  double* tab;               // 2D: TAB_VECS * n^2 spectral tables (owned order)
  double* work;              // 2D: per slice WORK_VECS * n^2 solver vectors
  int32_t* status;           // solver flags raised by fine/parallel-coarse kernels
  double nl_krylov_rtol;     // CG target inside Newton
  int32_t work_vecs;         // solver vectors per slice in `work`
  int32_t nn_base;           // learned propagator on top of the plain one
  // bounds of the inter-workgroup waits, in ticks of the 100 MHz wall clock:
  // a group barrier (default 0.2 s) and a hand-off of the pipelined launch
  // (default 10 s); a wait that runs out flags status bit 4
  uint64_t wait_ticks, pipe_wait_ticks;
  // Neumann-Neumann fine step: subdomains, iteration cap, relaxation, stop
  int32_t dd_sub, dd_max;
  int32_t direct_sub;        // subdomains of the direct 1D (2.4) solve
  double dd_theta, dd_tol;
  // per slice of the latest fine sweep that counted: [2 s] outer iterations
  // (Neumann-Neumann, or Newton in the group kernels), [2 s + 1] Krylov
  // operator applications (Newton group kernels)
  int32_t* iters;
};
constexpr uint64_t WAIT_TICKS_DEFAULT = 20000000ull;
constexpr uint64_t PIPE_WAIT_TICKS_DEFAULT = 1000000000ull;
constexpr int TAB_VECS = 4;   // d(coarse), 1/mu + tau(coarse), d(fine), 1/mu
constexpr int WORK_VECS = 7;  // x, r, p, q, minv, u_hat, y_hat (streamed Newton: 9)

struct WorkItem { int32_t inst, slice; };

// Device state of the judge of a learned-propagator instance.
struct JudgeDev {
  double delta_prev;     // update norm of the previous correction
  int32_t fallback_at;   // corrections done when it fell back (-1: not yet)
  int32_t enabled;       // the instance's kind on the host is the learned one
};

// Launch helpers implemented in ch_kernels.hip; return hipSuccess or an error.
// Fine sweep.  Work items with slice < *kmin (kmin may be null) or of an
// inactive instance are skipped; in_iter selects the iterate layout for the
// input states.
// waves: workgroup size variant (0 = default); j_steps > 0 overrides J (tuning).
hipError_t launch_fine_2d(int n, const WorkItem* items, int n_items, const InstDev* inst,
                          const double* Tsin, const double* U_in,
                          double* F_out, const uint8_t* mask, const int32_t* active,
                          const int32_t* kmin, int in_iter, hipStream_t s, int waves = 0,
                          int j_steps = 0);
int fine_wave_options(int n, int* out);
int fine_group_options(int n, int* out);
hipError_t launch_fine_newton_2d(int n, const WorkItem* items, int n_items, const InstDev* inst,
                                 const double* Tsin, const double* U_in, double* F_out,
                                 const uint8_t* mask, const int32_t* active, const int32_t* kmin,
                                 int in_iter, hipStream_t s);
// PA-I fine sweep: J steps of scheme (2.4) with tau = dt per item (2D, one
// workgroup per item; n = 256 streamed).
hipError_t launch_fine_approx2_2d(int n, const WorkItem* items, int n_items, const InstDev* inst,
                                  const double* Tsin, const double* U_in, double* F_out,
                                  const uint8_t* mask, const int32_t* active, const int32_t* kmin,
                                  int in_iter, hipStream_t s);
hipError_t launch_fine_split_2d(int n, const WorkItem* items, int n_items, const InstDev* inst,
                                const double* Tsin, const double* U_in, double* F_out,
                                const uint8_t* mask, const int32_t* active, const int32_t* kmin,
                                int in_iter, hipStream_t s);
// 1D fine sweep with the Neumann-Neumann step (n <= 128, one workgroup of
// 128 threads per item).
hipError_t launch_fine_dd_1d(int n, const WorkItem* items, int n_items, const InstDev* inst,
                             const double* U_in, double* F_out, const uint8_t* mask,
                             const int32_t* active, const int32_t* kmin, int in_iter,
                             hipStream_t s);
// sine = 0: the class's fine step needs no sine matrix in LDS (scheme (2.4),
// solved directly).
hipError_t launch_fine_1d(int n, const WorkItem* items, int n_items, const InstDev* inst,
                          const double* S, const double* U_in, double* F_out,
                          const uint8_t* mask, const int32_t* active, const int32_t* kmin,
                          int in_iter, hipStream_t s, int sine);
// mode 0: independent G per masked slice (parallel); 1: prediction chain;
// 2: correction chain starting at slice k+1 with U_{k+1} = F_k; modes 3-5:
// the plain scheme (2.4) of the given work items, outputs in the slice
// layout: 3 -- items of instances with gate[inst] != 0, inputs from the
// iterate layout U_in (U_0..U_{N-1}); 4 -- the items (one slice) when
// gate[0] != 0, iterate layout; 5 -- as 3 with slice-layout inputs.
hipError_t launch_coarse_2d(int n, int mode, const int32_t* insts, int n_insts,
                            const WorkItem* items, int n_items, const InstDev* inst,
                            const double* Tsin, const double* U_in,
                            double* G_out, const uint8_t* mask, double* U, const double* F,
                            double* G_old, double* delta, int32_t* status,
                            const int32_t* active, int k, const int32_t* kdev, hipStream_t s,
                            const int32_t* gate = nullptr);
hipError_t launch_coarse_1d(int n, int mode, const int32_t* insts, int n_insts,
                            const WorkItem* items, int n_items, const InstDev* inst,
                            const double* S, const double* U_in, double* G_out,
                            const uint8_t* mask, double* U, const double* F, double* G_old,
                            double* delta, int32_t* status, const int32_t* active, int k,
                            const int32_t* kdev, hipStream_t s);
// Linear FP64 fine sweep on groups of workgroups (2D, n = 128 or 256),
// persistent over the work items; sync: 512 ints per 8 items (cleared by the
// launch).  fine_group_capacity: largest item count for which it is the
// default; fine_group_default: the default group size.
int fine_group_capacity(int n);
int fine_group_default(int n);
hipError_t launch_fine_group(int n, int groups, const WorkItem* items, int n_items,
                             const InstDev* inst, const double* Tsin, const double* U_in,
                             double* F_out, const uint8_t* mask, const int32_t* active,
                             const int32_t* kmin, int in_iter, int32_t* sync, hipStream_t s,
                             int j_steps = 0);
// Implicit (Newton) fine sweep on groups of workgroups, persistent over the
// work items (2D; n = 128: 8 per group, n = 256: 16).
hipError_t launch_fine_newton_group(int n, int groups, const WorkItem* items, int n_items,
                                    const InstDev* inst, const double* Tsin, const double* U_in,
                                    double* F_out, const uint8_t* mask, const int32_t* active,
                                    const int32_t* kmin, int in_iter, int32_t* sync,
                                    hipStream_t s);
// Coarse chain (modes 1, 2) on a group of workgroups per instance (2D n = 128,
// scheme (2.4)); sync: 512 ints per 8 instances (cleared by the launch).
int chain_coop_capacity(int n);
hipError_t launch_chain_coop(int n, int groups, int mode, const int32_t* insts, int n_insts,
                             const InstDev* inst, const double* Tsin, double* U, const double* F,
                             double* G_old, double* delta, int32_t* status, const int32_t* active,
                             int k, const int32_t* kdev, int32_t* sync, hipStream_t s);
// Several Parareal iterations of one instance in one launch, the fine solves
// of iteration k + 1 overlapped with the coarse sweep of iteration k (2D,
// n = 128, scheme (2.4), linear FP64 fine step).  U: the instance's iterate
// layout (its first N states are copied to Uin before the launch); F0: its
// slice layout; F1 (N n^2 doubles), Uin (2 N n^2) scratch; sync:
// pipe_sync_words(N) ints (cleared by the launch).  K iterations at most,
// stopping after one whose update norm is below tol; sweep_all: no slice is
// skipped as finished.  The device counter kdev advances by the iterations
// done.
bool pipe_supported(int n);
int pipe_sync_words(int n_slices);
hipError_t launch_parareal_pipe(int n, const InstDev* inst, int ii, int n_slices,
                                const double* Tsin, double* U, double* F0, double* F1,
                                double* Uin, double* G_old, double* delta, int32_t* status,
                                const int32_t* active, int32_t* kdev, int K, int sweep_all,
                                double tol, int32_t* sync, hipStream_t s);
// Fill the per-instance CG tables (d and b-scale in the owned layout).
hipError_t launch_cg_tables(int n, int dim, const int32_t* insts, int n_insts,
                            const InstDev* inst, const double* lam, hipStream_t s);
hipError_t launch_energy(int n, int dim, const double* u, int count, double eps, double* E,
                         hipStream_t s);
// out[slice_base + slice] = ||A - B||_h per work item (slice layout).
hipError_t launch_slice_dist(const WorkItem* items, int n_items, const InstDev* inst,
                             const double* A, const double* B, double* out, hipStream_t s);
hipError_t launch_flag_active(const double* delta, int32_t* active, int n_inst, double tol,
                              int first, const int32_t* kdev, hipStream_t s);
hipError_t launch_counter(int32_t* kdev, int value, int add, hipStream_t s);
// judge of the learned propagator over the instances insts[0..n): what = 0
// reset, 1 live flags, 2 ratio of iteration *kdev, 3 fallback decision
hipError_t launch_judge(int what, const int32_t* insts, int n, InstDev* inst, const int32_t* active,
                        int32_t* live, JudgeDev* J, double* ratios, int rstride, int32_t* refresh,
                        const double* d_learned, const double* d_plain, const double* delta,
                        double tol, const int32_t* kdev, hipStream_t s);
// p[0..count) = 0 (a fill kernel, safe under stream capture)
hipError_t launch_zero_i32(int32_t* p, int count, hipStream_t s);
// dst[i] |= src[i], i < count
hipError_t launch_status_merge(int32_t* dst, const int32_t* src, int count, hipStream_t s);

// ---- learned coarse propagator (ch_nn.hip)
struct NNLayer { int c_in, c_out, k, stride, act, cat; };
constexpr int NN_LAYERS = 12;
extern const NNLayer kNNLayers[NN_LAYERS];
struct NNPlan {   // float offsets inside an NN workspace
  size_t x0, act[NN_LAYERS], wpf, grad[NN_LAYERS], tmp, part, wpart, wpd, floats;
};
NNPlan nn_plan(int batch, int n);
int64_t nn_param_count();
int64_t nn_param_offset(int layer);
// gate (device, nullable): every kernel of the pass returns at once when
// *gate == 0 (a graph-captured pass that the device switches off)
// base (nullable): out = clip(base + net(u)) instead of clip(u + net(u))
// pack: first copy the weights into the forward pass's layout in ws (false:
// nn_pack_forward has done so with these weights since ws last changed hands)
hipError_t nn_forward(const uint16_t* w, const double* u, int batch, int n, float* ws,
                      const NNPlan& p, double* out, hipStream_t s, const int32_t* gate = nullptr,
                      const double* base = nullptr, bool pack = true);
hipError_t nn_pack_forward(const uint16_t* w, float* ws, const NNPlan& p, hipStream_t s,
                           const int32_t* gate = nullptr);
// floats of workspace the forward pass alone uses (x0, the activations and
// the packed weights)
size_t nn_forward_floats(int batch, int n);
// the allocation-free forward pass: the file-scope device array of
// NN_STATIC_FLOATS floats; nn_static_scratch returns its address on the
// current device (looked up once per device)
constexpr size_t NN_STATIC_FLOATS = (size_t)8 << 20;
hipError_t nn_static_scratch(float** out);
hipError_t nn_train_step(const uint16_t* w, const double* u, const double* tgt, int batch, int n,
                         float* ws, const NNPlan& p, float* grad, float* loss, hipStream_t s);
hipError_t nn_adam(float* wm, uint16_t* wb, float* m, float* v, const float* g, int64_t count,
                   float lr, float b1, float b2, float eps, int t, hipStream_t s);
hipError_t nn_to_bf16(const float* wm, uint16_t* wb, int64_t count, hipStream_t s);
hipError_t pr_correct(double* Un1, const double* Fn, double* Gn, const double* g, int64_t count,
                      double* part, int predict, const int32_t* active, hipStream_t s);
hipError_t pr_delta(const double* part, int nb, int nslices, double h2, double* delta,
                    int32_t* status, const int32_t* active, hipStream_t s,
                    const int32_t* kdev = nullptr);
hipError_t pr_first(double* Ui, const double* Fi, int64_t P, int nslices, double* part, int nb,
                    const int32_t* kdev, const int32_t* gate, hipStream_t s);
hipError_t slice_gates(const int32_t* live, const int32_t* kdev, int nslices, int32_t* gates,
                       hipStream_t s);
hipError_t masked_copy(double* dst, const double* src, const uint8_t* mask, int64_t P, int nslices,
                       int64_t slice_base, hipStream_t s, const int32_t* gate = nullptr);

}  // namespace chk
