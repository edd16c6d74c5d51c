// Device code for the Cahn-Hilliard Parareal library, gfx950 (CDNA4).
//
// Central building block: the 2D sine transform X -> S X S^T of an n x n
// state, where S[j][k] = sqrt(2/(n+1)) sin((j+1)(k+1) pi/(n+1)) holds the
// eigenvectors of the Dirichlet difference Laplacian (paper, Section 3: D_h
// and its eigenvalues).  Each half of the transform ("stage") is one dense
// product Y = S X, done on the FP64 matrix cores (v_mfma_f64_16x16x4f64) and
// written back transposed, so two stages give S X S and four stages the
// inverse-after-forward pair of a spectral solve.  The product uses the
// even/odd symmetry S[n-1-a][b] = (-1)^b S[a][b]: with Se = S[0:n/2, even
// cols] and So = S[0:n/2, odd cols], E = Se X[even rows], O = So X[odd rows],
// Y[a] = E[a] + O[a] and Y[n-1-a] = E[a] - O[a] -- half the multiply-adds.
//
// A workgroup owns one n x n state for a whole sequence of steps: the state
// lives in LDS (n = 32, 64, 128) and never leaves the CU between the J fine
// steps of a slice.  The sine operands come from a 2(n+1)-entry table in LDS:
// S[a][b] depends only on (a+1)(b+1) mod 2(n+1), so each lane walks the table
// with an incremental index instead of holding rows of S in registers.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdint>
#include "ch_internal.h"

namespace chk {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

// A vector in "owned" order (element slot * NT + thread) accessed through a
// buffer descriptor: the per-slot offset goes in a scalar register, so an
// unrolled loop over slots needs one address register per thread instead of
// one per slot.  Accesses past n_elems read 0 / are dropped by the hardware.
struct OVec {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ OVec() {}
  __device__ __forceinline__ OVec(const double* p, int64_t n_elems)
      : r(__builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(n_elems * 8),
                                            0x00020000)) {}
  __device__ __forceinline__ double ld(int elem_off, int voff_bytes) const {
    return __builtin_bit_cast(
        double, __builtin_amdgcn_raw_buffer_load_b64(r, voff_bytes, elem_off * 8, 0));
  }
  __device__ __forceinline__ void st(int elem_off, int voff_bytes, double v) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff_bytes, elem_off * 8, 0);
  }
};

// ------------------------------------------------------------------ geometry
template <int N, int NW>
struct Geo {
  static constexpr int H = N / 2;        // folded rows
  static constexpr int TR = H / 16;      // 16-row tiles of E (and O)
  static constexpr int TC = N / 16;      // 16-col tiles
  static constexpr int WPR = NW / TR;    // waves per tile row
  static constexpr int CPW = TC / WPR;   // tile columns per wave
  static constexpr int KS = H / 4;       // k-steps of 4
  static constexpr int LDX = N + 3;      // LDS row stride: zero halo column each side, odd
                                         // stride (transposed writes spread over banks)
  static constexpr int NT = NW * 64;     // threads
  static constexpr int OWN = 8 * CPW;    // points owned per thread
  static constexpr int P2 = 2 * (N + 1);  // period of the sine table
  static constexpr int XSZ = (N + 2) * LDX;  // doubles of the LDS state incl. zero halo ring
  static constexpr int XOFF = LDX + 1;       // interior origin within the LDS state
  static_assert(NW % TR == 0, "waves must tile the folded rows");
  static_assert(TC % WPR == 0, "waves must tile the columns");
  static_assert(OWN * NT == N * N, "ownership must cover the grid");
};

// Lane coordinates.  MFMA f64 16x16x4 operand layout (lane l): A[i][k] with
// i = l%16, k = l/16; B[k][j] with k = l/16, j = l%16; D[i][j] in element r
// with i = l/16 + 4r, j = l%16.
template <int N, int NW>
struct Lane {
  int g, j, tr, c0;
  __device__ Lane() {
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    g = l >> 4;
    j = l & 15;
    tr = w / Geo<N, NW>::WPR;
    c0 = (w % Geo<N, NW>::WPR) * Geo<N, NW>::CPW;
  }
  // Output element (q, r) of this lane's E/O tiles is row a, column c; it
  // produces Y[a][c] (slot half 0) and Y[N-1-a][c] (half 1), which are
  // written transposed, i.e. to state positions (row c, col a) and
  // (row c, col N-1-a).  These are the points the thread "owns".
  __device__ __forceinline__ int row_a(int r) const { return 16 * tr + g + 4 * r; }
  __device__ __forceinline__ int col_c(int q) const { return 16 * (c0 + q) + j; }
};

// Sine-table walk of one lane: the A operand of k-step ks is
// Se[16 tr + j][4 ks + g] = S[a][2(4ks+g)]   (E)  and
// So[16 tr + j][4 ks + g] = S[a][2(4ks+g)+1] (O), a = 16 tr + j, i.e. table
// entries (a+1)(8ks+2g+1) and (a+1)(8ks+2g+2) mod 2(n+1).
struct SineWalk {
  int e0, o0, step;
};
template <int N, int NW>
__device__ __forceinline__ SineWalk sine_walk(const Lane<N, NW>& L) {
  constexpr int P2 = Geo<N, NW>::P2;
  const int a1 = 16 * L.tr + L.j + 1;
  SineWalk w;
  w.e0 = (a1 * (2 * L.g + 1)) % P2;
  w.o0 = (a1 * (2 * L.g + 2)) % P2;
  w.step = (8 * a1) % P2;
  return w;
}
// Table T[m] = sqrt(2/(n+1)) sin(m pi/(n+1)), m < 2(n+1), copied to LDS.
template <int N, int NW>
__device__ __forceinline__ void load_sine_table(double* T, const double* __restrict__ Tg) {
  for (int m = threadIdx.x; m < Geo<N, NW>::P2; m += Geo<N, NW>::NT) T[m] = Tg[m];
}

// One stage: accumulators E = Se X[even rows], O = So X[odd rows] for this
// wave's tiles.  X is the LDS state (row stride LDX), T the LDS sine table.
// Software-pipelined: the operands of k-step ks+1 are read from LDS while the
// MFMAs of k-step ks run; the scheduling barrier keeps the compiler from
// hoisting every read of the unrolled loop.
template <int N, int NW>
__device__ __forceinline__ void mma_stage(const double* X, const double* T, const SineWalk& sw,
                                          d4 (&aE)[Geo<N, NW>::CPW], d4 (&aO)[Geo<N, NW>::CPW],
                                          const Lane<N, NW>& L) {
  using G = Geo<N, NW>;
#pragma unroll
  for (int q = 0; q < G::CPW; ++q) {
    aE[q] = d4{0.0, 0.0, 0.0, 0.0};
    aO[q] = d4{0.0, 0.0, 0.0, 0.0};
  }
  const double* base = X + (2 * L.g) * G::LDX + 16 * L.c0 + L.j;
  int ie = sw.e0, io = sw.o0;
  double se = T[ie], so = T[io];
  double be[G::CPW], bo[G::CPW];
#pragma unroll
  for (int q = 0; q < G::CPW; ++q) {
    be[q] = base[16 * q];
    bo[q] = base[G::LDX + 16 * q];
  }
#pragma unroll
  for (int ks = 0; ks < G::KS; ++ks) {
    double ne[G::CPW], no[G::CPW], nse = 0.0, nso = 0.0;
    if (ks + 1 < G::KS) {
      ie += sw.step;
      ie -= (ie >= G::P2) ? G::P2 : 0;
      io += sw.step;
      io -= (io >= G::P2) ? G::P2 : 0;
      nse = T[ie];
      nso = T[io];
      const double* pe = base + (8 * (ks + 1)) * G::LDX;
#pragma unroll
      for (int q = 0; q < G::CPW; ++q) {
        ne[q] = pe[16 * q];
        no[q] = pe[G::LDX + 16 * q];
      }
    }
#pragma unroll
    for (int q = 0; q < G::CPW; ++q) {
      aE[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(se, be[q], aE[q], 0, 0, 0);
      aO[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(so, bo[q], aO[q], 0, 0, 0);
    }
    if (ks + 1 < G::KS) {
      se = nse;
      so = nso;
#pragma unroll
      for (int q = 0; q < G::CPW; ++q) {
        be[q] = ne[q];
        bo[q] = no[q];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Unfold accumulators into the owned values y[slot]: slot (q*4+r)*2 + 0 is
// Y[a][c], slot +1 is Y[N-1-a][c].
template <int N, int NW>
__device__ __forceinline__ void unfold(const d4 (&aE)[Geo<N, NW>::CPW],
                                       const d4 (&aO)[Geo<N, NW>::CPW],
                                       double (&y)[Geo<N, NW>::OWN]) {
#pragma unroll
  for (int q = 0; q < Geo<N, NW>::CPW; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      y[(q * 4 + r) * 2 + 0] = aE[q][r] + aO[q][r];
      y[(q * 4 + r) * 2 + 1] = aE[q][r] - aO[q][r];
    }
}

// Offsets (in X) of the owned points.
template <int N, int NW>
__device__ __forceinline__ int own_off(const Lane<N, NW>& L, int slot) {
  const int qr = slot >> 1, half = slot & 1;
  const int q = qr >> 2, r = qr & 3;
  const int a = L.row_a(r), c = L.col_c(q);
  return c * Geo<N, NW>::LDX + (half ? (N - 1 - a) : a);
}
template <int N, int NW>
__device__ __forceinline__ void own_rc(const Lane<N, NW>& L, int slot, int& row, int& col) {
  const int qr = slot >> 1, half = slot & 1;
  const int q = qr >> 2, r = qr & 3;
  const int a = L.row_a(r);
  row = L.col_c(q);
  col = half ? (N - 1 - a) : a;
}

template <int N, int NW>
__device__ __forceinline__ void store_owned(double* X, const Lane<N, NW>& L,
                                            const double (&y)[Geo<N, NW>::OWN]) {
#pragma unroll
  for (int s = 0; s < Geo<N, NW>::OWN; ++s) X[own_off<N, NW>(L, s)] = y[s];
}
template <int N, int NW>
__device__ __forceinline__ void load_owned(const double* X, const Lane<N, NW>& L,
                                           double (&y)[Geo<N, NW>::OWN]) {
#pragma unroll
  for (int s = 0; s < Geo<N, NW>::OWN; ++s) y[s] = X[own_off<N, NW>(L, s)];
}

// Full stage: X <- (S X)^T, optionally scaled pointwise by w at the owned
// (row, col) positions of the result (w in row-major n x n, may be null).
template <int N, int NW>
__device__ __forceinline__ void stage(double* X, const double* T, const SineWalk& sw,
                                      const Lane<N, NW>& L, const double* __restrict__ w) {
  using G = Geo<N, NW>;
  d4 aE[G::CPW], aO[G::CPW];
  mma_stage<N, NW>(X, T, sw, aE, aO, L);
  double y[G::OWN];
  unfold<N, NW>(aE, aO, y);
  if (w) {
    // w is symmetric: read w[col][row] so that lanes with consecutive
    // rows (consecutive j) read consecutive addresses.
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) {
      int row, col;
      own_rc<N, NW>(L, s, row, col);
      y[s] *= w[col * N + row];
    }
  }
  __syncthreads();  // every wave has finished reading X
  store_owned<N, NW>(X, L, y);
  __syncthreads();
}

// Last stage of a pass: the result stays in registers (owned values).
template <int N, int NW>
__device__ __forceinline__ void stage_regs(const double* X, const double* T, const SineWalk& sw,
                                           const Lane<N, NW>& L, double (&y)[Geo<N, NW>::OWN]) {
  using G = Geo<N, NW>;
  d4 aE[G::CPW], aO[G::CPW];
  mma_stage<N, NW>(X, T, sw, aE, aO, L);
  unfold<N, NW>(aE, aO, y);
}

// ------------------------------------------------------------ reductions
template <int NW>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <int NW>
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
// Deterministic block sums of K values at once (fixed tree, fixed wave order).
template <int NW, int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = wave_sum<NW>(v[i]);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0)
#pragma unroll
    for (int i = 0; i < K; ++i) red[i * NW + w] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double s = 0.0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) s += red[i * NW + ww];
    v[i] = s;
  }
}
template <int NW>
__device__ __forceinline__ void block_minmax(double& mn, double& mx, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o, 64));
    mx = fmax(mx, __shfl_xor(mx, o, 64));
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) {
    red[w] = mn;
    red[NW + w] = mx;
  }
  __syncthreads();
  mn = red[0];
  mx = red[NW];
#pragma unroll
  for (int ww = 1; ww < NW; ++ww) {
    mn = fmin(mn, red[ww]);
    mx = fmax(mx, red[NW + ww]);
  }
}

// ------------------------------------------------- linear stabilised step
// Right-hand side of the linear step at the owned points, from the owned
// state values v (in registers, state orientation):
//   r = u + c_lap * Lap5(f(u) - s u),  c_lap = tau / h^2  (zero boundary ghosts).
// Leaves r in X (state orientation).
template <int N, int NW>
__device__ __forceinline__ void rhs_owned(double* X, const Lane<N, NW>& L,
                                          double (&v)[Geo<N, NW>::OWN], double c_lap, double s,
                                          int f_zero) {
  using G = Geo<N, NW>;
#pragma unroll
  for (int k = 0; k < G::OWN; ++k) {
    const double u = v[k];  // w = f(u) - s u (zero on the boundary)
    X[own_off<N, NW>(L, k)] = f_zero ? (-s * u) : (u * u * u - (1.0 + s) * u);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < G::OWN; ++k) {
    int row, col;
    own_rc<N, NW>(L, k, row, col);
    // the zero halo ring of X supplies the Dirichlet ghost values
    const double* p = X + row * G::LDX + col;
    const double wc = p[0];
    const double wn = p[-G::LDX];
    const double ws = p[G::LDX];
    const double ww = p[-1];
    const double we = p[1];
    v[k] = v[k] + c_lap * ((wn + ws) + (ww + we) - 4.0 * wc);
  }
  __syncthreads();
  store_owned<N, NW>(X, L, v);
  __syncthreads();
}

// nsteps linear steps starting from the state in X (state orientation);
// the result is left in X and in v.
template <int N, int NW>
__device__ void linear_steps(double* X, const double* T, const SineWalk& sw, const Lane<N, NW>& L,
                             double (&v)[Geo<N, NW>::OWN], int nsteps, double c_lap, double s,
                             int f_zero, const double* __restrict__ rsig) {
  load_owned<N, NW>(X, L, v);
  for (int m = 0; m < nsteps; ++m) {
    rhs_owned<N, NW>(X, L, v, c_lap, s, f_zero);
    stage<N, NW>(X, T, sw, L, nullptr);  // X = (S r)^T
    stage<N, NW>(X, T, sw, L, rsig);     // X = (S r S) / sigma   (spectral)
    stage<N, NW>(X, T, sw, L, nullptr);
    stage_regs<N, NW>(X, T, sw, L, v);   // v = S (.) S   (state, owned)
    __syncthreads();
    store_owned<N, NW>(X, L, v);
    __syncthreads();
  }
}

// Zero the whole LDS state buffer (the halo ring stays zero afterwards: the
// transform stages only ever write interior points).  Xbuf = buffer start.
template <int N, int NW>
__device__ __forceinline__ void zero_state(double* Xbuf) {
  for (int i = threadIdx.x; i < Geo<N, NW>::XSZ; i += Geo<N, NW>::NT) Xbuf[i] = 0.0;
}
template <int N, int NW>
__device__ __forceinline__ void load_state(double* X, const double* __restrict__ src) {
  using G = Geo<N, NW>;
  for (int idx = threadIdx.x; idx < N * N; idx += G::NT) X[(idx / N) * G::LDX + (idx % N)] = src[idx];
}
template <int N, int NW>
__device__ __forceinline__ void store_state(const double* X, double* __restrict__ dst) {
  using G = Geo<N, NW>;
  for (int idx = threadIdx.x; idx < N * N; idx += G::NT) dst[idx] = X[(idx / N) * G::LDX + (idx % N)];
}

// Fine sweep: one workgroup per (instance, slice) work item; J linear steps
// of dt, the state resident in LDS throughout.
template <int N, int NW>
__global__ void __launch_bounds__(NW * 64)
k_fine_linear_2d(const WorkItem* __restrict__ items, const InstDev* __restrict__ inst,
                 const double* __restrict__ Tg, const double* __restrict__ U_in,
                 double* __restrict__ F_out, const uint8_t* __restrict__ mask,
                 const int32_t* __restrict__ active, const int32_t* __restrict__ kmin, int in_iter,
                 int j_steps) {
  extern __shared__ double smem[];
  double* X = smem + Geo<N, NW>::XOFF;   // interior origin
  double* T = smem + Geo<N, NW>::XSZ;
  const WorkItem it = items[blockIdx.x];
  const InstDev P = inst[it.inst];
  if (mask && !mask[P.slice_base + it.slice]) return;
  if ((kmin && it.slice < *kmin) || (active && !active[it.inst])) return;
  const int64_t off = P.off_slices + (int64_t)it.slice * N * N;
  const int64_t off_in = (in_iter ? P.off_iter : P.off_slices) + (int64_t)it.slice * N * N;
  Lane<N, NW> L;
  const SineWalk sw = sine_walk<N, NW>(L);
  load_sine_table<N, NW>(T, Tg);
  zero_state<N, NW>(smem);
  __syncthreads();
  load_state<N, NW>(X, U_in + off_in);
  __syncthreads();
  double v[Geo<N, NW>::OWN];
  linear_steps<N, NW>(X, T, sw, L, v, j_steps > 0 ? j_steps : P.j_fine, P.dt / (P.h * P.h),
                      P.s_fine, P.f_zero, P.rsig_fine);
  store_state<N, NW>(X, F_out + off);
}

// ------------------------------------------------------- spectral CG
constexpr int CG_CHUNK = 8;
// Both the coarse scheme (2.4) and the Newton steps of the implicit fine
// schemes need solves with operators of the form
//   I + tau eps^2 Lap^2 - tau Lap diag(q)      (q >= 0, or q = 3Y^2 - 1),
// which, multiplied by A^{-1} with A = -Lap (SPD), become the SPD operator
//   K = A^{-1} + tau eps^2 A + tau diag(q).
// In sine coordinates xh = S x S:  K_hat = diag(d) + tau S diag(q) S with
// d = 1/mu + tau eps^2 mu, mu = -(lam_p + lam_q).  CG from x = 0 with the
// diagonal preconditioner diag(d + tau c), c = (min q + max q)/2; one
// operator application = one inverse and one forward 2D sine transform.
// Vectors live in the work item's scratch in owned order (slot * NT +
// thread: coalesced for every thread).  b: owned spectral right-hand side.
// Returns the iteration count, or -1 when the cap is hit or the residual
// is not finite.  The result is left in cx.
template <int N, int NW>
__device__ int spectral_cg(double* X, double* red, const double* T, const SineWalk& sw,
                           const Lane<N, NW>& L, const OVec& cx, const OVec& cr_unused,
                           const OVec& cp_unused, const OVec& cq, const OVec& cm,
                           const OVec& cd, double tau, double cshift, double rtol, int maxit,
                           const double (&b)[Geo<N, NW>::OWN]) {
  // The direction p and the residual r stay in registers (owned values);
  // x, M^{-1}, d and q are read through buffer descriptors.
  using G = Geo<N, NW>;
  const int vo = threadIdx.x * 8;
  double y[G::OWN], pv[G::OWN], rv[G::OWN];
  double acc[2] = {0.0, 0.0};
  {
    double dv[G::OWN];
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) dv[s] = cd.ld(s * G::NT, vo);
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) {
      const int o = s * G::NT;
      const double mi = 1.0 / (dv[s] + tau * cshift);
      cm.st(o, vo, mi);
      cx.st(o, vo, 0.0);
      rv[s] = b[s];
      pv[s] = b[s] * mi;
      acc[0] += b[s] * pv[s];
      acc[1] += b[s] * b[s];
    }
  }
  block_sum<NW, 2>(acc, red);
  double rz = acc[0];
  const double bb = acc[1];
  if (!(bb > 0.0)) return 0;
  const double stop2 = rtol * rtol * bb;
  for (int it = 1; it <= maxit; ++it) {
    __syncthreads();
    store_owned<N, NW>(X, L, pv);  // X = p (spectral, owned orientation)
    __syncthreads();
    // K p = d p + tau S (q . S p S) S
    stage<N, NW>(X, T, sw, L, nullptr);
    stage_regs<N, NW>(X, T, sw, L, y);
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) y[s] *= cq.ld(s * G::NT, vo);
    __syncthreads();
    store_owned<N, NW>(X, L, y);
    __syncthreads();
    stage<N, NW>(X, T, sw, L, nullptr);
    stage_regs<N, NW>(X, T, sw, L, y);
    double a1[1] = {0.0};
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) {
      const double kp = cd.ld(s * G::NT, vo) * pv[s] + tau * y[s];
      y[s] = kp;
      a1[0] += pv[s] * kp;
    }
    block_sum<NW, 1>(a1, red);
    const double alpha = rz / a1[0];
    double a2[2] = {0.0, 0.0};
#pragma unroll
    for (int s0 = 0; s0 < G::OWN; s0 += CG_CHUNK) {
      double xv[CG_CHUNK], mv[CG_CHUNK];
#pragma unroll
      for (int c = 0; c < CG_CHUNK; ++c) {
        xv[c] = cx.ld((s0 + c) * G::NT, vo);
        mv[c] = cm.ld((s0 + c) * G::NT, vo);
      }
#pragma unroll
      for (int c = 0; c < CG_CHUNK; ++c) {
        const int s = s0 + c;
        xv[c] += alpha * pv[s];
        rv[s] -= alpha * y[s];
        const double z = rv[s] * mv[c];
        a2[0] += rv[s] * rv[s];
        a2[1] += rv[s] * z;
        y[s] = z;
      }
#pragma unroll
      for (int c = 0; c < CG_CHUNK; ++c) cx.st((s0 + c) * G::NT, vo, xv[c]);
    }
    block_sum<NW, 2>(a2, red);
    if (a2[0] <= stop2) return it;
    if (!(a2[0] == a2[0])) return -1;
    const double beta = a2[1] / rz;
    rz = a2[1];
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) pv[s] = y[s] + beta * pv[s];
  }
  return -1;
}

// Variant with every CG vector in memory (lower register use).
template <int N, int NW>
__device__ int spectral_cg_mem(double* X, double* red, const double* T, const SineWalk& sw,
                           const Lane<N, NW>& L, const OVec& cx, const OVec& cr, const OVec& cp,
                           const OVec& cq, const OVec& cm, const OVec& cd, double tau,
                           double cshift, double rtol, int maxit,
                           const double (&b)[Geo<N, NW>::OWN]) {
  using G = Geo<N, NW>;
  const int vo = threadIdx.x * 8;
  double y[G::OWN];
  double acc[2] = {0.0, 0.0};
  double dv[G::OWN];
#pragma unroll
  for (int s = 0; s < G::OWN; ++s) dv[s] = cd.ld(s * G::NT, vo);
#pragma unroll
  for (int s = 0; s < G::OWN; ++s) {
    const int o = s * G::NT;
    const double mi = 1.0 / (dv[s] + tau * cshift);
    cm.st(o, vo, mi);
    cx.st(o, vo, 0.0);
    cr.st(o, vo, b[s]);
    const double z = b[s] * mi;
    cp.st(o, vo, z);
    y[s] = z;
    acc[0] += b[s] * z;
    acc[1] += b[s] * b[s];
  }
  block_sum<NW, 2>(acc, red);
  double rz = acc[0];
  const double bb = acc[1];
  if (!(bb > 0.0)) return 0;
  const double stop2 = rtol * rtol * bb;
  __syncthreads();
  store_owned<N, NW>(X, L, y);  // X = p (spectral, owned orientation)
  __syncthreads();
  for (int it = 1; it <= maxit; ++it) {
    // K p = d p + tau S (q . S p S) S: two stages to the state, the pointwise
    // q at the owned state points, two stages back.
    stage<N, NW>(X, T, sw, L, nullptr);
    stage_regs<N, NW>(X, T, sw, L, y);
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) y[s] *= cq.ld(s * G::NT, vo);
    __syncthreads();
    store_owned<N, NW>(X, L, y);
    __syncthreads();
    stage<N, NW>(X, T, sw, L, nullptr);
    stage_regs<N, NW>(X, T, sw, L, y);
    double a1[1] = {0.0};
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) {
      const int o = s * G::NT;
      const double p = cp.ld(o, vo);
      const double kp = cd.ld(o, vo) * p + tau * y[s];
      y[s] = kp;
      a1[0] += p * kp;
    }
    block_sum<NW, 1>(a1, red);
    const double alpha = rz / a1[0];
    double a2[2] = {0.0, 0.0};
    // Chunked: the buffer accesses carry no alias information, so every
    // load of a chunk is issued before its stores (one memory round trip
    // per chunk instead of one per slot).
#pragma unroll
    for (int s0 = 0; s0 < G::OWN; s0 += CG_CHUNK) {
      double xv[CG_CHUNK], pv[CG_CHUNK], rv[CG_CHUNK], mv[CG_CHUNK];
#pragma unroll
      for (int c = 0; c < CG_CHUNK; ++c) {
        const int o = (s0 + c) * G::NT;
        xv[c] = cx.ld(o, vo);
        pv[c] = cp.ld(o, vo);
        rv[c] = cr.ld(o, vo);
        mv[c] = cm.ld(o, vo);
      }
#pragma unroll
      for (int c = 0; c < CG_CHUNK; ++c) {
        xv[c] += alpha * pv[c];
        rv[c] -= alpha * y[s0 + c];
        a2[0] += rv[c] * rv[c];
        a2[1] += rv[c] * (rv[c] * mv[c]);
        y[s0 + c] = rv[c] * mv[c];   // z = M^{-1} r, kept for the direction update
      }
#pragma unroll
      for (int c = 0; c < CG_CHUNK; ++c) {
        const int o = (s0 + c) * G::NT;
        cx.st(o, vo, xv[c]);
        cr.st(o, vo, rv[c]);
      }
    }
    block_sum<NW, 2>(a2, red);
    if (a2[0] <= stop2) return it;
    if (!(a2[0] == a2[0])) return -1;
    const double beta = a2[1] / rz;
    rz = a2[1];
#pragma unroll
    for (int s0 = 0; s0 < G::OWN; s0 += CG_CHUNK) {
      double pv[CG_CHUNK];
#pragma unroll
      for (int c = 0; c < CG_CHUNK; ++c) pv[c] = cp.ld((s0 + c) * G::NT, vo);
#pragma unroll
      for (int c = 0; c < CG_CHUNK; ++c) {
        y[s0 + c] = y[s0 + c] + beta * pv[c];
        cp.st((s0 + c) * G::NT, vo, y[s0 + c]);
      }
    }
    __syncthreads();
    store_owned<N, NW>(X, L, y);
    __syncthreads();
  }
  return -1;
}

// Work vectors of one work item (owned order, n^2 each) and the instance's
// spectral tables.
struct Work {
  OVec x, r, p, q, m, uh, yh;
  OVec d_coarse, b_coarse, d_fine, imu;
};
__device__ __forceinline__ Work work_vectors(const InstDev& P, int slice) {
  const int64_t NN = (int64_t)P.n * P.n;
  double* w = P.work + (int64_t)slice * P.work_vecs * NN;
  Work W;
  W.x = OVec(w, NN);
  W.r = OVec(w + NN, NN);
  W.p = OVec(w + 2 * NN, NN);
  W.q = OVec(w + 3 * NN, NN);
  W.m = OVec(w + 4 * NN, NN);
  W.uh = OVec(w + 5 * NN, NN);
  W.yh = OVec(w + 6 * NN, NN);
  W.d_coarse = OVec(P.tab, NN);
  W.b_coarse = OVec(P.tab + NN, NN);
  W.d_fine = OVec(P.tab + 2 * NN, NN);
  W.imu = OVec(P.tab + 3 * NN, NN);
  return W;
}

// q at the owned state points (state values in y), stored to cq; returns the
// preconditioner shift (min q + max q)/2.
template <int N, int NW>
__device__ __forceinline__ double set_q(const OVec& cq, double* red,
                                        const double (&y)[Geo<N, NW>::OWN], double a3, double a0) {
  using G = Geo<N, NW>;
  const int vo = threadIdx.x * 8;
  double mn = 1e300, mx = -1e300;
#pragma unroll
  for (int s = 0; s < G::OWN; ++s) {
    const double q = a3 * y[s] * y[s] + a0;
    cq.st(s * G::NT, vo, q);
    mn = fmin(mn, q);
    mx = fmax(mx, q);
  }
  block_minmax<NW>(mn, mx, red);
  return 0.5 * (mn + mx);
}

// Scheme (2.4): (I - tau Lap diag(u^2) + eps^2 tau Lap^2) v = (I - tau Lap) u,
// i.e. K v = A^{-1} u + tau u with q = u^2 (f == 0: q = 0 and K v = A^{-1} u).
// The state u is in X (state orientation) on entry; v is left there after
// `steps` steps of tau.  d: the table 1/mu + tau eps^2 mu of this tau; the
// right-hand side scale is bt + boff (bt a table, boff a constant), i.e.
// 1/mu + tau (f == 0: 1/mu): the coarse step passes the table 1/mu + tau with
// boff = 0 (f == 0: -tau), the fine step (PA-I) the table 1/mu with boff =
// tau (f == 0: 0).  rtol: the CG stop.
template <int N, int NW>
__device__ void approx2_steps(double* X, double* red, const double* T, const SineWalk& sw,
                              const Lane<N, NW>& L, const InstDev& P, const Work& W, double tau,
                              int steps, const OVec& d, const OVec& bt, double boff, double rtol,
                              int& status) {
  using G = Geo<N, NW>;
  const int vo = threadIdx.x * 8;
  double y[G::OWN], b[G::OWN];
  for (int sub = 0; sub < steps; ++sub) {
    load_owned<N, NW>(X, L, y);
    const double cshift = set_q<N, NW>(W.q, red, y, P.f_zero ? 0.0 : 1.0, 0.0);
    stage<N, NW>(X, T, sw, L, nullptr);
    stage_regs<N, NW>(X, T, sw, L, y);   // u_hat
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) {
      const double cb = bt.ld(s * G::NT, vo);
      b[s] = (cb + boff) * y[s];
    }
    const int its = spectral_cg<N, NW>(X, red, T, sw, L, W.x, W.r, W.p, W.q, W.m, d, tau,
                                       cshift, rtol, P.krylov_max, b);
    if (its < 0) status |= 1;
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) y[s] = W.x.ld(s * G::NT, vo);
    __syncthreads();
    store_owned<N, NW>(X, L, y);
    __syncthreads();
    stage<N, NW>(X, T, sw, L, nullptr);
    stage<N, NW>(X, T, sw, L, nullptr);
  }
}

// ------------------------------------------------ implicit fine step
// One step of scheme (2.3) (nl_variant 0) or of backward Euler (1) from the
// state u to the root Y of H, by Newton's method from Y_0 = u, stopped when
// ||Y_{m+1} - Y_m||_h <= newton_tol (returning Y_{m+1}).  With A = -Lap,
//   (2.3): A^{-1} H(Y) = A^{-1}(Y - u) + tau eps^2 A Y + tau (Y^3 - u),
//   BE   : A^{-1} H(Y) = A^{-1}(Y - u) + tau eps^2 A Y + tau (Y^3 - Y),
// and the Newton matrix A^{-1} H'(Y) = A^{-1} + tau eps^2 A + tau diag(q),
// q = 3Y^2 (2.3) or 3Y^2 - 1 (BE), is SPD (BE: for tau < 4 eps^2).  In sine
// coordinates A^{-1} H = d Yh + tau S(Y^3)S - (1/mu + tau) uh (2.3), or
// d Yh + tau S(Y^3)S - tau Yh - uh/mu (BE), with d = 1/mu + tau eps^2 mu.
// The state is carried in sine coordinates (Yh, uh in the work vectors).
// Returns false if Newton or CG hit a cap.
// tau: the step; dtab: the table 1/mu + tau eps^2 mu of that tau; be: the
// backward-Euler variant.
template <int N, int NW>
__device__ bool newton_step(double* X, double* red, const double* T, const SineWalk& sw,
                            const Lane<N, NW>& L, const InstDev& P, const Work& W, double tau,
                            const OVec& dtab, bool be) {
  using G = Geo<N, NW>;
  const int vo = threadIdx.x * 8;
  double y[G::OWN], b[G::OWN];
  bool ok = true;
  for (int it = 0; it < P.newton_max; ++it) {
    // Y at the owned state points: two stages from Yh
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) y[s] = W.yh.ld(s * G::NT, vo);
    __syncthreads();
    store_owned<N, NW>(X, L, y);
    __syncthreads();
    stage<N, NW>(X, T, sw, L, nullptr);
    stage_regs<N, NW>(X, T, sw, L, y);
    const double cshift = set_q<N, NW>(W.q, red, y, P.f_zero ? 0.0 : 3.0,
                                       (be && !P.f_zero) ? -1.0 : 0.0);
    // S (Y^3) S
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) y[s] = P.f_zero ? 0.0 : y[s] * y[s] * y[s];
    __syncthreads();
    store_owned<N, NW>(X, L, y);
    __syncthreads();
    stage<N, NW>(X, T, sw, L, nullptr);
    stage_regs<N, NW>(X, T, sw, L, y);
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) {
      const int o = s * G::NT;
      const double yh = W.yh.ld(o, vo), uh = W.uh.ld(o, vo);
      const double d = dtab.ld(o, vo), im = W.imu.ld(o, vo);
      double g;
      if (P.f_zero) g = d * yh - im * uh;
      else if (be) g = d * yh + tau * y[s] - tau * yh - im * uh;
      else g = d * yh + tau * y[s] - (im + tau) * uh;
      b[s] = -g;
    }
    const int its = spectral_cg_mem<N, NW>(X, red, T, sw, L, W.x, W.r, W.p, W.q, W.m, dtab,
                                           tau, cshift, P.nl_krylov_rtol, P.krylov_max, b);
    if (its < 0) ok = false;
    double a[1] = {0.0};
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) {
      const int o = s * G::NT;
      const double dx = W.x.ld(o, vo);
      W.yh.st(o, vo, W.yh.ld(o, vo) + dx);
      a[0] += dx * dx;
    }
    block_sum<NW, 1>(a, red);
    const double step = sqrt(P.h * P.h * a[0]);  // ||S dYh S||_h = h ||dYh||_F
    if (step <= P.newton_tol) return ok;
    if (!(step == step)) return false;
  }
  return false;
}

// Implicit fine sweep: one workgroup per work item, J Newton-solved steps.
template <int N, int NW>
__global__ void __launch_bounds__(NW * 64)
k_fine_newton_2d(const WorkItem* __restrict__ items, const InstDev* __restrict__ inst,
                 const double* __restrict__ Tg, const double* __restrict__ U_in,
                 double* __restrict__ F_out, const uint8_t* __restrict__ mask,
                 const int32_t* __restrict__ active, const int32_t* __restrict__ kmin, int in_iter) {
  using G = Geo<N, NW>;
  extern __shared__ double smem[];
  double* X = smem + G::XOFF;
  double* T = smem + G::XSZ;
  double* red = T + G::P2;
  const WorkItem it = items[blockIdx.x];
  const InstDev P = inst[it.inst];
  if (mask && !mask[P.slice_base + it.slice]) return;
  if ((kmin && it.slice < *kmin) || (active && !active[it.inst])) return;
  const int64_t off = P.off_slices + (int64_t)it.slice * N * N;
  const int64_t off_in = (in_iter ? P.off_iter : P.off_slices) + (int64_t)it.slice * N * N;
  Lane<N, NW> L;
  const SineWalk sw = sine_walk<N, NW>(L);
  const Work W = work_vectors(P, it.slice);
  const int vo = threadIdx.x * 8;
  load_sine_table<N, NW>(T, Tg);
  zero_state<N, NW>(smem);
  __syncthreads();
  load_state<N, NW>(X, U_in + off_in);
  __syncthreads();
  double y[G::OWN];
  stage<N, NW>(X, T, sw, L, nullptr);
  stage_regs<N, NW>(X, T, sw, L, y);   // u_hat
#pragma unroll
  for (int s = 0; s < G::OWN; ++s) {
    W.uh.st(s * G::NT, vo, y[s]);
    W.yh.st(s * G::NT, vo, y[s]);
  }
  bool ok = true;
  for (int m = 0; m < P.j_fine; ++m) {
    ok = newton_step<N, NW>(X, red, T, sw, L, P, W, P.dt, W.d_fine, P.nl_variant == 1) && ok;
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) W.uh.st(s * G::NT, vo, W.yh.ld(s * G::NT, vo));
  }
#pragma unroll
  for (int s = 0; s < G::OWN; ++s) y[s] = W.uh.ld(s * G::NT, vo);
  __syncthreads();
  store_owned<N, NW>(X, L, y);
  __syncthreads();
  stage<N, NW>(X, T, sw, L, nullptr);
  stage<N, NW>(X, T, sw, L, nullptr);
  store_state<N, NW>(X, F_out + off);
  if (!ok && threadIdx.x == 0) atomicOr(P.status, 1);
}

// Scheme (2.3) as the coarse step (NPA-II): m_coarse Newton-solved steps of
// tau = dT/m_coarse (the Newton iteration of newton_step with the coarse
// tables).  State in X (state orientation) on entry and exit.
template <int N, int NW>
__device__ void eyre_coarse(double* X, double* red, const double* T, const SineWalk& sw,
                            const Lane<N, NW>& L, const InstDev& P, const Work& W, int& status) {
  using G = Geo<N, NW>;
  const int vo = threadIdx.x * 8;
  const double tau = P.dT / P.m_coarse;
  double y[G::OWN];
  for (int sub = 0; sub < P.m_coarse; ++sub) {
    stage<N, NW>(X, T, sw, L, nullptr);
    stage_regs<N, NW>(X, T, sw, L, y);   // u_hat
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) {
      W.uh.st(s * G::NT, vo, y[s]);
      W.yh.st(s * G::NT, vo, y[s]);
    }
    if (!newton_step<N, NW>(X, red, T, sw, L, P, W, tau, W.d_coarse, false)) status |= 1;
#pragma unroll
    for (int s = 0; s < G::OWN; ++s) y[s] = W.yh.ld(s * G::NT, vo);
    __syncthreads();
    store_owned<N, NW>(X, L, y);
    __syncthreads();
    stage<N, NW>(X, T, sw, L, nullptr);
    stage<N, NW>(X, T, sw, L, nullptr);
  }
}

// One coarse propagation of the state in X (state orientation), result in X.
template <int N, int NW>
__device__ void coarse_apply(double* X, double* red, const double* T, const SineWalk& sw,
                             const Lane<N, NW>& L, const InstDev& P, const Work& W, int& status) {
  if (P.coarse_kind == 1) {  // stabilised step with tau = dT/m
    double v[Geo<N, NW>::OWN];
    const double tau = P.dT / P.m_coarse;
    linear_steps<N, NW>(X, T, sw, L, v, P.m_coarse, tau / (P.h * P.h), P.s_fine, P.f_zero,
                        P.rsig_stab);
  } else if (P.coarse_kind == 3) {
    eyre_coarse<N, NW>(X, red, T, sw, L, P, W, status);
  } else {
    const double tau = P.dT / P.m_coarse;
    approx2_steps<N, NW>(X, red, T, sw, L, P, W, tau, P.m_coarse, W.d_coarse, W.b_coarse,
                         P.f_zero ? -tau : 0.0, P.krylov_rtol, status);
  }
}

// PA-I fine sweep: J steps of scheme (2.4) with tau = dt per work item, one
// workgroup each (variable-coefficient solve by spectral CG every step).
template <int N, int NW>
__global__ void __launch_bounds__(NW * 64)
k_fine_approx2_2d(const WorkItem* __restrict__ items, const InstDev* __restrict__ inst,
                  const double* __restrict__ Tg, const double* __restrict__ U_in,
                  double* __restrict__ F_out, const uint8_t* __restrict__ mask,
                  const int32_t* __restrict__ active, const int32_t* __restrict__ kmin,
                  int in_iter) {
  using G = Geo<N, NW>;
  extern __shared__ double smem[];
  double* X = smem + G::XOFF;
  double* T = smem + G::XSZ;
  double* red = T + G::P2;
  const WorkItem it = items[blockIdx.x];
  const InstDev P = inst[it.inst];
  if (mask && !mask[P.slice_base + it.slice]) return;
  if ((kmin && it.slice < *kmin) || (active && !active[it.inst])) return;
  const int64_t off = P.off_slices + (int64_t)it.slice * N * N;
  const int64_t off_in = (in_iter ? P.off_iter : P.off_slices) + (int64_t)it.slice * N * N;
  Lane<N, NW> L;
  const SineWalk sw = sine_walk<N, NW>(L);
  const Work W = work_vectors(P, it.slice);
  load_sine_table<N, NW>(T, Tg);
  zero_state<N, NW>(smem);
  __syncthreads();
  load_state<N, NW>(X, U_in + off_in);
  __syncthreads();
  int status = 0;
  approx2_steps<N, NW>(X, red, T, sw, L, P, W, P.dt, P.j_fine, W.d_fine, W.imu,
                       P.f_zero ? 0.0 : P.dt, P.krylov_rtol, status);
  __syncthreads();
  store_state<N, NW>(X, F_out + off);
  if (status && threadIdx.x == 0) atomicOr(P.status, status);
}

// mode 0: G on each masked work item independently.
// mode 1: prediction chain per instance: U_{n+1} = G(U_n), G_old_n = U_{n+1}.
// mode 2: correction chain per instance from slice k+1 (U_{k+1} = F_k).
template <int N, int NW>
__global__ void __launch_bounds__(NW * 64)
k_coarse_2d(int mode, const int32_t* __restrict__ insts, const WorkItem* __restrict__ items,
            const InstDev* __restrict__ inst, const double* __restrict__ Tg,
            const double* __restrict__ U_in,
            double* __restrict__ G_out, const uint8_t* __restrict__ mask, double* U,
            const double* __restrict__ F, double* G_old, double* delta, int32_t* status_out,
            const int32_t* __restrict__ active, int k, const int32_t* __restrict__ kdev,
            const int32_t* __restrict__ gate) {
  using G = Geo<N, NW>;
  if (kdev) k = *kdev;
  extern __shared__ double smem[];
  double* X = smem + G::XOFF;   // interior origin
  double* T = smem + G::XSZ;
  double* red = T + G::P2;
  Lane<N, NW> L;
  const SineWalk sw = sine_walk<N, NW>(L);
  int status = 0;
  const int64_t NN = (int64_t)N * N;
  if (mode == 0 || mode >= 3) {
    const WorkItem it = items[blockIdx.x];
    InstDev P = inst[it.inst];
    int64_t off_in = P.off_slices + (int64_t)it.slice * NN;
    if (mode == 0) {
      if (mask && !mask[P.slice_base + it.slice]) return;
      if (P.coarse_kind == 2) return;  // learned propagator: separate path
    } else {
      // the plain propagator (2.4) of gated slices (see launch_coarse_2d)
      if (!gate[mode == 4 ? 0 : it.inst]) return;
      P.coarse_kind = 0;
      if (mode != 5) off_in = P.off_iter + (int64_t)it.slice * NN;
    }
    load_sine_table<N, NW>(T, Tg);
    zero_state<N, NW>(smem);
    __syncthreads();
    const int64_t off = P.off_slices + (int64_t)it.slice * NN;
    load_state<N, NW>(X, U_in + off_in);
    __syncthreads();
    coarse_apply<N, NW>(X, red, T, sw, L, P, work_vectors(P, it.slice), status);
    store_state<N, NW>(X, G_out + off);
    if (status && threadIdx.x == 0) atomicOr(P.status, status);
    return;
  }
  const int ii = insts[blockIdx.x];
  if (active && !active[ii]) return;
  const InstDev P = inst[ii];
  if (P.coarse_kind == 2) return;  // learned propagator: separate path
  const Work W = work_vectors(P, 0);
  load_sine_table<N, NW>(T, Tg);
  zero_state<N, NW>(smem);
  __syncthreads();
  double* Ui = U + P.off_iter;
  const double* Fi = F + P.off_slices;
  double* Gi = G_old + P.off_slices;
  const int Ns = P.n_slices;
  if (mode == 1) {
    load_state<N, NW>(X, Ui);
    __syncthreads();
    for (int n = 0; n < Ns; ++n) {
      coarse_apply<N, NW>(X, red, T, sw, L, P, W, status);
      for (int idx = threadIdx.x; idx < NN; idx += G::NT) {
        const double gv = X[(idx / N) * G::LDX + idx % N];
        Ui[(n + 1) * NN + idx] = gv;
        Gi[n * NN + idx] = gv;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) status_out[ii] = status | *P.status;
    return;
  }
  // mode 2
  if (k >= Ns) {  // every slice already final (finite termination)
    if (threadIdx.x == 0) delta[ii] = 0.0;
    return;
  }
  double dmax = 0.0;
  {
    // U_{k+1} = F_k + (G(U_k) - G_old_k) with G(U_k) == G_old_k exactly.
    double acc[1] = {0.0};
    for (int idx = threadIdx.x; idx < NN; idx += G::NT) {
      const double unew = Fi[k * NN + idx];
      const double dd = unew - Ui[(k + 1) * NN + idx];
      acc[0] += dd * dd;
      Ui[(k + 1) * NN + idx] = unew;
      X[(idx / N) * G::LDX + idx % N] = unew;
    }
    block_sum<NW, 1>(acc, red);
    dmax = acc[0];
    __syncthreads();
  }
  for (int n = k + 1; n < Ns; ++n) {
    coarse_apply<N, NW>(X, red, T, sw, L, P, W, status);
    double acc[1] = {0.0};
    for (int idx = threadIdx.x; idx < NN; idx += G::NT) {
      const int xo = (idx / N) * G::LDX + idx % N;
      const double gv = X[xo];
      const double unew = Fi[n * NN + idx] + (gv - Gi[n * NN + idx]);
      const double dd = unew - Ui[(n + 1) * NN + idx];
      acc[0] += dd * dd;
      Ui[(n + 1) * NN + idx] = unew;
      Gi[n * NN + idx] = gv;
      X[xo] = unew;
    }
    block_sum<NW, 1>(acc, red);
    dmax = fmax(dmax, acc[0]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double dlt = sqrt(P.h * P.h * dmax);
    delta[ii] = dlt;
    if (!(dlt == dlt) || dlt > 1e300) status |= 2;
    status_out[ii] |= status | *P.status;
  }
}

// Per-instance spectral tables in owned order (2D): d = 1/mu + tau eps^2 mu and
// 1/mu + tau for the coarse tau = dT/m; d for the fine tau = dt; 1/mu.
// mu = -(lam_row + lam_col).
template <int N, int NW>
__global__ void __launch_bounds__(NW * 64)
k_cg_tables_2d(const int32_t* __restrict__ insts, const InstDev* __restrict__ inst,
               const double* __restrict__ lam) {
  using G = Geo<N, NW>;
  const InstDev P = inst[insts[blockIdx.x]];
  Lane<N, NW> L;
  const int t = threadIdx.x;
  const double tc = P.dT / P.m_coarse, tf = P.dt;
  const int64_t NN = (int64_t)N * N;
  for (int s = 0; s < G::OWN; ++s) {
    int row, col;
    own_rc<N, NW>(L, s, row, col);
    const double mu = -(lam[row] + lam[col]);
    const int64_t o = (int64_t)s * G::NT + t;
    P.tab[o] = 1.0 / mu + tc * P.eps * P.eps * mu;           // d, coarse tau
    P.tab[NN + o] = 1.0 / mu + tc;                           // b-scale, coarse tau
    P.tab[2 * NN + o] = 1.0 / mu + tf * P.eps * P.eps * mu;  // d, fine tau
    P.tab[3 * NN + o] = 1.0 / mu;                            // 1/mu
  }
}

// ------------------------------------------- cooperative coarse chain
// The coarse sweep is sequential over slices, so one instance's chain runs
// on a group of G workgroups (same XCD: member m of group x is workgroup
// x + 8 m under round-robin dispatch) that split every 2D transform.  A
// "slab stage" multiplies S by an N x B block held in LDS (B = N/G).  A 2D
// transform alternates a left product (column-local: block of columns of X)
// and a right product (row-local: the transposed block of rows), so one
// operator application S diag(q) S ... S needs two transposing exchanges
// through global memory per CG iteration; every CG vector of a group member
// is a block of N x B values held in registers.
// Lane index for the group kernels.  With OPQ it passes through an empty asm,
// so the lane-dependent addresses derived from it (slab positions, exchange
// tiles) are recomputed where they are used instead of being hoisted out of
// the step and CG loops, where dozens of them stay live.  That trades a few
// integer operations for registers: at n = 256 it removes the spills of the
// Newton kernel (6.4 -> 5.0 ms per step), and it lets the pipelined kernel
// hold the coarse sweep in 256 registers; the n = 128 linear kernels, which
// fit either way, are 5-10% faster without it.
template <bool OPQ>
__device__ __forceinline__ int lane_tid() {
  int t = threadIdx.x;
  if constexpr (OPQ) asm volatile("" : "+v"(t));
  return t;
}

template <int N, int G, int NW>
struct GeoC {
  static constexpr int B = N / G, H = N / 2, TR = H / 16, TCB = B / 16;
  static constexpr int WPR = NW / TR, CPW = TCB / WPR, KS = H / 4;
  // slab row stride: B + 8 with B a multiple of 16 puts the four k-rows of an
  // MFMA B operand (rows 2g) on alternating bank halves (conflict-free)
  static constexpr int LDB = B + 8;
  static constexpr int NT = NW * 64, OWN = 8 * CPW, P2 = 2 * (N + 1);
  static_assert(NW % TR == 0 && TCB % WPR == 0 && CPW >= 1, "wave tiling");
  static_assert(OWN * NT == N * B, "ownership");
  static_assert(B % 16 == 0 && N % 8 == 0, "bank-split slab stride, 8 x 8 exchange tiles");
};

// Owned slot s of a slab-stage output: row a' (0..N-1), slab column c (0..B-1).
template <int N, int G, int NW, bool OPQ>
__device__ __forceinline__ void slab_rc(int s, int& row, int& col) {
  using C = GeoC<N, G, NW>;
  const int t = lane_tid<OPQ>(), l = t & 63, w = t >> 6;
  const int g = l >> 4, j = l & 15, tr = w / C::WPR, c0 = (w % C::WPR) * C::CPW;
  const int qr = s >> 1, half = s & 1, q = qr >> 2, r = qr & 3;
  const int a = 16 * tr + g + 4 * r;
  row = half ? (N - 1 - a) : a;
  col = 16 * (c0 + q) + j;
}

// y = S * slab (N x B in LDS), folded; owned results in y.  Software-
// pipelined like the full-width stage: the sine and data operands of k-step
// ks+1 are read from LDS while the MFMAs of k-step ks run.
template <int N, int G, int NW, bool OPQ>
__device__ __forceinline__ void slab_stage(const double* Xs, const double* T,
                                           double (&y)[GeoC<N, G, NW>::OWN]) {
  using C = GeoC<N, G, NW>;
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int g = l >> 4, j = l & 15, tr = w / C::WPR, c0 = (w % C::WPR) * C::CPW;
  d4 aE[C::CPW], aO[C::CPW];
#pragma unroll
  for (int q = 0; q < C::CPW; ++q) {
    aE[q] = d4{0.0, 0.0, 0.0, 0.0};
    aO[q] = d4{0.0, 0.0, 0.0, 0.0};
  }
  const int a1 = 16 * tr + j + 1;
  int ie = (a1 * (2 * g + 1)) % C::P2, io = (a1 * (2 * g + 2)) % C::P2;
  const int step = (8 * a1) % C::P2;
  const double* base = Xs + (2 * g) * C::LDB + 16 * c0 + j;
  double se = T[ie], so = T[io];
  double be[C::CPW], bo[C::CPW];
#pragma unroll
  for (int q = 0; q < C::CPW; ++q) {
    be[q] = base[16 * q];
    bo[q] = base[C::LDB + 16 * q];
  }
#pragma unroll
  for (int ks = 0; ks < C::KS; ++ks) {
    double ne[C::CPW], no[C::CPW], nse = 0.0, nso = 0.0;
    if (ks + 1 < C::KS) {
      ie += step;
      ie -= (ie >= C::P2) ? C::P2 : 0;
      io += step;
      io -= (io >= C::P2) ? C::P2 : 0;
      // at 32 k-steps keep the compiler from precomputing every k-step's
      // table index up front (64 index registers held through the stage
      // spill at n = 256; at 16 k-steps the precomputed indices are faster)
      if constexpr (C::KS > 16) asm volatile("" : "+v"(ie), "+v"(io));
      nse = T[ie];
      nso = T[io];
      const double* pe = base + (8 * (ks + 1)) * C::LDB;
#pragma unroll
      for (int q = 0; q < C::CPW; ++q) {
        ne[q] = pe[16 * q];
        no[q] = pe[C::LDB + 16 * q];
      }
    }
#pragma unroll
    for (int q = 0; q < C::CPW; ++q) {
      aE[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(se, be[q], aE[q], 0, 0, 0);
      aO[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(so, bo[q], aO[q], 0, 0, 0);
    }
    if (ks + 1 < C::KS) {
      se = nse;
      so = nso;
#pragma unroll
      for (int q = 0; q < C::CPW; ++q) {
        be[q] = ne[q];
        bo[q] = no[q];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int q = 0; q < C::CPW; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      y[(q * 4 + r) * 2 + 0] = aE[q][r] + aO[q][r];
      y[(q * 4 + r) * 2 + 1] = aE[q][r] - aO[q][r];
    }
}

template <int N, int G, int NW, bool OPQ>
__device__ __forceinline__ void slab_put(double* Xs, const double (&v)[GeoC<N, G, NW>::OWN]) {
  using C = GeoC<N, G, NW>;
#pragma unroll
  for (int s = 0; s < C::OWN; ++s) {
    int row, col;
    slab_rc<N, G, NW, OPQ>(s, row, col);
    Xs[row * C::LDB + col] = v[s];
  }
}

// State of one group member: barrier counter, exchange buffers, partial
// sums.  Consecutive exchanges (and consecutive reductions) alternate between
// two buffers, so a buffer is rewritten only after a later barrier has shown
// that every member finished reading it; one barrier per exchange suffices.
struct CoopCtx {
  int32_t* cnt;     // arrivals, monotonic over the launch (zeroed before it)
  double* xg;       // two exchange matrices N x N (natural order)
  double* part;     // two slots of 4 x 16 partial sums (value i of member m at i * 16 + m)
  int mem, ok, xsel, psel, nb;
  uint64_t limit;   // wall-clock ticks a barrier waits before it gives up
};

// Barrier of the G members of one group: barrier b is passed once the
// counter reaches G (b + 1).  Each wave first waits until its own stores are
// acknowledged (s_waitcnt vmcnt(0)).  Then one thread arrives, polls and
// leaves; the spin is bounded by the wall clock (cc.limit, 0.2 s by default): on time-out
// the member clears cc.ok and every later barrier of the launch returns at
// once, so a lost member can never hang the kernel; the host sees the failure
// in the status word.
// Ordering of the exchanged data: every value that crosses members (exchange
// matrices, partial sums) is written and read with agent-scope atomics
// (xg_store, xg_load), which go to the device coherence point (write-through
// stores, loads that bypass L1/L2).  A store's vmcnt acknowledgement comes
// from that point, so after the waits every member's data is there before its
// counter increment is issued, and loads issued after the counter was seen
// return it.  No cache maintenance is needed: this is the acknowledgement the
// compiler's agent-scope release sequence relies on, without the L2
// write-back and invalidate that only non-atomic data needs (those stall the
// other groups sharing an XCD's L2: measured 18% per fine step).
template <int G>
__device__ __forceinline__ void group_barrier(CoopCtx& cc) {
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0) (gfx9 encoding; lgkm/exp not waited)
  __syncthreads();
  __shared__ int ok_s;
  if (threadIdx.x == 0) {
    int ok = cc.ok;
    if (ok) {
      const int target = G * (cc.nb + 1);
      const int arrived =
          __hip_atomic_fetch_add(cc.cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (arrived != target - 1) {
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(cc.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
          if (wall_clock64() - t0 > cc.limit) { ok = 0; break; }
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
    ok_s = ok;
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);   // no compiler motion across the poll
  __syncthreads();
  cc.ok = ok_s;
  cc.nb += 1;
}

// Store and load of data that crosses group members (see group_barrier).
__device__ __forceinline__ void xg_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double xg_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Group-wide sum of K values in a fixed order (partials exchanged in memory,
// summed by every member in member order, so all members agree bitwise).
template <int NW, int G, int K>
__device__ __forceinline__ void group_sum(double (&v)[K], double* red, CoopCtx& cc) {
  static_assert(K <= 4 && G <= 16, "partial slots");
  block_sum<NW, K>(v, red);
  double* part = cc.part + 64 * cc.psel;
  cc.psel ^= 1;
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < K; ++i) xg_store(&part[i * 16 + cc.mem], v[i]);
  group_barrier<G>(cc);
  double pv[K][G];
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int m = 0; m < G; ++m) pv[i][m] = xg_load(&part[i * 16 + m]);
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < G; ++m) s += pv[i][m];
    v[i] = s;
  }
}
// Exchange A: from a column block (left-product output v: rows 0..N-1, block
// columns C_m) to the transposed row block slab[k][r'] = M[R_m[r']][k].
template <int N, int G, int NW, bool OPQ>
__device__ void xchg_cols_to_rowsT(const double (&v)[GeoC<N, G, NW>::OWN], double* Xs,
                                   CoopCtx& cc) {
  using C = GeoC<N, G, NW>;
  double* xg = cc.xg + (int64_t)N * N * cc.xsel;
  cc.xsel ^= 1;
#pragma unroll
  for (int s = 0; s < C::OWN; ++s) {
    int row, col;
    slab_rc<N, G, NW, OPQ>(s, row, col);
    xg_store(&xg[(int64_t)row * N + cc.mem * C::B + col], v[s]);
  }
  group_barrier<G>(cc);
  // 8 x 8 tiles (8 consecutive k per row, 8 rows per wave instruction): 64-byte
  // global segments and bank-conflict-free transposed LDS writes
  constexpr int R = C::B * N / C::NT;
  const int l = lane_tid<OPQ>() & 63, w = lane_tid<OPQ>() >> 6;
  double t[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int tile = w + NW * j, rr = 8 * (tile % (C::B / 8)) + (l >> 3);
    const int k = 8 * (tile / (C::B / 8)) + (l & 7);
    t[j] = xg_load(&xg[(int64_t)(cc.mem * C::B + rr) * N + k]);
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int tile = w + NW * j, rr = 8 * (tile % (C::B / 8)) + (l >> 3);
    const int k = 8 * (tile / (C::B / 8)) + (l & 7);
    Xs[k * C::LDB + rr] = t[j];
  }
  __syncthreads();
}

// Exchange B: from a right-product output v (slab form: element (a, c) is
// M[R_m[c]][a]) to the column block slab[k][c] = M[k][C_m[c]].  The exchange
// matrix holds M transposed (X[a][R_m[c]] = M[R_m[c]][a]): the writer stores
// contiguous 128-byte runs straight from registers and the reader takes 8 x 8
// tiles, as in exchange A (measured 5-12% faster per fine step than a
// transpose through LDS before the stores).  With K > 0 a
// group reduction of acc[0..K) rides on the same barrier (per-member values
// posted before it, combined in member order after it): sums, or with MINMAX
// (K = 2) the minimum of acc[0] and the maximum of acc[1].
template <int N, int G, int NW, bool OPQ, int K, bool MINMAX = false>
__device__ void xchg_rowsT_to_cols(const double (&v)[GeoC<N, G, NW>::OWN], double* Xs,
                                   CoopCtx& cc, double* acc, double* red) {
  using C = GeoC<N, G, NW>;
  double* xg = cc.xg + (int64_t)N * N * cc.xsel;
  cc.xsel ^= 1;
  constexpr int R = C::B * N / C::NT;
  const int l = lane_tid<OPQ>() & 63, w = lane_tid<OPQ>() >> 6;
#pragma unroll
  for (int s = 0; s < C::OWN; ++s) {
    int row, col;
    slab_rc<N, G, NW, OPQ>(s, row, col);
    xg_store(&xg[(int64_t)row * N + cc.mem * C::B + col], v[s]);
  }
  double* part = cc.part + 64 * cc.psel;
  if constexpr (K > 0) {
    double v2[K];
#pragma unroll
    for (int i = 0; i < K; ++i) v2[i] = acc[i];
    if constexpr (MINMAX)
      block_minmax<NW>(v2[0], v2[1], red);
    else
      block_sum<NW, K>(v2, red);
    cc.psel ^= 1;
    if (threadIdx.x == 0)
#pragma unroll
      for (int i = 0; i < K; ++i) xg_store(&part[i * 16 + cc.mem], v2[i]);
  }
  group_barrier<G>(cc);
  double t[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int tile = w + NW * j, c = 8 * (tile % (C::B / 8)) + (l >> 3);
    const int k = 8 * (tile / (C::B / 8)) + (l & 7);
    t[j] = xg_load(&xg[(int64_t)(cc.mem * C::B + c) * N + k]);
  }
  if constexpr (K > 0) {
    // lane i G + m of every wave loads member m's value i; the wave then
    // combines them by shuffles in member order
    static_assert(K * G <= 64 && K <= 4 && G <= 16, "one value per lane, partial slots");
    const double pl = l < K * G ? xg_load(&part[(l / G) * 16 + l % G]) : 0.0;
    if constexpr (MINMAX) {
      double a = 1e300, b = -1e300;
#pragma unroll
      for (int m = 0; m < G; ++m) {
        a = fmin(a, __shfl(pl, m));
        b = fmax(b, __shfl(pl, G + m));
      }
      acc[0] = a;
      acc[1] = b;
    } else {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < G; ++m) s += __shfl(pl, i * G + m);
        acc[i] = s;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int tile = w + NW * j, c = 8 * (tile % (C::B / 8)) + (l >> 3);
    const int k = 8 * (tile / (C::B / 8)) + (l & 7);
    Xs[k * C::LDB + c] = t[j];
  }
  __syncthreads();
}

// y = S (q . S v S) S, the coupling part of K v = d v + tau S (q . S v S) S
// (the SPD form of (2.4)), for v a column block in registers (two transposing
// exchanges; v is not needed after the first stage).  acc[0], acc[2] hold this
// thread's terms of two inner products on entry; acc[1] gets those of
// (K v, v) = sum d v^2 + tau sum q (S v S)^2 (S is orthogonal and symmetric),
// and all three come back as group sums, reduced on the second exchange's
// barrier.
template <int N, int G, int NW, bool OPQ>
__device__ __forceinline__ void coop_apply_K(double* Xs, const double* T, CoopCtx& cc,
                                             const double (&v)[GeoC<N, G, NW>::OWN],
                                             double (&y)[GeoC<N, G, NW>::OWN],
                                             const double* Dl, const double* Ql, double tau,
                                             double (&acc)[3], double* red) {
  using C = GeoC<N, G, NW>;
  const int t = threadIdx.x;
  double dvv = 0.0, qyy = 0.0;
#pragma unroll
  for (int s = 0; s < C::OWN; ++s) dvv += Dl[s * C::NT + t] * v[s] * v[s];
  __syncthreads();
  slab_put<N, G, NW, OPQ>(Xs, v);
  __syncthreads();
  slab_stage<N, G, NW, OPQ>(Xs, T, y);          // left: S v (column block)
  xchg_cols_to_rowsT<N, G, NW, OPQ>(y, Xs, cc);
  slab_stage<N, G, NW, OPQ>(Xs, T, y);          // right: (S v S) row block
#pragma unroll
  for (int s = 0; s < C::OWN; ++s) {
    const double q = Ql[s * C::NT + t];
    qyy += q * y[s] * y[s];
    y[s] *= q;
  }
  acc[1] = dvv + tau * qyy;
  __syncthreads();
  slab_put<N, G, NW, OPQ>(Xs, y);
  __syncthreads();
  slab_stage<N, G, NW, OPQ>(Xs, T, y);          // right: (q . S v S) S
  xchg_rowsT_to_cols<N, G, NW, OPQ, 3>(y, Xs, cc, acc, red);
  slab_stage<N, G, NW, OPQ>(Xs, T, y);          // left: column block
}

// Preconditioned CG for K x = b, K = diag(d) + tau S diag(q) S (the SPD form
// shared by (2.4) and the Newton matrices of the implicit steps), on the
// group: column blocks in registers, d, the preconditioner 1 / (d + tau c)
// and q in LDS at [s * NT + thread] (q in the row-block layout of S v S).
// Chronopoulos-Gear form: one operator application and one group reduction
// of three inner products per iteration (in exact arithmetic the iterates of
// plain PCG), from x = 0, stopped when ||r|| <= rtol ||b||.  On entry rv = b;
// on exit xv = x (rv and y are overwritten).  Returns false if maxit was
// reached or the residual is not finite.
template <int N, int G, int NW, bool OPQ>
__device__ bool coop_cg(double* Xs, const double* T, double* red, CoopCtx& cc, const double* Dl,
                        const double* Ml, const double* Ql, double tau, double rtol, int maxit,
                        double (&rv)[GeoC<N, G, NW>::OWN], double (&xv)[GeoC<N, G, NW>::OWN],
                        double (&y)[GeoC<N, G, NW>::OWN], int& applies) {
  using C = GeoC<N, G, NW>;
  const int t = threadIdx.x;
  double pv[C::OWN], sv[C::OWN];
#pragma unroll
  for (int s = 0; s < C::OWN; ++s) {
    xv[s] = 0.0;
    pv[s] = rv[s] * Ml[s * C::NT + t];   // z_0 = M r_0
  }
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < C::OWN; ++s) {
    acc[0] += rv[s] * pv[s];
    acc[2] += rv[s] * rv[s];
  }
  coop_apply_K<N, G, NW, OPQ>(Xs, T, cc, pv, sv, Dl, Ql, tau, acc, red);
  ++applies;
#pragma unroll
  for (int s = 0; s < C::OWN; ++s) sv[s] = Dl[s * C::NT + t] * pv[s] + tau * sv[s];   // w_0 = K z_0
  double gam = acc[0];
  const double stop2 = rtol * rtol * acc[2];
  bool done = !(acc[2] > 0.0);
  double alpha = gam / acc[1];
  for (int it = 1; !done && it <= maxit; ++it) {
#pragma unroll
    for (int s = 0; s < C::OWN; ++s) {
      xv[s] += alpha * pv[s];
      rv[s] -= alpha * sv[s];
    }
    double z[C::OWN];
    double a3[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < C::OWN; ++s) {
      z[s] = rv[s] * Ml[s * C::NT + t];
      a3[0] += rv[s] * z[s];
      a3[2] += rv[s] * rv[s];
    }
    coop_apply_K<N, G, NW, OPQ>(Xs, T, cc, z, y, Dl, Ql, tau, a3, red);
    ++applies;
    if (a3[2] <= stop2) { done = true; break; }
    // a3 is the same in every member; cc.ok drops only on a barrier time-out
    if (!(a3[2] == a3[2]) || !cc.ok) break;
    const double beta = a3[0] / gam;
    alpha = a3[0] / (a3[1] - beta * a3[0] / alpha);
    gam = a3[0];
#pragma unroll
    for (int s = 0; s < C::OWN; ++s) {
      const double zs = rv[s] * Ml[s * C::NT + t];
      const double ws = Dl[s * C::NT + t] * zs + tau * y[s];   // w = K z
      pv[s] = zs + beta * pv[s];
      sv[s] = ws + beta * sv[s];
    }
  }
  return done;
}

// One solve of scheme (2.4) by the group.  On entry u holds the member's row
// block of the state in slab form (element (a, c) = u[R_m[c]][a]); on exit it
// holds the result in the same form.  Per-point tables live in LDS at
// [s * NT + thread]: Dl = d of (2.4), Ml = the preconditioner, Ql = q = u^2.
// The linear solve is coop_cg, stopped when ||r|| <= rtol ||b|| as in the
// one-workgroup solver.
template <int N, int G, int NW, bool OPQ>
__device__ void coop_approx2(double* Xs, double (&u)[GeoC<N, G, NW>::OWN], const double* T,
                             double* red, CoopCtx& cc, const InstDev& P, const double* Dl,
                             double* Ml, double* Ql, const double* lamS, int& status) {
  using C = GeoC<N, G, NW>;
  const double tau = P.dT / P.m_coarse;
  const int t = threadIdx.x;
  double y[C::OWN], rv[C::OWN], xv[C::OWN];
  for (int sub = 0; sub < P.m_coarse; ++sub) {
    double mn = 1e300, mx = -1e300;
#pragma unroll
    for (int s = 0; s < C::OWN; ++s) {
      const double q = P.f_zero ? 0.0 : u[s] * u[s];
      Ql[s * C::NT + t] = q;
      mn = fmin(mn, q);
      mx = fmax(mx, q);
    }
    // u_hat = S u S: right product on the row block, exchange, left product;
    // the range of q rides on the exchange
    __syncthreads();
    slab_put<N, G, NW, OPQ>(Xs, u);
    __syncthreads();
    slab_stage<N, G, NW, OPQ>(Xs, T, y);
    {
      double mm[2] = {mn, mx};
      xchg_rowsT_to_cols<N, G, NW, OPQ, 2, true>(y, Xs, cc, mm, red);
      mn = mm[0];
      mx = mm[1];
    }
    const double cshift = 0.5 * (mn + mx);
    slab_stage<N, G, NW, OPQ>(Xs, T, y);   // column block of u_hat
#pragma unroll
    for (int s = 0; s < C::OWN; ++s) {
      int row, col;
      slab_rc<N, G, NW, OPQ>(s, row, col);
      const double mu = -(lamS[row] + lamS[cc.mem * C::B + col]);
      const double bs = P.f_zero ? 1.0 / mu : 1.0 / mu + tau;
      Ml[s * C::NT + t] = 1.0 / (Dl[s * C::NT + t] + tau * cshift);
      rv[s] = bs * y[s];
    }
    int applies = 0;
    if (!coop_cg<N, G, NW, OPQ>(Xs, T, red, cc, Dl, Ml, Ql, tau, P.krylov_rtol, P.krylov_max, rv,
                           xv, y, applies))
      status |= 1;
    // v = S x S: left product, exchange, right product -> row block
    __syncthreads();
    slab_put<N, G, NW, OPQ>(Xs, xv);
    __syncthreads();
    slab_stage<N, G, NW, OPQ>(Xs, T, y);
    xchg_cols_to_rowsT<N, G, NW, OPQ>(y, Xs, cc);
    slab_stage<N, G, NW, OPQ>(Xs, T, u);
  }
}

// Fine sweep of the linear step (2.5) on groups of G workgroups (same XCD
// mapping and barriers as the coarse sweep).  Since the 5-point Laplacian is
// diagonal in the sine basis (eigenvalues lam_p + lam_q), one step
//   (I + dt eps^2 Lap^2 - s dt Lap) v = u + dt Lap g,   g = f(u) - s u,
// is, with hats for S . S,  v_hat = (u_hat + dt lam g_hat) / sigma:  one
// forward transform of g and one inverse transform per step.  u_hat stays in
// registers (column block); u in slab form (row block) for the pointwise g.
//
// One work item on the group: J steps from the state at src to dst (both
// N x N, row-major).  With COHERENT the state is read and written with the
// agent-scope accesses of the exchanges, for producers and consumers in
// other workgroups of the same launch.  Rs: LDS for 1 / sigma.
template <int N, int G, int NW, bool OPQ, bool COHERENT>
__device__ __forceinline__ void fine_group_item(const InstDev& P, double* Xs, const double* T,
                                                const double* lamS, double* Rs, CoopCtx& cc,
                                                const double* src, double* dst, int j_steps) {
  using C = GeoC<N, G, NW>;
  const int t = threadIdx.x, mem = cc.mem;
  // slab-form element (a, c) is u[R_m[c]][a]
  auto gidx = [&](int s) {
    int row, col;
    slab_rc<N, G, NW, OPQ>(s, row, col);
    return (int64_t)(mem * C::B + col) * N + row;
  };
  double u[C::OWN], uh[C::OWN], y[C::OWN];
  __syncthreads();   // every wave is done with the slab and Rs of the previous item
#pragma unroll
  for (int s = 0; s < C::OWN; ++s) {
    int row, col;
    slab_rc<N, G, NW, OPQ>(s, row, col);
    Rs[s * C::NT + t] = P.rsig_fine[(int64_t)row * N + mem * C::B + col];   // column block
    u[s] = COHERENT ? xg_load(&src[gidx(s)]) : src[gidx(s)];
  }
  // u_hat = S u S (right product on the row block, exchange, left product)
  slab_put<N, G, NW, OPQ>(Xs, u);
  __syncthreads();
  slab_stage<N, G, NW, OPQ>(Xs, T, y);
  xchg_rowsT_to_cols<N, G, NW, OPQ, 0>(y, Xs, cc, nullptr, nullptr);
  slab_stage<N, G, NW, OPQ>(Xs, T, uh);
  const int J = j_steps > 0 ? j_steps : P.j_fine;
  const double s1 = 1.0 + P.s_fine;
  for (int m = 0; m < J; ++m) {
#pragma unroll
    for (int s = 0; s < C::OWN; ++s)
      y[s] = P.f_zero ? (-P.s_fine * u[s]) : (u[s] * u[s] * u[s] - s1 * u[s]);
    __syncthreads();
    slab_put<N, G, NW, OPQ>(Xs, y);
    __syncthreads();
    slab_stage<N, G, NW, OPQ>(Xs, T, y);
    xchg_rowsT_to_cols<N, G, NW, OPQ, 0>(y, Xs, cc, nullptr, nullptr);
    slab_stage<N, G, NW, OPQ>(Xs, T, y);   // g_hat, column block
#pragma unroll
    for (int s = 0; s < C::OWN; ++s) {
      int row, col;
      slab_rc<N, G, NW, OPQ>(s, row, col);
      const double tl = P.dt * (lamS[row] + lamS[mem * C::B + col]);
      uh[s] = Rs[s * C::NT + t] * (uh[s] + tl * y[s]);
    }
    __syncthreads();
    slab_put<N, G, NW, OPQ>(Xs, uh);
    __syncthreads();
    slab_stage<N, G, NW, OPQ>(Xs, T, y);
    xchg_cols_to_rowsT<N, G, NW, OPQ>(y, Xs, cc);
    slab_stage<N, G, NW, OPQ>(Xs, T, u);   // new state, row block
  }
#pragma unroll
  for (int s = 0; s < C::OWN; ++s) {
    if (COHERENT) xg_store(&dst[gidx(s)], u[s]);
    else dst[gidx(s)] = u[s];
  }
}

// The fine sweep: persistent, the grid holds as many groups as can be
// resident at once and group q takes work items q, q + groups, ...  On a
// barrier time-out the instance's status word gets bit 4.
template <int N, int G, int NW, bool OPQ>
__global__ void __launch_bounds__(NW * 64)
k_fine_group(const WorkItem* __restrict__ items, int n_items, const InstDev* __restrict__ inst,
             const double* __restrict__ Tg, const double* __restrict__ lam,
             const double* __restrict__ U_in, double* __restrict__ F_out,
             const uint8_t* __restrict__ mask, const int32_t* __restrict__ active,
             const int32_t* __restrict__ kmin, int in_iter, int j_steps, int32_t* sync) {
  using C = GeoC<N, G, NW>;
  extern __shared__ double smem[];
  double* Xs = smem;
  double* T = smem + N * C::LDB;
  double* lamS = T + C::P2;
  double* Rs = lamS + N;             // 1 / sigma of the current item [s * NT + thread]
  const int xcd = blockIdx.x % 8, rest = blockIdx.x / 8;
  const int mem = rest % G, grp = rest / G;
  const int idx = grp * 8 + xcd;                  // group index
  const int n_groups = gridDim.x / G;
  const int64_t NN = (int64_t)N * N;
  const int t = threadIdx.x;
  for (int m = t; m < C::P2; m += C::NT) T[m] = Tg[m];
  for (int m = t; m < N; m += C::NT) lamS[m] = lam[m];
  __syncthreads();
  CoopCtx cc;
  cc.cnt = sync + idx * 64;
  cc.mem = mem;
  cc.ok = 1;
  cc.xsel = 0;
  cc.psel = 0;
  cc.nb = 0;
  cc.limit = inst[0].wait_ticks;   // the same for every instance of a context
  for (int item = idx; item < n_items; item += n_groups) {
    const WorkItem it = items[item];
    const InstDev P = inst[it.inst];
    if (mask && !mask[P.slice_base + it.slice]) continue;
    if ((kmin && it.slice < *kmin) || (active && !active[it.inst])) continue;
    cc.xg = P.work + (int64_t)it.slice * P.work_vecs * NN;   // the item's work vectors
    cc.part = cc.xg + 2 * NN;
    const int64_t off = P.off_slices + (int64_t)it.slice * NN;
    const int64_t off_in = (in_iter ? P.off_iter : P.off_slices) + (int64_t)it.slice * NN;
    fine_group_item<N, G, NW, OPQ, false>(P, Xs, T, lamS, Rs, cc, U_in + off_in, F_out + off,
                                     j_steps);
    if (!cc.ok && t == 0 && mem == 0) atomicOr(P.status, 4);
  }
}

// Implicit fine sweep on groups of G workgroups, persistent over the work
// items as k_fine_group.  Each step solves scheme (2.3) (nl_variant 0) or
// backward Euler (1) by Newton's method from Y_0 = u, exactly as the
// one-workgroup kernel: in sine coordinates, with A = -Lap and mu its
// eigenvalues, A^{-1} H(Y) = d Yh + tau S(Y^3)S - (1/mu + tau) uh (2.3), or
// d Yh + tau S(Y^3)S - tau Yh - uh/mu (BE), d = 1/mu + tau eps^2 mu; the
// Newton matrix d + tau S diag(q) S, q = 3Y^2 (2.3) or 3Y^2 - 1 (BE), is solved
// by coop_cg; stop when ||Y_{m+1} - Y_m||_h <= newton_tol.  Yh and uh live in
// registers (column block), Y in slab form (row block).  A Newton or CG cap
// sets status bit 1, a barrier time-out bit 4.
template <int N, int G, int NW, bool OPQ>
__global__ void __launch_bounds__(NW * 64)
k_fine_newton_group(const WorkItem* __restrict__ items, int n_items,
                    const InstDev* __restrict__ inst, const double* __restrict__ Tg,
                    const double* __restrict__ lam, const double* __restrict__ U_in,
                    double* __restrict__ F_out, const uint8_t* __restrict__ mask,
                    const int32_t* __restrict__ active, const int32_t* __restrict__ kmin,
                    int in_iter, int32_t* sync) {
  using C = GeoC<N, G, NW>;
  extern __shared__ double smem[];
  double* Xs = smem;
  double* T = smem + N * C::LDB;
  double* lamS = T + C::P2;
  double* red = lamS + N;
  double* Dl = red + 4 * NW;
  double* Ml = Dl + C::OWN * C::NT;
  double* Ql = Ml + C::OWN * C::NT;
  const int xcd = blockIdx.x % 8, rest = blockIdx.x / 8;
  const int mem = rest % G, grp = rest / G;
  const int idx = grp * 8 + xcd;
  const int n_groups = gridDim.x / G;
  const int64_t NN = (int64_t)N * N;
  const int t = threadIdx.x;
  for (int m = t; m < C::P2; m += C::NT) T[m] = Tg[m];
  for (int m = t; m < N; m += C::NT) lamS[m] = lam[m];
  __syncthreads();
  CoopCtx cc;
  cc.cnt = sync + idx * 64;
  cc.mem = mem;
  cc.ok = 1;
  cc.xsel = 0;
  cc.psel = 0;
  cc.nb = 0;
  cc.limit = inst[0].wait_ticks;   // the same for every instance of a context
  auto gidx = [&](int s) {
    int row, col;
    slab_rc<N, G, NW, OPQ>(s, row, col);
    return (int64_t)(mem * C::B + col) * N + row;
  };
  for (int item = idx; item < n_items; item += n_groups) {
    const WorkItem it = items[item];
    const InstDev P = inst[it.inst];
    if (mask && !mask[P.slice_base + it.slice]) continue;
    if ((kmin && it.slice < *kmin) || (active && !active[it.inst])) continue;
    cc.xg = P.work + (int64_t)it.slice * P.work_vecs * NN;
    cc.part = cc.xg + 2 * NN;
    const int64_t off = P.off_slices + (int64_t)it.slice * NN;
    const int64_t off_in = (in_iter ? P.off_iter : P.off_slices) + (int64_t)it.slice * NN;
    const double tau = P.dt;
    const bool be = P.nl_variant == 1;
    const double a3q = P.f_zero ? 0.0 : 3.0, a0q = (be && !P.f_zero) ? -1.0 : 0.0;
    double uh[C::OWN], yh[C::OWN], y[C::OWN], rv[C::OWN], xv[C::OWN];
    __syncthreads();   // every wave is done with the LDS tables of the previous item
#pragma unroll
    for (int s = 0; s < C::OWN; ++s) {
      int row, col;
      slab_rc<N, G, NW, OPQ>(s, row, col);
      const double mu = -(lamS[row] + lamS[mem * C::B + col]);
      Dl[s * C::NT + t] = 1.0 / mu + tau * P.eps * P.eps * mu;
      y[s] = U_in[off_in + gidx(s)];
    }
    // u_hat = S u S
    slab_put<N, G, NW, OPQ>(Xs, y);
    __syncthreads();
    slab_stage<N, G, NW, OPQ>(Xs, T, rv);
    xchg_rowsT_to_cols<N, G, NW, OPQ, 0>(rv, Xs, cc, nullptr, nullptr);
    slab_stage<N, G, NW, OPQ>(Xs, T, uh);
#pragma unroll
    for (int s = 0; s < C::OWN; ++s) yh[s] = uh[s];
    bool ok = true;
    int newton_its = 0, applies = 0;
    for (int m = 0; m < P.j_fine; ++m) {
      bool conv = false;
      for (int nit = 0; nit < P.newton_max && !conv; ++nit) {
        // Y = S Yh S (row block)
        __syncthreads();
        slab_put<N, G, NW, OPQ>(Xs, yh);
        __syncthreads();
        slab_stage<N, G, NW, OPQ>(Xs, T, y);
        xchg_cols_to_rowsT<N, G, NW, OPQ>(y, Xs, cc);
        slab_stage<N, G, NW, OPQ>(Xs, T, y);
        // q and Y^3; S (Y^3) S with the range of q on the exchange
        double mn = 1e300, mx = -1e300;
#pragma unroll
        for (int s = 0; s < C::OWN; ++s) {
          const double q = a3q * y[s] * y[s] + a0q;
          Ql[s * C::NT + t] = q;
          mn = fmin(mn, q);
          mx = fmax(mx, q);
          y[s] = P.f_zero ? 0.0 : y[s] * y[s] * y[s];
        }
        __syncthreads();
        slab_put<N, G, NW, OPQ>(Xs, y);
        __syncthreads();
        slab_stage<N, G, NW, OPQ>(Xs, T, y);
        double mm[2] = {mn, mx};
        xchg_rowsT_to_cols<N, G, NW, OPQ, 2, true>(y, Xs, cc, mm, red);
        slab_stage<N, G, NW, OPQ>(Xs, T, y);   // S (Y^3) S, column block
        const double cshift = 0.5 * (mm[0] + mm[1]);
#pragma unroll
        for (int s = 0; s < C::OWN; ++s) {
          int row, col;
          slab_rc<N, G, NW, OPQ>(s, row, col);
          const double im = -1.0 / (lamS[row] + lamS[mem * C::B + col]);   // 1 / mu
          const double d = Dl[s * C::NT + t];
          double g;
          if (P.f_zero) g = d * yh[s] - im * uh[s];
          else if (be) g = d * yh[s] + tau * y[s] - tau * yh[s] - im * uh[s];
          else g = d * yh[s] + tau * y[s] - (im + tau) * uh[s];
          rv[s] = -g;
          Ml[s * C::NT + t] = 1.0 / (d + tau * cshift);
        }
        ++newton_its;
        if (!coop_cg<N, G, NW, OPQ>(Xs, T, red, cc, Dl, Ml, Ql, tau, P.nl_krylov_rtol, P.krylov_max,
                               rv, xv, y, applies))
          ok = false;
        double a[1] = {0.0};
#pragma unroll
        for (int s = 0; s < C::OWN; ++s) {
          yh[s] += xv[s];
          a[0] += xv[s] * xv[s];
        }
        group_sum<NW, G, 1>(a, red, cc);
        const double step = sqrt(P.h * P.h * a[0]);   // ||S dYh S||_h = h ||dYh||_F
        if (step <= P.newton_tol) conv = true;
        else if (!(step == step) || !cc.ok) break;
      }
      if (!conv) ok = false;
#pragma unroll
      for (int s = 0; s < C::OWN; ++s) uh[s] = yh[s];
    }
    // u = S uh S (row block)
    __syncthreads();
    slab_put<N, G, NW, OPQ>(Xs, uh);
    __syncthreads();
    slab_stage<N, G, NW, OPQ>(Xs, T, y);
    xchg_cols_to_rowsT<N, G, NW, OPQ>(y, Xs, cc);
    slab_stage<N, G, NW, OPQ>(Xs, T, y);
#pragma unroll
    for (int s = 0; s < C::OWN; ++s) F_out[off + gidx(s)] = y[s];
    if (t == 0 && mem == 0) {
      // the item's Newton iterations and Krylov operator applications
      P.iters[2 * it.slice] = newton_its;
      P.iters[2 * it.slice + 1] = applies;
      if (!ok || !cc.ok) atomicOr(P.status, (ok ? 0 : 1) | (cc.ok ? 0 : 4));
    }
  }
}

// Cooperative chain (modes 1 and 2 of k_coarse_2d) for scheme (2.4), n = N.
template <int N, int G, int NW, bool OPQ>
__global__ void __launch_bounds__(NW * 64)
k_chain_coop(int mode, const int32_t* __restrict__ insts, int n_insts,
             const InstDev* __restrict__ inst, const double* __restrict__ Tg,
             const double* __restrict__ lam, double* U, const double* __restrict__ F,
             double* G_old, double* delta, int32_t* status_out, const int32_t* __restrict__ active,
             int k, const int32_t* __restrict__ kdev, int32_t* sync) {
  using C = GeoC<N, G, NW>;
  extern __shared__ double smem[];
  double* Xs = smem;
  double* T = smem + N * C::LDB;
  double* lamS = T + C::P2;
  double* red = lamS + N;
  double* Dl = red + 4 * NW;
  double* Ml = Dl + C::OWN * C::NT;
  double* Ql = Ml + C::OWN * C::NT;
  if (kdev) k = *kdev;
  const int xcd = blockIdx.x % 8, rest = blockIdx.x / 8;
  const int mem = rest % G, grp = rest / G;
  const int idx = grp * 8 + xcd;
  if (idx >= n_insts) return;
  const int ii = insts[idx];
  if (active && !active[ii]) return;
  const InstDev P = inst[ii];
  if (P.coarse_kind != 0) return;
  CoopCtx cc;
  cc.cnt = sync + idx * 64;
  cc.xg = P.work;                      // slice-0 work vectors of the instance
  cc.part = P.work + 2 * (int64_t)N * N;
  cc.mem = mem;
  cc.ok = 1;
  cc.xsel = 0;
  cc.psel = 0;
  cc.nb = 0;
  cc.limit = P.wait_ticks;
  for (int m = threadIdx.x; m < C::P2; m += C::NT) T[m] = Tg[m];
  for (int m = threadIdx.x; m < N; m += C::NT) lamS[m] = lam[m];
  // d of (2.4) on the member's column block (owned slots)
  const double tau = P.dT / P.m_coarse;
  double u[C::OWN];
#pragma unroll
  for (int s = 0; s < C::OWN; ++s) {
    int row, col;
    slab_rc<N, G, NW, OPQ>(s, row, col);
    const double mu = -(lam[row] + lam[mem * C::B + col]);
    Dl[s * C::NT + threadIdx.x] = 1.0 / mu + tau * P.eps * P.eps * mu;
  }
  __syncthreads();
  const int64_t NN = (int64_t)N * N;
  double* Ui = U + P.off_iter;
  const double* Fi = F + P.off_slices;
  double* Gi = G_old + P.off_slices;
  const int Ns = P.n_slices;
  int status = 0;
  // state element (a, c) of the slab form is u[R_m[c]][a] = row mem*B + c, column a
  auto gidx = [&](int s) {
    int row, col;
    slab_rc<N, G, NW, OPQ>(s, row, col);
    return (int64_t)(mem * C::B + col) * N + row;
  };
  if (mode == 1) {
#pragma unroll
    for (int s = 0; s < C::OWN; ++s) u[s] = Ui[gidx(s)];
    for (int n = 0; n < Ns; ++n) {
      coop_approx2<N, G, NW, OPQ>(Xs, u, T, red, cc, P, Dl, Ml, Ql, lamS, status);
#pragma unroll
      for (int s = 0; s < C::OWN; ++s) {
        Ui[(n + 1) * NN + gidx(s)] = u[s];
        Gi[n * NN + gidx(s)] = u[s];
      }
    }
    if (threadIdx.x == 0 && mem == 0) status_out[ii] = status | *P.status | (cc.ok ? 0 : 4);
    return;
  }
  if (k >= Ns) {
    if (threadIdx.x == 0 && mem == 0) delta[ii] = 0.0;
    return;
  }
  double dmax;
  {
    double acc[1] = {0.0};
#pragma unroll
    for (int s = 0; s < C::OWN; ++s) {
      const int64_t o = gidx(s);
      const double un = Fi[k * NN + o];
      const double d = un - Ui[(k + 1) * NN + o];
      acc[0] += d * d;
      Ui[(k + 1) * NN + o] = un;
      u[s] = un;
    }
    group_sum<NW, G, 1>(acc, red, cc);
    dmax = acc[0];
  }
  for (int n = k + 1; n < Ns; ++n) {
    coop_approx2<N, G, NW, OPQ>(Xs, u, T, red, cc, P, Dl, Ml, Ql, lamS, status);
    double acc[1] = {0.0};
#pragma unroll
    for (int s = 0; s < C::OWN; ++s) {
      const int64_t o = gidx(s);
      const double gv = u[s];
      const double un = Fi[n * NN + o] + (gv - Gi[n * NN + o]);
      const double d = un - Ui[(n + 1) * NN + o];
      acc[0] += d * d;
      Ui[(n + 1) * NN + o] = un;
      Gi[n * NN + o] = gv;
      u[s] = un;
    }
    group_sum<NW, G, 1>(acc, red, cc);
    dmax = fmax(dmax, acc[0]);
  }
  if (threadIdx.x == 0 && mem == 0) {
    const double dlt = sqrt(P.h * P.h * dmax);
    delta[ii] = dlt;
    if (!(dlt == dlt) || dlt > 1e300) status |= 2;
    status_out[ii] |= status | *P.status | (cc.ok ? 0 : 4);
  }
}

// ------------------------------------------------- pipelined iteration
// Several Parareal iterations (2.2) of one instance in one launch, with the
// fine solves of iteration j + 1 overlapped with the coarse sweep of
// iteration j.  The input U_n^{j+1} of a fine solve is final as soon as the
// sweep of iteration j has corrected slice n - 1, so the solve can start then
// rather than after the whole sweep; the sweep of iteration j + 1 in turn
// waits slice by slice for F(U_n^{j+1}).  Every value comes from the same
// code, in the same order, as in the two-launch iteration (fine_group_item,
// coop_approx2, the update of (2.2), the update norm), so the iterates agree
// bit for bit; only the schedule differs.
//
// Roles: group 0 runs the coarse sweep; the other groups (one may be left
// idle, see parareal_pipe) are fine groups 0..n_fine-1, persistent over the
// items (j, n) taken in iteration-major order (fine group q takes items q,
// q + n_fine, ...).  Iteration j covers slices k_j..N-1, with k_j = k0 + j
// (finished slices skipped) or k_j = k0 (sweep_all: every slice from k0 in
// every iteration, the same iterates with equal work per iteration).
// Hand-off buffers, written and read with the coherent accesses of the
// exchanges: Uin[j % 2] holds the fine inputs of iteration j, F0 / F1 the
// fine results of even / odd iterations.  Uin[j % 2][n] is rewritten only by
// the sweep of iteration j + 1, which starts after the sweep of iteration j
// has consumed item (j, n); F[j % 2][n] only by item (j + 2, n), whose input
// comes from that same later sweep.
// Counters (zeroed before the launch): ucnt[n] counts coarse-sweep members
// that have posted their part of a new input of slice n, fcnt[n] fine-group
// members that have posted F of slice n; ctl[0] = 1 + completed sweeps, set
// when the coarse sweep ends; ctl[1] = failure.
// No wait can deadlock while every workgroup is resident: item i waits only
// for the coarse sweep, which needs only items before i, and for its group's
// previous item, which comes before i.  Every wait is bounded by the wall
// clock as well (about 10 s).
struct PipeArgs {
  const InstDev* inst;
  const double* Tg;
  const double* lam;
  double* U;          // iterate layout (the instance's U_0..U_N)
  double* F0;         // slice layout: fine results of even iterations
  double* F1;         // N x n^2: fine results of odd iterations
  double* Uin;        // 2 x N x n^2: fine inputs
  double* G_old;
  double* delta;
  int32_t* status_out;
  const int32_t* active;
  const int32_t* kdev;
  int32_t* bar;       // barrier counters, 64 words per group
  int32_t* ucnt;
  int32_t* fcnt;
  int32_t* ctl;
  int ii, K, sweep_all, n_fine;
  int idle;           // group left without work (-1: none), see parareal_pipe
  double tol;
};

__device__ __forceinline__ int32_t pipe_ld(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Producer side of a hand-off: every wave waits until its coherent stores
// are acknowledged, then one thread adds the member's arrival.
__device__ __forceinline__ void pipe_post(int32_t* cnt) {
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Consumer side: one thread polls until *cnt >= target, then the workgroup
// reads the data with coherent loads.  Returns 1 when the count is reached;
// 0 (with until_end) when the coarse sweep has ended and a last look still
// finds the count short, so it will never come; -1 on a failure flagged by
// another group, on a time-out, or when this member has already failed.
__device__ int pipe_wait(const int32_t* cnt, int target, const int32_t* ctl, bool until_end,
                         int ok, uint64_t limit) {
  __shared__ int res_s;
  if (threadIdx.x == 0) {
    int res = -1;
    if (ok) {
      const uint64_t t0 = wall_clock64();
      while (true) {
        if (pipe_ld(cnt) >= target) { res = 1; break; }
        if (pipe_ld(ctl + 1)) { res = -1; break; }
        if (until_end && pipe_ld(ctl)) { res = pipe_ld(cnt) >= target ? 1 : 0; break; }
        if (wall_clock64() - t0 > limit) { res = -1; break; }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    res_s = res;
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);   // no compiler motion across the poll
  __syncthreads();
  return res_s;
}

__device__ __forceinline__ void pipe_fail(int32_t* ctl) {
  if (threadIdx.x == 0) __hip_atomic_store(ctl + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Coarse-sweep role: the correction sweeps of iterations 0..K-1 (the loop of
// k_chain_coop's mode 2, with the hand-offs added).
template <int N, int G, int NW, bool OPQ>
__device__ void pipe_coarse(const PipeArgs& A, const InstDev& P, int k0, double* Xs,
                            const double* T, const double* lamS, double* red, double* Dl,
                            double* Ml, double* Ql, CoopCtx& cc) {
  using C = GeoC<N, G, NW>;
  const int t = threadIdx.x, mem = cc.mem;
  const double tau = P.dT / P.m_coarse;
#pragma unroll
  for (int s = 0; s < C::OWN; ++s) {
    int row, col;
    slab_rc<N, G, NW, OPQ>(s, row, col);
    const double mu = -(lamS[row] + lamS[mem * C::B + col]);
    Dl[s * C::NT + t] = 1.0 / mu + tau * P.eps * P.eps * mu;
  }
  __syncthreads();
  const int64_t NN = (int64_t)N * N;
  const int Ns = P.n_slices;
  double* Ui = A.U + P.off_iter;
  double* Gi = A.G_old + P.off_slices;
  auto gidx = [&](int s) {
    int row, col;
    slab_rc<N, G, NW, OPQ>(s, row, col);
    return (int64_t)(mem * C::B + col) * N + row;
  };
  int status = 0, jdone = 0;
  bool fail = false;
  double u[C::OWN];
  for (int j = 0; j < A.K; ++j) {
    const int kj = A.sweep_all ? k0 : k0 + j;
    if (kj >= Ns) break;
    const double* Fj = (j & 1) ? A.F1 : A.F0 + P.off_slices;
    double* Un = A.Uin + (int64_t)((j + 1) & 1) * Ns * NN;   // inputs of iteration j + 1
    const int target = G * (j + 1);                          // members posting item (j, n)
    if (pipe_wait(A.fcnt + kj, target, A.ctl, false, cc.ok, P.pipe_wait_ticks) <= 0) { fail = true; break; }
    double dmax;
    {
      // U_{k+1} = F_k (slices up to k are final)
      double acc[1] = {0.0};
#pragma unroll
      for (int s = 0; s < C::OWN; ++s) {
        const int64_t o = gidx(s);
        const double un = xg_load(&Fj[kj * NN + o]);
        const double d = un - Ui[(kj + 1) * NN + o];
        acc[0] += d * d;
        Ui[(kj + 1) * NN + o] = un;
        u[s] = un;
        if (kj + 1 < Ns) xg_store(&Un[(kj + 1) * NN + o], un);
      }
      if (kj + 1 < Ns) pipe_post(A.ucnt + kj + 1);
      group_sum<NW, G, 1>(acc, red, cc);
      dmax = acc[0];
    }
    for (int n = kj + 1; n < Ns; ++n) {
      coop_approx2<N, G, NW, OPQ>(Xs, u, T, red, cc, P, Dl, Ml, Ql, lamS, status);
      if (pipe_wait(A.fcnt + n, target, A.ctl, false, cc.ok, P.pipe_wait_ticks) <= 0) { fail = true; break; }
      double acc[1] = {0.0};
#pragma unroll
      for (int s = 0; s < C::OWN; ++s) {
        const int64_t o = gidx(s);
        const double gv = u[s];
        const double un = xg_load(&Fj[n * NN + o]) + (gv - Gi[n * NN + o]);
        const double d = un - Ui[(n + 1) * NN + o];
        acc[0] += d * d;
        Ui[(n + 1) * NN + o] = un;
        Gi[n * NN + o] = gv;
        u[s] = un;
        if (n + 1 < Ns) xg_store(&Un[(n + 1) * NN + o], un);
      }
      if (n + 1 < Ns) pipe_post(A.ucnt + n + 1);
      group_sum<NW, G, 1>(acc, red, cc);
      dmax = fmax(dmax, acc[0]);
    }
    if (fail) break;
    const double dlt = sqrt(P.h * P.h * dmax);
    if (t == 0 && mem == 0) A.delta[A.ii] = dlt;
    jdone = j + 1;
    if (!(dlt == dlt) || dlt > 1e300) { status |= 2; break; }
    if (!cc.ok || dlt < A.tol) break;   // the rule of the active flags (k_flag_active)
  }
  // every member's posts are done before the end is published
  group_barrier<G>(cc);
  if (t == 0 && mem == 0) {
    const bool bad = fail || !cc.ok || pipe_ld(A.ctl + 1);
    A.status_out[A.ii] |= status | *P.status | (bad ? 4 : 0);
    if (bad) __hip_atomic_store(A.ctl + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(A.ctl, jdone + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else if (fail || !cc.ok) {
    pipe_fail(A.ctl);
  }
}

// Fine role: fine group q's items (j, n) in iteration-major order.
template <int N, int G, int NW, bool OPQ>
__device__ void pipe_fine(const PipeArgs& A, const InstDev& P, int k0, int q, double* Xs,
                          const double* T, const double* lamS, double* Rs, CoopCtx& cc) {
  const int64_t NN = (int64_t)N * N;
  const int Ns = P.n_slices;
  auto count = [&](int j) { return Ns - (A.sweep_all ? k0 : k0 + j); };   // items of iteration j
  int j = 0, r = q;
  while (j < A.K && count(j) > 0 && r >= count(j)) r -= count(j++);
  while (j < A.K && count(j) > 0) {
    const int n = (A.sweep_all ? k0 : k0 + j) + r;
    // the input comes from the copy made before the launch (iteration 0, and
    // slice k0, which no sweep rewrites) or from the sweep of iteration j - 1
    if (j > 0 && n > k0) {
      const int w = pipe_wait(A.ucnt + n, G * j, A.ctl, true, cc.ok, P.pipe_wait_ticks);
      if (w < 0) pipe_fail(A.ctl);
      if (w <= 0) break;
    }
    const double* src = A.Uin + (int64_t)(j & 1) * Ns * NN + n * NN;
    double* dst = ((j & 1) ? A.F1 : A.F0 + P.off_slices) + n * NN;
    fine_group_item<N, G, NW, OPQ, true>(P, Xs, T, lamS, Rs, cc, src, dst, 0);
    if (!cc.ok) {
      if (threadIdx.x == 0 && cc.mem == 0) atomicOr(P.status, 4);
      pipe_fail(A.ctl);
    }
    pipe_post(A.fcnt + n);
    r += A.n_fine;
    while (j < A.K && count(j) > 0 && r >= count(j)) r -= count(j++);
  }
}

// LDS: the coarse-sweep layout (the fine role uses the table region for 1 / sigma).
// Two workgroups per CU (at most 256 registers per lane) so that the coarse
// group and the fine groups fit a 256-CU device at once.
template <int N, int G, int NW>
__global__ void __launch_bounds__(NW * 64, 2)
k_parareal_pipe(PipeArgs A) {
  using C = GeoC<N, G, NW>;
  extern __shared__ double smem[];
  double* Xs = smem;
  double* T = smem + N * C::LDB;
  double* lamS = T + C::P2;
  double* red = lamS + N;
  double* Dl = red + 4 * NW;
  double* Ml = Dl + C::OWN * C::NT;
  double* Ql = Ml + C::OWN * C::NT;
  const int xcd = blockIdx.x % 8, rest = blockIdx.x / 8;
  const int mem = rest % G, grp = rest / G;
  const int idx = grp * 8 + xcd;   // 0: coarse sweep, then the fine groups
  if (idx == A.idle) return;
  const int q = idx - 1 - ((A.idle >= 0 && idx > A.idle) ? 1 : 0);   // fine group index
  if (idx > 0 && q >= A.n_fine) return;
  if (A.active && !A.active[A.ii]) return;
  const int slot = idx == 0 ? 0 : q + 1;   // barrier words and exchange area
  const InstDev P = A.inst[A.ii];
  for (int m = threadIdx.x; m < C::P2; m += C::NT) T[m] = A.Tg[m];
  for (int m = threadIdx.x; m < N; m += C::NT) lamS[m] = A.lam[m];
  __syncthreads();
  CoopCtx cc;
  cc.cnt = A.bar + slot * 64;
  cc.xg = P.work + (int64_t)slot * P.work_vecs * N * N;   // exchange area of the group
  cc.part = cc.xg + 2 * (int64_t)N * N;
  cc.mem = mem;
  cc.ok = 1;
  cc.xsel = 0;
  cc.psel = 0;
  cc.nb = 0;
  cc.limit = P.wait_ticks;
  const int k0 = *A.kdev;
  // the coarse sweep with recomputed lane addresses (it would need 370
  // registers otherwise), the fine solves with hoisted ones (faster, and they
  // fit the 256 registers of two workgroups per CU as they are)
  if (idx == 0) pipe_coarse<N, G, NW, true>(A, P, k0, Xs, T, lamS, red, Dl, Ml, Ql, cc);
  else pipe_fine<N, G, NW, false>(A, P, k0, q, Xs, T, lamS, Dl, cc);
}

__global__ void k_copy2(const double* __restrict__ src, double* __restrict__ d0,
                        double* __restrict__ d1, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) {
    const double v = src[i];
    d0[i] = v;
    d1[i] = v;
  }
}

// The device iteration counter advances by the completed sweeps.
__global__ void k_pipe_finish(int32_t* kdev, const int32_t* ctl) {
  if (threadIdx.x == 0 && ctl[0] > 0) *kdev += ctl[0] - 1;
}

// ------------------------------------------------- streamed large grids
// n = 256: the 512 KB FP64 state does not fit on a CU, so each transform
// stage streams it between two global buffers of the work item (L2 / MALL
// resident) and stages its B operand through a double-buffered LDS chunk.
// A stage computes Y = S X for the folded rows in two column halves (the
// accumulators of one half fill the register budget) and writes Y^T.
template <int N, int NW>
struct GeoS {
  static constexpr int H = N / 2, TR = H / 16, HALF = N / 2, TCH = HALF / 16;
  static constexpr int MC = 16;                 // folded k (m) per LDS chunk
  static constexpr int CR = 2 * MC;             // X rows per chunk
  static constexpr int LDC = HALF + 8;          // chunk row stride (doubles)
  static constexpr int CHUNK = CR * LDC;        // doubles per chunk buffer
  static constexpr int NT = NW * 64, P2 = 2 * (N + 1);
  static_assert(TR == NW, "one wave per 16 folded rows");
  static_assert((CR * HALF) % NT == 0, "chunk load tiling");
};

template <int N, int NW>
__device__ __attribute__((noinline)) void stream_stage(const double* __restrict__ Xg, double* __restrict__ Out,
                             const double* __restrict__ w, double* Lc, const double* T) {
  using G = GeoS<N, NW>;
  const int t = threadIdx.x, l = t & 63, wv = t >> 6, g = l >> 4, j = l & 15;
  const int tr = wv;
  const int a1 = 16 * tr + j + 1;
  constexpr int PER = G::CR * G::HALF / G::NT;   // doubles per thread per chunk load
  for (int hc = 0; hc < 2; ++hc) {
    d4 aE[G::TCH], aO[G::TCH];
#pragma unroll
    for (int q = 0; q < G::TCH; ++q) {
      aE[q] = d4{0.0, 0.0, 0.0, 0.0};
      aO[q] = d4{0.0, 0.0, 0.0, 0.0};
    }
    double pf[PER];
    // chunk c covers X rows [2 MC c, 2 MC c + 2 MC), columns [HALF hc, HALF hc + HALF)
    auto fetch = [&](int c) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = i * G::NT + t, r = e / G::HALF, col = e % G::HALF;
        pf[i] = Xg[(int64_t)(2 * G::MC * c + r) * N + G::HALF * hc + col];
      }
    };
    auto put = [&](double* buf) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = i * G::NT + t, r = e / G::HALF, col = e % G::HALF;
        buf[r * G::LDC + col] = pf[i];
      }
    };
    constexpr int NCH = G::H / G::MC;
    fetch(0);
    __syncthreads();   // previous users of the chunk buffers are done
    put(Lc);
    __syncthreads();
    int ie = (a1 * (2 * g + 1)) % G::P2, io = (a1 * (2 * g + 2)) % G::P2;
    const int step = (8 * a1) % G::P2;
    for (int c = 0; c < NCH; ++c) {
      double* cur = Lc + (c & 1) * G::CHUNK;
      if (c + 1 < NCH) fetch(c + 1);
#pragma unroll
      for (int kl = 0; kl < G::MC / 4; ++kl) {
        const double se = T[ie], so = T[io];
        ie += step; ie -= (ie >= G::P2) ? G::P2 : 0;
        io += step; io -= (io >= G::P2) ? G::P2 : 0;
        const double* pe = cur + (2 * (4 * kl + g)) * G::LDC + j;
#pragma unroll
        for (int q = 0; q < G::TCH; ++q) {
          aE[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(se, pe[16 * q], aE[q], 0, 0, 0);
          aO[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(so, pe[G::LDC + 16 * q], aO[q], 0, 0, 0);
        }
      }
      if (c + 1 < NCH) put(Lc + ((c + 1) & 1) * G::CHUNK);
      __syncthreads();
    }
    // epilogue: Out[c][a] = Y[a][c] times w[c][a] (w indexed like Out)
#pragma unroll
    for (int q = 0; q < G::TCH; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * tr + g + 4 * r, cc = G::HALF * hc + 16 * q + j;
        double top = aE[q][r] + aO[q][r], bot = aE[q][r] - aO[q][r];
        if (w) {
          top *= w[(int64_t)cc * N + a];
          bot *= w[(int64_t)cc * N + (N - 1 - a)];
        }
        Out[(int64_t)cc * N + a] = top;
        Out[(int64_t)cc * N + (N - 1 - a)] = bot;
      }
  }
  __syncthreads();   // Out complete before anyone reads it
}

// r = u + c_lap Lap5(f(u) - s u) on global arrays (zero boundary ghosts).
template <int N, int NW>
__device__ void stream_rhs(const double* __restrict__ u, double* __restrict__ r, double c_lap,
                           double s, int f_zero) {
  for (int idx = threadIdx.x; idx < N * N; idx += NW * 64) {
    const int iy = idx / N, ix = idx % N;
    auto wof = [&](double v) { return f_zero ? -s * v : v * v * v - (1.0 + s) * v; };
    const double c = u[idx];
    const double wn = iy > 0 ? wof(u[idx - N]) : 0.0, ws = iy < N - 1 ? wof(u[idx + N]) : 0.0;
    const double ww = ix > 0 ? wof(u[idx - 1]) : 0.0, we = ix < N - 1 ? wof(u[idx + 1]) : 0.0;
    r[idx] = c + c_lap * ((wn + ws) + (ww + we) - 4.0 * wof(c));
  }
  __syncthreads();
}

// nsteps linear steps of the state in b0 (global); the result ends in b0.
template <int N, int NW>
__device__ void stream_linear_steps(double* b0, double* b1, double* Lc, const double* T,
                                    int nsteps, double c_lap, double s, int f_zero,
                                    const double* __restrict__ rsig) {
  for (int m = 0; m < nsteps; ++m) {
    stream_rhs<N, NW>(b0, b1, c_lap, s, f_zero);
    stream_stage<N, NW>(b1, b0, nullptr, Lc, T);
    stream_stage<N, NW>(b0, b1, rsig, Lc, T);
    stream_stage<N, NW>(b1, b0, nullptr, Lc, T);
    stream_stage<N, NW>(b0, b1, nullptr, Lc, T);
    for (int idx = threadIdx.x; idx < N * N; idx += NW * 64) b0[idx] = b1[idx];
    __syncthreads();
  }
}

template <int N, int NW>
__global__ void __launch_bounds__(NW * 64)
k_fine_linear_stream(const WorkItem* __restrict__ items, const InstDev* __restrict__ inst,
                     const double* __restrict__ Tg, const double* __restrict__ U_in,
                     double* __restrict__ F_out, const uint8_t* __restrict__ mask,
                     const int32_t* __restrict__ active, const int32_t* __restrict__ kmin, int in_iter,
                     int j_steps) {
  using G = GeoS<N, NW>;
  extern __shared__ double smem[];
  double* Lc = smem;
  double* T = smem + 2 * G::CHUNK;
  const WorkItem it = items[blockIdx.x];
  const InstDev P = inst[it.inst];
  if (mask && !mask[P.slice_base + it.slice]) return;
  if ((kmin && it.slice < *kmin) || (active && !active[it.inst])) return;
  const int64_t NN = (int64_t)N * N;
  const int64_t off = P.off_slices + (int64_t)it.slice * NN;
  const int64_t off_in = (in_iter ? P.off_iter : P.off_slices) + (int64_t)it.slice * NN;
  double* b0 = P.work + (int64_t)it.slice * P.work_vecs * NN;
  double* b1 = b0 + NN;
  for (int m = threadIdx.x; m < G::P2; m += G::NT) T[m] = Tg[m];
  for (int idx = threadIdx.x; idx < NN; idx += G::NT) b0[idx] = U_in[off_in + idx];
  __syncthreads();
  stream_linear_steps<N, NW>(b0, b1, Lc, T, j_steps > 0 ? j_steps : P.j_fine, P.dt / (P.h * P.h),
                             P.s_fine, P.f_zero, P.rsig_fine);
  for (int idx = threadIdx.x; idx < NN; idx += G::NT) F_out[off + idx] = b0[idx];
}

// Whole-workgroup reductions of values produced in strided passes.
template <int NW, int K>
__device__ __forceinline__ void wg_sum(double (&v)[K], double* red) { block_sum<NW, K>(v, red); }

// Streamed spectral CG for diag(d) + tau S diag(q) S (see spectral_cg): the
// right-hand side is in cr on entry (natural order), the solution is left in
// cx.  b0, b1 are transform scratch.  Returns iterations or -1.
template <int N, int NW>
__device__ int stream_spectral_cg(double* b0, double* b1, double* cx, double* cr, double* cp,
                                  const double* cq, double* cm, const double* cd, double tau,
                                  double cshift, double rtol, int maxit, double* Lc,
                                  const double* T, double* red) {
  const int NN = N * N, NT = NW * 64, t = threadIdx.x;
  double acc[2] = {0.0, 0.0};
  for (int i = t; i < NN; i += NT) {
    const double b = cr[i];
    const double mi = 1.0 / (cd[i] + tau * cshift);
    cm[i] = mi;
    cx[i] = 0.0;
    cp[i] = b * mi;
    acc[0] += b * b * mi;
    acc[1] += b * b;
  }
  wg_sum<NW, 2>(acc, red);
  double rz = acc[0];
  const double stop2 = rtol * rtol * acc[1];
  if (!(acc[1] > 0.0)) return 0;
  for (int it = 1; it <= maxit; ++it) {
    stream_stage<N, NW>(cp, b0, nullptr, Lc, T);
    stream_stage<N, NW>(b0, b1, cq, Lc, T);       // q . (S p S)
    stream_stage<N, NW>(b1, b0, nullptr, Lc, T);
    stream_stage<N, NW>(b0, b1, nullptr, Lc, T);  // b1 = S (q . S p S) S
    double a1[1] = {0.0};
    for (int i = t; i < NN; i += NT) {
      const double kp = cd[i] * cp[i] + tau * b1[i];
      b1[i] = kp;
      a1[0] += cp[i] * kp;
    }
    wg_sum<NW, 1>(a1, red);
    const double alpha = rz / a1[0];
    double a2[2] = {0.0, 0.0};
    for (int i = t; i < NN; i += NT) {
      cx[i] += alpha * cp[i];
      const double r = cr[i] - alpha * b1[i];
      cr[i] = r;
      a2[0] += r * r;
      a2[1] += r * (r * cm[i]);
    }
    wg_sum<NW, 2>(a2, red);
    if (a2[0] <= stop2) return it;
    if (!(a2[0] == a2[0])) return -1;
    const double beta = a2[1] / rz;
    rz = a2[1];
    for (int i = t; i < NN; i += NT) cp[i] = cr[i] * cm[i] + beta * cp[i];
    __syncthreads();
  }
  return -1;
}

// Scheme (2.4) on the streamed state in b0 (global), result in b0.  Tables
// d (coarse tau) and 1/mu + tau in P.tab (natural order for n = 256).
// `steps` steps of tau; cd, cb, boff as in approx2_steps.
template <int N, int NW>
__device__ void stream_approx2(double* b0, double* b1, double* cx, double* cr, double* cp,
                               double* cq, double* cm, double* Lc, const double* T, double* red,
                               const InstDev& P, double tau, int steps, const double* cd,
                               const double* cb, double boff, int& status) {
  const int NN = N * N, NT = NW * 64, t = threadIdx.x;
  for (int sub = 0; sub < steps; ++sub) {
    double mn = 1e300, mx = -1e300;
    for (int i = t; i < NN; i += NT) {
      const double q = P.f_zero ? 0.0 : b0[i] * b0[i];
      cq[i] = q;
      mn = fmin(mn, q);
      mx = fmax(mx, q);
    }
    block_minmax<NW>(mn, mx, red);
    const double cshift = 0.5 * (mn + mx);
    stream_stage<N, NW>(b0, b1, nullptr, Lc, T);
    stream_stage<N, NW>(b1, b0, nullptr, Lc, T);   // b0 = u_hat
    for (int i = t; i < NN; i += NT) cr[i] = (cb[i] + boff) * b0[i];
    __syncthreads();
    const int its = stream_spectral_cg<N, NW>(b0, b1, cx, cr, cp, cq, cm, cd, tau, cshift,
                                              P.krylov_rtol, P.krylov_max, Lc, T, red);
    if (its < 0) status |= 1;
    stream_stage<N, NW>(cx, b1, nullptr, Lc, T);
    stream_stage<N, NW>(b1, b0, nullptr, Lc, T);   // b0 = v
  }
}

// Implicit fine step (see newton_step) on streamed vectors: the state is
// carried in sine coordinates (uh, yh, natural order).
// tau, cd (the table 1/mu + tau eps^2 mu of that tau), be: as in newton_step.
template <int N, int NW>
__device__ bool stream_newton_step(double* b0, double* b1, double* cx, double* cr, double* cp,
                                   double* cq, double* cm, double* uh, double* yh, double* Lc,
                                   const double* T, double* red, const InstDev& P, double tau,
                                   const double* cd, bool be) {
  const int NN = N * N, NT = NW * 64, t = threadIdx.x;
  const double* imu = P.tab + 3 * NN;
  bool ok = true;
  for (int it = 0; it < P.newton_max; ++it) {
    stream_stage<N, NW>(yh, b1, nullptr, Lc, T);
    stream_stage<N, NW>(b1, b0, nullptr, Lc, T);   // b0 = Y (state)
    double mn = 1e300, mx = -1e300;
    for (int i = t; i < NN; i += NT) {
      const double y = b0[i];
      const double q = P.f_zero ? 0.0 : 3.0 * y * y + (be ? -1.0 : 0.0);
      cq[i] = q;
      b1[i] = P.f_zero ? 0.0 : y * y * y;
      mn = fmin(mn, q);
      mx = fmax(mx, q);
    }
    block_minmax<NW>(mn, mx, red);
    const double cshift = 0.5 * (mn + mx);
    stream_stage<N, NW>(b1, b0, nullptr, Lc, T);
    stream_stage<N, NW>(b0, b1, nullptr, Lc, T);   // b1 = S Y^3 S
    for (int i = t; i < NN; i += NT) {
      double g;
      if (P.f_zero) g = cd[i] * yh[i] - imu[i] * uh[i];
      else if (be) g = cd[i] * yh[i] + tau * b1[i] - tau * yh[i] - imu[i] * uh[i];
      else g = cd[i] * yh[i] + tau * b1[i] - (imu[i] + tau) * uh[i];
      cr[i] = -g;
    }
    __syncthreads();
    const int its = stream_spectral_cg<N, NW>(b0, b1, cx, cr, cp, cq, cm, cd, tau, cshift,
                                              P.nl_krylov_rtol, P.krylov_max, Lc, T, red);
    if (its < 0) ok = false;
    double a[1] = {0.0};
    for (int i = t; i < NN; i += NT) {
      yh[i] += cx[i];
      a[0] += cx[i] * cx[i];
    }
    wg_sum<NW, 1>(a, red);
    const double step = sqrt(P.h * P.h * a[0]);
    if (step <= P.newton_tol) return ok;
    if (!(step == step)) return false;
  }
  return false;
}

template <int N, int NW>
__global__ void __launch_bounds__(NW * 64)
k_fine_newton_stream(const WorkItem* __restrict__ items, const InstDev* __restrict__ inst,
                     const double* __restrict__ Tg, const double* __restrict__ U_in,
                     double* __restrict__ F_out, const uint8_t* __restrict__ mask,
                     const int32_t* __restrict__ active, const int32_t* __restrict__ kmin,
                     int in_iter) {
  using G = GeoS<N, NW>;
  extern __shared__ double smem[];
  double* Lc = smem;
  double* T = smem + 2 * G::CHUNK;
  double* red = T + G::P2;
  const WorkItem it = items[blockIdx.x];
  const InstDev P = inst[it.inst];
  if (mask && !mask[P.slice_base + it.slice]) return;
  if ((kmin && it.slice < *kmin) || (active && !active[it.inst])) return;
  const int64_t NN = (int64_t)N * N;
  const int64_t off = P.off_slices + (int64_t)it.slice * NN;
  const int64_t off_in = (in_iter ? P.off_iter : P.off_slices) + (int64_t)it.slice * NN;
  double* w = P.work + (int64_t)it.slice * P.work_vecs * NN;
  double *b0 = w, *b1 = w + NN, *cx = w + 2 * NN, *cr = w + 3 * NN, *cp = w + 4 * NN;
  double *cq = w + 5 * NN, *cm = w + 6 * NN, *uh = w + 7 * NN, *yh = w + 8 * NN;
  const int t = threadIdx.x;
  for (int m = t; m < G::P2; m += G::NT) T[m] = Tg[m];
  for (int64_t i = t; i < NN; i += G::NT) b0[i] = U_in[off_in + i];
  __syncthreads();
  stream_stage<N, NW>(b0, b1, nullptr, Lc, T);
  stream_stage<N, NW>(b1, uh, nullptr, Lc, T);   // u_hat
  for (int64_t i = t; i < NN; i += G::NT) yh[i] = uh[i];
  __syncthreads();
  bool ok = true;
  for (int m = 0; m < P.j_fine; ++m) {
    ok = stream_newton_step<N, NW>(b0, b1, cx, cr, cp, cq, cm, uh, yh, Lc, T, red, P, P.dt,
                                   P.tab + 2 * NN, P.nl_variant == 1) && ok;
    for (int64_t i = t; i < NN; i += G::NT) uh[i] = yh[i];
    __syncthreads();
  }
  stream_stage<N, NW>(uh, b1, nullptr, Lc, T);
  stream_stage<N, NW>(b1, b0, nullptr, Lc, T);
  for (int64_t i = t; i < NN; i += G::NT) F_out[off + i] = b0[i];
  if (!ok && t == 0) atomicOr(P.status, 1);
}

// Coarse step on the streamed state in b0 = w (work vectors w: 7 for the
// linear kinds, 9 for scheme (2.3)).
template <int N, int NW>
__device__ void stream_coarse_apply(double* b0, const InstDev& P, double* w, double* Lc,
                                    const double* T, double* red, int& status) {
  const int64_t NN = (int64_t)N * N;
  const double tau = P.dT / P.m_coarse;
  if (P.coarse_kind == 1) {
    stream_linear_steps<N, NW>(b0, w + NN, Lc, T, P.m_coarse, tau / (P.h * P.h), P.s_fine,
                               P.f_zero, P.rsig_stab);
  } else if (P.coarse_kind == 3) {
    // NPA-II: m_coarse steps of scheme (2.3) by Newton, state in sine
    // coordinates (uh, yh) between the steps
    double *b1 = w + NN, *uh = w + 7 * NN, *yh = w + 8 * NN;
    const int t = threadIdx.x, NT = NW * 64;
    for (int sub = 0; sub < P.m_coarse; ++sub) {
      stream_stage<N, NW>(b0, b1, nullptr, Lc, T);
      stream_stage<N, NW>(b1, uh, nullptr, Lc, T);   // u_hat
      for (int64_t i = t; i < NN; i += NT) yh[i] = uh[i];
      __syncthreads();
      if (!stream_newton_step<N, NW>(b0, b1, w + 2 * NN, w + 3 * NN, w + 4 * NN, w + 5 * NN,
                                     w + 6 * NN, uh, yh, Lc, T, red, P, tau, P.tab, false))
        status |= 1;
      stream_stage<N, NW>(yh, b1, nullptr, Lc, T);
      stream_stage<N, NW>(b1, b0, nullptr, Lc, T);   // b0 = the new state
    }
  } else {
    stream_approx2<N, NW>(b0, w + NN, w + 2 * NN, w + 3 * NN, w + 4 * NN, w + 5 * NN, w + 6 * NN,
                          Lc, T, red, P, tau, P.m_coarse, P.tab, P.tab + NN,
                          P.f_zero ? -tau : 0.0, status);
  }
}

// PA-I fine sweep on streamed vectors (n = 256): J steps of scheme (2.4)
// with tau = dt per work item, one workgroup each.
template <int N, int NW>
__global__ void __launch_bounds__(NW * 64)
k_fine_approx2_stream(const WorkItem* __restrict__ items, const InstDev* __restrict__ inst,
                      const double* __restrict__ Tg, const double* __restrict__ U_in,
                      double* __restrict__ F_out, const uint8_t* __restrict__ mask,
                      const int32_t* __restrict__ active, const int32_t* __restrict__ kmin,
                      int in_iter) {
  using G = GeoS<N, NW>;
  extern __shared__ double smem[];
  double* Lc = smem;
  double* T = smem + 2 * G::CHUNK;
  double* red = T + G::P2;
  const WorkItem it = items[blockIdx.x];
  const InstDev P = inst[it.inst];
  if (mask && !mask[P.slice_base + it.slice]) return;
  if ((kmin && it.slice < *kmin) || (active && !active[it.inst])) return;
  const int64_t NN = (int64_t)N * N;
  const int64_t off = P.off_slices + (int64_t)it.slice * NN;
  const int64_t off_in = (in_iter ? P.off_iter : P.off_slices) + (int64_t)it.slice * NN;
  double* w = P.work + (int64_t)it.slice * P.work_vecs * NN;
  const int t = threadIdx.x;
  for (int m = t; m < G::P2; m += G::NT) T[m] = Tg[m];
  for (int64_t i = t; i < NN; i += G::NT) w[i] = U_in[off_in + i];
  __syncthreads();
  int status = 0;
  stream_approx2<N, NW>(w, w + NN, w + 2 * NN, w + 3 * NN, w + 4 * NN, w + 5 * NN, w + 6 * NN,
                        Lc, T, red, P, P.dt, P.j_fine, P.tab + 2 * NN, P.tab + 3 * NN,
                        P.f_zero ? 0.0 : P.dt, status);
  for (int64_t i = t; i < NN; i += G::NT) F_out[off + i] = w[i];
  if (status && t == 0) atomicOr(P.status, status);
}

// Streamed counterpart of k_coarse_2d (same modes).  Work vectors: b0 =
// work[0] holds the state, the rest are solver scratch.
template <int N, int NW>
__global__ void __launch_bounds__(NW * 64)
k_coarse_stream(int mode, const int32_t* __restrict__ insts, const WorkItem* __restrict__ items,
                const InstDev* __restrict__ inst, const double* __restrict__ Tg,
                const double* __restrict__ U_in, double* __restrict__ G_out,
                const uint8_t* __restrict__ mask, double* U, const double* __restrict__ F,
                double* G_old, double* delta, int32_t* status_out,
                const int32_t* __restrict__ active, int k, const int32_t* __restrict__ kdev,
                const int32_t* __restrict__ gate) {
  using G = GeoS<N, NW>;
  if (kdev) k = *kdev;
  extern __shared__ double smem[];
  double* Lc = smem;
  double* T = smem + 2 * G::CHUNK;
  double* red = T + G::P2;
  const int64_t NN = (int64_t)N * N;
  const int t = threadIdx.x;
  int status = 0;
  for (int m = t; m < G::P2; m += G::NT) T[m] = Tg[m];
  if (mode == 0 || mode >= 3) {
    const WorkItem it = items[blockIdx.x];
    InstDev P = inst[it.inst];
    int64_t off_in = P.off_slices + (int64_t)it.slice * NN;
    if (mode == 0) {
      if (mask && !mask[P.slice_base + it.slice]) return;
      if (P.coarse_kind == 2) return;
    } else {   // plain (2.4) of gated slices (see k_coarse_2d)
      if (!gate[mode == 4 ? 0 : it.inst]) return;
      P.coarse_kind = 0;
      if (mode != 5) off_in = P.off_iter + (int64_t)it.slice * NN;
    }
    double* w = P.work + (int64_t)it.slice * P.work_vecs * NN;
    const int64_t off = P.off_slices + (int64_t)it.slice * NN;
    for (int64_t i = t; i < NN; i += G::NT) w[i] = U_in[off_in + i];
    __syncthreads();
    stream_coarse_apply<N, NW>(w, P, w, Lc, T, red, status);
    for (int64_t i = t; i < NN; i += G::NT) G_out[off + i] = w[i];
    if (status && t == 0) atomicOr(P.status, status);
    return;
  }
  const int ii = insts[blockIdx.x];
  if (active && !active[ii]) return;
  const InstDev P = inst[ii];
  if (P.coarse_kind == 2) return;
  double* w = P.work;
  double* Ui = U + P.off_iter;
  const double* Fi = F + P.off_slices;
  double* Gi = G_old + P.off_slices;
  const int Ns = P.n_slices;
  if (mode == 1) {
    for (int64_t i = t; i < NN; i += G::NT) w[i] = Ui[i];
    __syncthreads();
    for (int n = 0; n < Ns; ++n) {
      stream_coarse_apply<N, NW>(w, P, w, Lc, T, red, status);
      for (int64_t i = t; i < NN; i += G::NT) {
        Ui[(n + 1) * NN + i] = w[i];
        Gi[n * NN + i] = w[i];
      }
      __syncthreads();
    }
    if (t == 0) status_out[ii] = status | *P.status;
    return;
  }
  if (k >= Ns) {
    if (t == 0) delta[ii] = 0.0;
    return;
  }
  double dmax;
  {
    double acc[1] = {0.0};
    for (int64_t i = t; i < NN; i += G::NT) {
      const double un = Fi[k * NN + i];
      const double d = un - Ui[(k + 1) * NN + i];
      acc[0] += d * d;
      Ui[(k + 1) * NN + i] = un;
      w[i] = un;
    }
    block_sum<NW, 1>(acc, red);
    dmax = acc[0];
  }
  for (int n = k + 1; n < Ns; ++n) {
    stream_coarse_apply<N, NW>(w, P, w, Lc, T, red, status);
    double acc[1] = {0.0};
    for (int64_t i = t; i < NN; i += G::NT) {
      const double gv = w[i];
      const double un = Fi[n * NN + i] + (gv - Gi[n * NN + i]);
      const double d = un - Ui[(n + 1) * NN + i];
      acc[0] += d * d;
      Ui[(n + 1) * NN + i] = un;
      Gi[n * NN + i] = gv;
      w[i] = un;
    }
    block_sum<NW, 1>(acc, red);
    dmax = fmax(dmax, acc[0]);
  }
  if (t == 0) {
    const double dlt = sqrt(P.h * P.h * dmax);
    delta[ii] = dlt;
    if (!(dlt == dlt) || dlt > 1e300) status |= 2;
    status_out[ii] |= status | *P.status;
  }
}

// Natural-order spectral tables for streamed instances (see k_cg_tables_2d).
__global__ void k_cg_tables_natural(const int32_t* __restrict__ insts,
                                    const InstDev* __restrict__ inst, const double* __restrict__ lam) {
  const InstDev P = inst[insts[blockIdx.y]];
  const int n = P.n;
  const int64_t NN = (int64_t)n * n;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= NN) return;
  const double mu = -(lam[i / n] + lam[i % n]);
  const double tc = P.dT / P.m_coarse, tf = P.dt;
  P.tab[i] = 1.0 / mu + tc * P.eps * P.eps * mu;
  P.tab[NN + i] = 1.0 / mu + tc;
  P.tab[2 * NN + i] = 1.0 / mu + tf * P.eps * P.eps * mu;
  P.tab[3 * NN + i] = 1.0 / mu;
}

// ------------------------------------------- split-BF16 linear fine step
// Reduced-precision variant of the linear step: the sine transforms run on
// the BF16 matrix cores as three products S_hi X_hi + S_hi X_lo + S_lo X_hi
// (hi = bf16(x), lo = bf16(x - hi), both round-to-nearest-even; lo*lo
// dropped) accumulated in FP32, inside an FP64 defect correction:
//   u1 = u + P^{-1}_lp d,        d = tau Lap (f(u) - eps^2 Lap u)       (= rhs - P u)
//   u2 = u1 + P^{-1}_lp r,       r = (u - u1) + tau Lap (f(u) - s u - eps^2 Lap u1 + s u1)
// with P = I + tau eps^2 Lap^2 - s tau Lap.  The FP64 state lives in
// registers; the defect and residual stencils use an FP64 LDS buffer that
// aliases the BF16 transform buffer.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <int N, int NW>
struct GeoB {
  static constexpr int H = N / 2, TR = H / 16, TC = N / 16, WPR = NW / TR, CPW = TC / WPR;
  static constexpr int KS = H / 32;           // k-steps of 32
  static constexpr int RS = 2 * N + 8;        // split-buffer row stride (bf16): Eh|El|Oh|Ol|pad
  static constexpr int NT = NW * 64, OWN = 8 * CPW;
  static constexpr int LDX = N + 3, XSZ = (N + 2) * LDX, XOFF = LDX + 1;  // FP64 stencil buffer
  static_assert(KS >= 1, "bf16 k-steps need n >= 64");
  static_assert(NW % TR == 0 && TC % WPR == 0, "wave tiling");
  static_assert(OWN * NT == N * N, "ownership");
  static_assert((size_t)N * RS * 2 <= (size_t)XSZ * 8, "split buffer fits in the FP64 buffer");
};

// BF16 MFMA 16x16x32 lane layout: A[i][k] i = l%16, k = 8(l/16)+e; B[k][j]
// k = 8(l/16)+e, j = l%16; D[i][j] in element r: i = 4(l/16) + r, j = l%16.
template <int N, int NW>
struct LaneB {
  int g, j, tr, c0;
  __device__ LaneB() {
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    g = l >> 4;
    j = l & 15;
    tr = w / GeoB<N, NW>::WPR;
    c0 = (w % GeoB<N, NW>::WPR) * GeoB<N, NW>::CPW;
  }
  __device__ __forceinline__ int row_a(int r) const { return 16 * tr + 4 * g + r; }
  __device__ __forceinline__ int col_c(int q) const { return 16 * (c0 + q) + j; }
};
// slot (q*4 + r)*2 + half: Y[a][c] (half 0) / Y[N-1-a][c] (half 1); state point (row c, col a|N-1-a)
template <int N, int NW>
__device__ __forceinline__ void ownb_rc(const LaneB<N, NW>& L, int slot, int& row, int& col) {
  const int qr = slot >> 1, half = slot & 1, q = qr >> 2, r = qr & 3;
  const int a = L.row_a(r);
  row = L.col_c(q);
  col = half ? (N - 1 - a) : a;
}

__device__ __forceinline__ __bf16 bf16_rne(float x) { return (__bf16)x; }

// Write value v of logical position Y[yr][yc] into the split buffer (row yr,
// even/odd column halves, hi and lo parts).
template <int N, int NW>
__device__ __forceinline__ void split_put(__bf16* SB, int yr, int yc, float v) {
  using G = GeoB<N, NW>;
  const __bf16 hi = bf16_rne(v);
  const __bf16 lo = bf16_rne(v - (float)hi);
  const int base = yr * G::RS + ((yc & 1) ? 2 * G::H : 0) + (yc >> 1);
  SB[base] = hi;
  SB[base + G::H] = lo;
}

// Owned values (state orientation, see ownb_rc) as the input of a transform:
// the value at state (row c, col a) is the logical Y_0[a][c].
template <int N, int NW>
__device__ __forceinline__ void split_store_owned(__bf16* SB, const LaneB<N, NW>& L,
                                                  const double (&v)[GeoB<N, NW>::OWN]) {
#pragma unroll
  for (int s = 0; s < GeoB<N, NW>::OWN; ++s) {
    int row, col;
    ownb_rc<N, NW>(L, s, row, col);
    split_put<N, NW>(SB, col, row, (float)v[s]);
  }
}

struct SineB {       // A operands (hi/lo of the folded sine rows), k-steps of 32
  bf8 eh[2], el[2], oh[2], ol[2];
};
template <int N, int NW>
__device__ __forceinline__ void sine_operands(const double* __restrict__ Tg, const LaneB<N, NW>& L,
                                              SineB& A) {
  using G = GeoB<N, NW>;
  constexpr int P2 = 2 * (N + 1);
  const int a1 = 16 * L.tr + L.j + 1;
#pragma unroll
  for (int ks = 0; ks < G::KS; ++ks)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 32 * ks + 8 * L.g + e;
      const double se = Tg[(a1 * (2 * k + 1)) % P2];
      const double so = Tg[(a1 * (2 * k + 2)) % P2];
      const __bf16 seh = bf16_rne((float)se), soh = bf16_rne((float)so);
      A.eh[ks][e] = seh;
      A.el[ks][e] = bf16_rne((float)(se - (double)(float)seh));
      A.oh[ks][e] = soh;
      A.ol[ks][e] = bf16_rne((float)(so - (double)(float)soh));
    }
}

// One split-BF16 stage: Y = S X (three BF16 products, FP32 accumulation),
// unfolded into owned FP32 values y[slot] (see ownb_rc for the positions).
template <int N, int NW>
__device__ __forceinline__ void split_stage(const __bf16* SB, const SineB& A, const LaneB<N, NW>& L,
                                            float (&y)[GeoB<N, NW>::OWN]) {
  using G = GeoB<N, NW>;
  f4 aE[G::CPW], aO[G::CPW];
#pragma unroll
  for (int q = 0; q < G::CPW; ++q) {
    aE[q] = f4{0.f, 0.f, 0.f, 0.f};
    aO[q] = f4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int ks = 0; ks < G::KS; ++ks) {
#pragma unroll
    for (int q = 0; q < G::CPW; ++q) {
      const __bf16* row = SB + (16 * (L.c0 + q) + L.j) * G::RS + 32 * ks + 8 * L.g;
      const bf8 beh = *(const bf8*)(row);
      const bf8 bel = *(const bf8*)(row + G::H);
      const bf8 boh = *(const bf8*)(row + 2 * G::H);
      const bf8 bol = *(const bf8*)(row + 3 * G::H);
      aE[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.eh[ks], beh, aE[q], 0, 0, 0);
      aE[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.eh[ks], bel, aE[q], 0, 0, 0);
      aE[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.el[ks], beh, aE[q], 0, 0, 0);
      aO[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.oh[ks], boh, aO[q], 0, 0, 0);
      aO[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.oh[ks], bol, aO[q], 0, 0, 0);
      aO[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.ol[ks], boh, aO[q], 0, 0, 0);
    }
  }
#pragma unroll
  for (int q = 0; q < G::CPW; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      y[(q * 4 + r) * 2 + 0] = aE[q][r] + aO[q][r];
      y[(q * 4 + r) * 2 + 1] = aE[q][r] - aO[q][r];
    }
}

// Low-precision solve P^{-1} v of the owned FP64 values v (state orientation),
// result (FP64 of the FP32 result) back in v.  Four stages; the symbol
// 1/sigma is applied after the second, computed from the eigenvalues lamS
// (LDS) as 1/(1 + tau eps^2 Lam^2 - s tau Lam), Lam = lam_p + lam_q, at the
// owned spectral positions (no table reads from memory inside the step).
template <int N, int NW>
__device__ void split_solve(__bf16* SB, const SineB& A, const LaneB<N, NW>& L,
                            double (&v)[GeoB<N, NW>::OWN], const double* __restrict__ lamS,
                            double tau, double e2, double sfine) {
  using G = GeoB<N, NW>;
  float y[G::OWN];
  __syncthreads();
  split_store_owned<N, NW>(SB, L, v);
  __syncthreads();
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    split_stage<N, NW>(SB, A, L, y);
    if (st == 1) {
#pragma unroll
      for (int s = 0; s < G::OWN; ++s) {
        const int qr = s >> 1, half = s & 1, q = qr >> 2, r = qr & 3;
        const int a = L.row_a(r), yr = half ? (N - 1 - a) : a, yc = L.col_c(q);
        const double Lam = lamS[yr] + lamS[yc];
        y[s] *= (float)(1.0 / (1.0 + tau * e2 * Lam * Lam - sfine * tau * Lam));
      }
    }
    if (st < 3) {
      __syncthreads();
#pragma unroll
      for (int s = 0; s < G::OWN; ++s) {
        const int qr = s >> 1, half = s & 1, q = qr >> 2, r = qr & 3;
        const int a = L.row_a(r);
        split_put<N, NW>(SB, half ? (N - 1 - a) : a, L.col_c(q), y[s]);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int s = 0; s < G::OWN; ++s) v[s] = (double)y[s];
}

// FP64 5-point Laplacian (times c) of owned values v, via the LDS stencil
// buffer X (interior origin, zero halo ring).
template <int N, int NW>
__device__ __forceinline__ void lap_owned(double* X, const LaneB<N, NW>& L,
                                          const double (&v)[GeoB<N, NW>::OWN],
                                          double (&out)[GeoB<N, NW>::OWN], double c) {
  using G = GeoB<N, NW>;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < G::OWN; ++s) {
    int row, col;
    ownb_rc<N, NW>(L, s, row, col);
    X[row * G::LDX + col] = v[s];
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < G::OWN; ++s) {
    int row, col;
    ownb_rc<N, NW>(L, s, row, col);
    const double* p = X + row * G::LDX + col;
    out[s] = c * ((p[-G::LDX] + p[G::LDX]) + (p[-1] + p[1]) - 4.0 * p[0]);
  }
}

// Zero the halo ring of the FP64 stencil buffer (row -1, row N, columns -1
// and N): the stencil reads nothing else outside the interior, and the
// interior is rewritten before every stencil.
template <int N, int NW>
__device__ __forceinline__ void split_halo_zero(double* X) {
  using G = GeoB<N, NW>;
  for (int i = threadIdx.x; i < N + 2; i += G::NT) {
    X[-G::LDX - 1 + i] = 0.0;
    X[N * G::LDX - 1 + i] = 0.0;
  }
  for (int i = threadIdx.x; i < N; i += G::NT) {
    X[i * G::LDX - 1] = 0.0;
    X[i * G::LDX + N] = 0.0;
  }
}

template <int N, int NW>
__global__ void __launch_bounds__(NW * 64)
k_fine_split_2d(const WorkItem* __restrict__ items, const InstDev* __restrict__ inst,
                const double* __restrict__ Tg, const double* __restrict__ U_in,
                double* __restrict__ F_out, const uint8_t* __restrict__ mask,
                const int32_t* __restrict__ active, const int32_t* __restrict__ kmin, int in_iter) {
  using G = GeoB<N, NW>;
  extern __shared__ double smem[];
  double* X = smem + G::XOFF;            // FP64 stencil buffer (interior origin)
  __bf16* SB = (__bf16*)smem;            // BF16 transform buffer (aliases X)
  double* lamS = smem + G::XSZ;          // eigenvalues of the 1D Laplacian
  const WorkItem it = items[blockIdx.x];
  const InstDev P = inst[it.inst];
  if (mask && !mask[P.slice_base + it.slice]) return;
  if ((kmin && it.slice < *kmin) || (active && !active[it.inst])) return;
  const int64_t off = P.off_slices + (int64_t)it.slice * N * N;
  const int64_t off_in = (in_iter ? P.off_iter : P.off_slices) + (int64_t)it.slice * N * N;
  LaneB<N, NW> L;
  SineB A;
  sine_operands<N, NW>(Tg, L, A);
  const double tau = P.dt, ih2 = 1.0 / (P.h * P.h), e2 = P.eps * P.eps, s = P.s_fine;
  double u[G::OWN], t1[G::OWN], t2[G::OWN];
  for (int i = threadIdx.x; i < G::XSZ; i += G::NT) smem[i] = 0.0;
  for (int i = threadIdx.x; i < N; i += G::NT) lamS[i] = Tg[2 * (N + 1) + i];
  __syncthreads();
  for (int idx = threadIdx.x; idx < N * N; idx += G::NT)
    X[(idx / N) * G::LDX + idx % N] = U_in[off_in + idx];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < G::OWN; ++k) {
    int row, col;
    ownb_rc<N, NW>(L, k, row, col);
    u[k] = X[row * G::LDX + col];
  }
  // u and u1 are parked in the work item's scratch during the two solves so
  // that only one FP64 vector is held in registers next to the MFMA state.
  const Work W = work_vectors(P, it.slice);
  const int vo = threadIdx.x * 8;
  for (int m = 0; m < P.j_fine; ++m) {
    // defect d = tau Lap(f(u) - eps^2 Lap u)
    lap_owned<N, NW>(X, L, u, t1, ih2);
#pragma unroll
    for (int k = 0; k < G::OWN; ++k) {
      t1[k] = (P.f_zero ? 0.0 : u[k] * u[k] * u[k] - u[k]) - e2 * t1[k];
      W.x.st(k * G::NT, vo, u[k]);
    }
    lap_owned<N, NW>(X, L, t1, t2, tau * ih2);
    // delta1 = P^{-1}_lp d
    split_solve<N, NW>(SB, A, L, t2, lamS, tau, e2, s);
    // u1 = u + delta1 (t2); w = f(u) - s u + s u1 (t1)
#pragma unroll
    for (int k = 0; k < G::OWN; ++k) u[k] = W.x.ld(k * G::NT, vo);
#pragma unroll
    for (int k = 0; k < G::OWN; ++k) {
      t2[k] = u[k] + t2[k];
      W.r.st(k * G::NT, vo, t2[k]);
      t1[k] = (P.f_zero ? 0.0 : u[k] * u[k] * u[k] - u[k]) - s * u[k] + s * t2[k];
    }
    __syncthreads();
    split_halo_zero<N, NW>(X);   // the BF16 buffer overwrote part of the halo ring
    // residual r = (u - u1) + tau Lap(w - eps^2 Lap u1)
    lap_owned<N, NW>(X, L, t2, u, ih2);
#pragma unroll
    for (int k = 0; k < G::OWN; ++k) t1[k] -= e2 * u[k];
    lap_owned<N, NW>(X, L, t1, t2, tau * ih2);
#pragma unroll
    for (int k = 0; k < G::OWN; ++k)
      t2[k] += W.x.ld(k * G::NT, vo) - W.r.ld(k * G::NT, vo);
    split_solve<N, NW>(SB, A, L, t2, lamS, tau, e2, s);
#pragma unroll
    for (int k = 0; k < G::OWN; ++k) u[k] = W.r.ld(k * G::NT, vo) + t2[k];
    __syncthreads();
    split_halo_zero<N, NW>(X);   // the BF16 buffer overwrote part of the halo ring
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < G::OWN; ++k) {
    int row, col;
    ownb_rc<N, NW>(L, k, row, col);
    X[row * G::LDX + col] = u[k];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < N * N; idx += G::NT)
    F_out[off + idx] = X[(idx / N) * G::LDX + idx % N];
}

template <int N, int NW>
static hipError_t split2d(const WorkItem* items, int n_items, const InstDev* inst, const double* Tg,
                          const double* U_in, double* F_out, const uint8_t* mask,
                          const int32_t* active, const int32_t* kmin, int in_iter, hipStream_t s) {
  const size_t lds = ((size_t)GeoB<N, NW>::XSZ + N) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_fine_split_2d<N, NW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fine_split_2d<N, NW>), dim3(n_items), dim3(NW * 64), lds, s, items, inst,
                     Tg, U_in, F_out, mask, active, kmin, in_iter);
  return hipGetLastError();
}

hipError_t launch_fine_split_2d(int n, const WorkItem* items, int n_items, const InstDev* inst,
                                const double* Tg, const double* U_in, double* F_out,
                                const uint8_t* mask, const int32_t* active, const int32_t* kmin, int in_iter,
                                hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  switch (n) {
    case 64: return split2d<64, 4>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s);
    case 128: return split2d<128, 8>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------- 1D
// One workgroup per state, NT = n rounded up to 64 threads; thread i < n
// owns grid point i (state) and sine index i (spectral), the others hold
// zeros.  S (n x n) is staged in LDS.  Any n <= 128.
struct Ctx1 {
  const double* Sl;   // S in LDS, S[k][i] at k * n + i
  double* buf;        // n values
  double* red;        // 64 partials
  int n, i;
  bool on;            // i < n
  double* dl;         // scratch of the direct (2.4) solve
};

// (S v)_i, v given per thread (zero off the grid)
__device__ __forceinline__ double sine1(const Ctx1& c, double v) {
  __syncthreads();
  if (c.on) c.buf[c.i] = v;
  __syncthreads();
  double acc = 0.0;
  if (c.on)
    for (int k = 0; k < c.n; ++k) acc += c.Sl[k * c.n + c.i] * c.buf[k];
  return acc;
}

// Deterministic block sum (fixed wave order); every thread gets the sum.
__device__ __forceinline__ double bsum1(const Ctx1& c, double v) {
  v = wave_sum<1>(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) c.red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int ww = 0; ww < nw; ++ww) s += c.red[ww];
  return s;
}

// (min + max)/2 over the grid points of a per-thread value
__device__ __forceinline__ double bmid1(const Ctx1& c, double v) {
  double mn = c.on ? v : 1e300, mx = c.on ? v : -1e300;
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o, 64));
    mx = fmax(mx, __shfl_xor(mx, o, 64));
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) { c.red[w] = mn; c.red[32 + w] = mx; }
  __syncthreads();
  mn = c.red[0]; mx = c.red[32];
  for (int ww = 1; ww < nw; ++ww) { mn = fmin(mn, c.red[ww]); mx = fmax(mx, c.red[32 + ww]); }
  return 0.5 * (mn + mx);
}

// u + c * Lap_h-stencil(w) * h^2 with zero ghosts: the right-hand side form
// u + tau Lap_h w (c = tau / h^2)
__device__ __forceinline__ double lap_rhs1(const Ctx1& c, double u, double w, double coef) {
  __syncthreads();
  if (c.on) c.buf[c.i] = w;
  __syncthreads();
  if (!c.on) return 0.0;
  const double wl = c.i > 0 ? c.buf[c.i - 1] : 0.0, wr = c.i < c.n - 1 ? c.buf[c.i + 1] : 0.0;
  return u + coef * ((wl + wr) - 2.0 * w);
}

// ------------------------------------------ 1D subdomain solves of (2.4)
// Scheme (2.4) in mixed form, [I, -tau L; eps^2 L - diag(c), I][u; v] =
// [u_n; f_v] with c = u_n^2 and f_v = -u_n (f == 0: c = 0, f_v = 0), on N0
// equal subdomains (Section 4).  Nodes 0..n+1, interfaces at p_q = q m,
// m = (n+1)/N0.  Per node the unknowns form a 2-vector (u, v); the matrix is
// block tridiagonal with the coupling E = [[0, -a], [b, 0]] (a = tau/h^2,
// b = eps^2/h^2) to both neighbours and the diagonal block
// [[w, e a], [-e b - w c_j, w]]: w = 1, e = 2 inside (and next to the
// physical boundary), w = 1/2, e = 1 at an interface node of a Neumann
// problem (half of the shared node, one edge of the subdomain).
//
// The subdomain matrices are factored once per step (block Thomas, 2x2
// pivots).  The Dirichlet solution of a subdomain is an affine function of
// its four trace values (its responses to the data and to a unit value of
// each trace), and the Neumann solution at an interface is linear in the
// subdomain's interface residuals (its responses to unit residuals).  Two
// uses:
//  * the Neumann-Neumann iteration of Section 4 (dd1_step) runs on the
//    interface traces, one lane per interface: each iteration computes the
//    residuals, the Neumann corrections and the trace update for all
//    interfaces at once; the iterates are the method's own (up to rounding);
//  * the direct solve (dd1_direct_step) eliminates the interface equations
//    themselves (block tridiagonal in the traces) on one lane: a
//    substructured elimination of the whole system.
// Both end with the subdomain states of the final traces.
struct DD1 {
  int n, N0, m, MD, MN;
  double a, b;
  double fvs;   // f_v = fvs u_n
  bool cz;      // c = 0
  double *ub, *fD, *fN, *rD, *tN, *nr, *ib, *tg, *th;
};

// nn: with the Neumann parts (else they take no space and ib holds the
// interface blocks of the direct solve)
__device__ __forceinline__ DD1 dd1_layout(const InstDev& P, int N0, double tau, double* L,
                                          bool nn) {
  DD1 d;
  d.n = P.n; d.N0 = N0; d.m = (P.n + 1) / N0; d.MD = d.m - 1; d.MN = nn ? d.m + 1 : 0;
  d.a = tau / (P.h * P.h); d.b = P.eps * P.eps / (P.h * P.h);
  d.fvs = P.f_zero ? 0.0 : -1.0;
  d.cz = P.f_zero != 0;
  d.ub = L;                                 // u_n on nodes 0..n+1
  d.fD = d.ub + d.n + 2;                    // Dirichlet pivots: N0 x MD x 4
  d.fN = d.fD + N0 * d.MD * 4;              // Neumann pivots:   N0 x MN x 4
  d.rD = d.fN + N0 * d.MN * 4;              // Dirichlet responses: N0 x 5 x MD x 2
  d.tN = d.rD + N0 * 5 * d.MD * 2;          // Neumann solves: N0 x 4 x MN x 2
  d.nr = d.tN + N0 * 4 * d.MN * 2;          // Neumann interface responses: N0 x 4 x 4
  d.ib = d.nr + (nn ? N0 * 16 : 0);         // direct: interface blocks, 14 per interface
  d.tg = d.ib + (nn ? 0 : 14 * (N0 + 1));   // traces g_q, q = 0..N0 (ends 0)
  d.th = d.tg + N0 + 1;                     // traces h_q
  return d;
}

// LDS doubles of the Neumann-Neumann layout for n (any N0 with m >= 2)
__host__ __device__ constexpr size_t dd1_lds_doubles(int n) {
  return (size_t)(n + 2) + 26 * (size_t)(n + 1) + 18 * (size_t)((n + 1) / 2) + 2 + 64;
}
// ... and of the direct layout (any N0 <= 64 with m >= 2, or N0 = 1)
__host__ __device__ constexpr size_t direct1_lds_doubles(int n) {
  return (size_t)(n + 2) + 14 * (size_t)(n + 1) + 16 * 65 + 64;
}

// 1/x by Newton's iteration r <- r (2 - x r) from the hardware estimate,
// twice (each step squares the relative error): a shorter dependent chain
// than a correctly rounded division, accurate to an ulp or so.
__device__ __forceinline__ double dd1_recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// Block Thomas over M nodes with pivots F (inverse 2x2 blocks, row-major) and
// the coupling E: X holds d on entry and the solution on exit.  The next
// node's operands are loaded before the current node's results are stored,
// so the chain does not wait for the stores.
__device__ void dd1_solve(const DD1& d, const double* F, double* X, int M) {
  // the running y_k stays in registers (no LDS round trip on the chain)
  double y0 = X[0], y1 = X[1];
  double q0 = 0, q1 = 0, q2 = 0, q3 = 0, n0 = 0, n1 = 0;
  if (M > 1) { q0 = F[0]; q1 = F[1]; q2 = F[2]; q3 = F[3]; n0 = X[2]; n1 = X[3]; }
  for (int k = 1; k < M; ++k) {
    // y_k = d_k - E Binv_{k-1} y_{k-1}
    const double p0 = q0, p1 = q1, p2 = q2, p3 = q3, d0 = n0, d1 = n1;
    if (k + 1 < M) {
      q0 = F[4 * k]; q1 = F[4 * k + 1]; q2 = F[4 * k + 2]; q3 = F[4 * k + 3];
      n0 = X[2 * k + 2]; n1 = X[2 * k + 3];
    }
    const double t0 = p2 * y0 + p3 * y1, t1 = p0 * y0 + p1 * y1;
    y0 = d0 + d.a * t0;
    y1 = d1 - d.b * t1;
    X[2 * k] = y0;
    X[2 * k + 1] = y1;
  }
  const double* p = F + (M - 1) * 4;
  double x0 = p[0] * y0 + p[1] * y1;
  double x1 = p[2] * y0 + p[3] * y1;
  if (M > 1) {
    q0 = F[4 * (M - 2)]; q1 = F[4 * (M - 2) + 1]; q2 = F[4 * (M - 2) + 2]; q3 = F[4 * (M - 2) + 3];
    n0 = X[2 * (M - 2)]; n1 = X[2 * (M - 2) + 1];
  }
  X[2 * M - 2] = x0; X[2 * M - 1] = x1;
  for (int k = M - 2; k >= 0; --k) {
    // x_k = Binv_k (y_k - E x_{k+1}),  E x = (-a x1, b x0)
    const double p0 = q0, p1 = q1, p2 = q2, p3 = q3;
    const double r0 = n0 + d.a * x1, r1 = n1 - d.b * x0;
    if (k > 0) {
      q0 = F[4 * (k - 1)]; q1 = F[4 * (k - 1) + 1]; q2 = F[4 * (k - 1) + 2]; q3 = F[4 * (k - 1) + 3];
      n0 = X[2 * (k - 1)]; n1 = X[2 * (k - 1) + 1];
    }
    x0 = p0 * r0 + p1 * r1;
    x1 = p2 * r0 + p3 * r1;
    X[2 * k] = x0; X[2 * k + 1] = x1;
  }
}

// Factor one subdomain problem: nodes lo..hi, pivots to F; il, ir: lo, hi
// are interface nodes of a Neumann problem.
__device__ void dd1_factor(const DD1& d, double* F, int lo, int hi, bool il, bool ir) {
  double p0 = 0, p1 = 0, p2 = 0, p3 = 0;
  double un = d.ub[lo];                       // next node's u_n, loaded ahead
  for (int j = lo; j <= hi; ++j) {
    const double uj = un;
    if (j < hi) un = d.ub[j + 1];
    const bool iface = (j == lo && il) || (j == hi && ir);
    const double w = iface ? 0.5 : 1.0, e = iface ? 1.0 : 2.0;
    const double cj = d.cz ? 0.0 : uj * uj;
    double B0 = w, B1 = e * d.a, B2 = -e * d.b - w * cj, B3 = w;
    if (j > lo) {
      // B -= (E Binv_prev) E;  E Binv = [[-a p2, -a p3], [b p0, b p1]]
      const double W0 = -d.a * p2, W1 = -d.a * p3, W2 = d.b * p0, W3 = d.b * p1;
      B0 -= d.b * W1; B1 += d.a * W0; B2 -= d.b * W3; B3 += d.a * W2;
    }
    const double id = dd1_recip(B0 * B3 - B1 * B2);
    p0 = B3 * id; p1 = -B1 * id; p2 = -B2 * id; p3 = B0 * id;
    double* q = F + (j - lo) * 4;
    q[0] = p0; q[1] = p1; q[2] = p2; q[3] = p3;
  }
}

// Stage u_n (the thread's node value u, node tid + 1), factor the subdomain
// problems and solve for the responses.
__device__ void dd1_prepare(const DD1& d, double u, bool nn) {
  const int tid = threadIdx.x, N0 = d.N0, m = d.m, MD = d.MD, MN = d.MN, n = d.n;
  __syncthreads();   // the previous step's readers are done
  if (tid < n) d.ub[tid + 1] = u;
  if (tid == 0) { d.ub[0] = 0.0; d.ub[n + 1] = 0.0; }
  __syncthreads();
  // Dirichlet work on the first wave, Neumann work on the second: the two
  // run side by side instead of one after the other in a divergent wave
  const int w = tid >> 6, l = tid & 63;
  const bool neu = nn && N0 > 1 && w == 1;
  if (w == 0 || neu)
    for (int i = l; i < N0; i += 64) {
      if (!neu) dd1_factor(d, d.fD + i * MD * 4, i * m + 1, (i + 1) * m - 1, false, false);
      else dd1_factor(d, d.fN + i * MN * 4, max(i * m, 1), min((i + 1) * m, n), i > 0, i < N0 - 1);
    }
  __syncthreads();
  const int nd = 5 * N0;
  for (int t = w == 0 ? l : (neu ? nd + l : 9 * N0); t < (w == 0 ? nd : 9 * N0); t += 64) {
    if (t < nd) {
      // Dirichlet responses of subdomain i: 0 = to the data (traces zero),
      // 1..4 = to a unit g, h of the left interface, g, h of the right one
      const int i = t / 5, k = t % 5;
      double* X = d.rD + (i * 5 + k) * MD * 2;
      const int lo = i * m + 1;
      for (int j = 0; j < MD; ++j) {
        X[2 * j] = k == 0 ? d.ub[lo + j] : 0.0;
        X[2 * j + 1] = k == 0 ? d.fvs * d.ub[lo + j] : 0.0;
      }
      if ((i == 0 && (k == 1 || k == 2)) || (i == N0 - 1 && (k == 3 || k == 4))) continue;
      // the coupling -E (g, h) of a trace moves to the right-hand side: (a h, -b g)
      const int at = k <= 2 ? 0 : MD - 1;
      if (k == 1 || k == 3) X[2 * at + 1] = -d.b;
      if (k == 2 || k == 4) X[2 * at] = d.a;
      dd1_solve(d, d.fD + i * MD * 4, X, MD);
    } else {
      // Neumann responses of subdomain i to a unit residual: 0, 1 = u, v rows
      // of its left interface node, 2, 3 = of its right one; kept at both ends
      const int i = (t - nd) / 4, e = (t - nd) % 4;
      double* out = d.nr + (i * 4 + e) * 4;
      if (N0 == 1 || (i == 0 && e < 2) || (i == N0 - 1 && e >= 2)) {
        out[0] = out[1] = out[2] = out[3] = 0.0;
        continue;
      }
      const int lo = max(i * m, 1), M = min((i + 1) * m, n) - lo + 1;
      double* X = d.tN + (i * 4 + e) * MN * 2;
      for (int j = 0; j < 2 * M; ++j) X[j] = 0.0;
      X[(e < 2 ? 0 : 2 * (M - 1)) + (e & 1)] = 1.0;
      dd1_solve(d, d.fN + i * MN * 4, X, M);
      out[0] = X[0]; out[1] = X[1]; out[2] = X[2 * M - 2]; out[3] = X[2 * M - 1];
    }
  }
  __syncthreads();
}

// Dirichlet responses next to interface q (1..N0-1): RL of the left
// subdomain's last interior node, RR of the right one's first (u, v each).
__device__ __forceinline__ void dd1_near(const DD1& d, int q, double (&RL)[5][2],
                                         double (&RR)[5][2]) {
  for (int k = 0; k < 5; ++k)
    for (int s = 0; s < 2; ++s) {
      RL[k][s] = d.rD[(((q - 1) * 5 + k) * d.MD + d.MD - 1) * 2 + s];
      RR[k][s] = d.rD[((q * 5 + k) * d.MD) * 2 + s];
    }
}

// The step's result at the thread's node from the traces tg, th.
__device__ __forceinline__ double dd1_result(const DD1& d) {
  const int tid = threadIdx.x;
  if (tid >= d.n) return 0.0;
  const int j = tid + 1, i = j / d.m;
  if (j % d.m == 0) return d.tg[i];
  const int k = j - i * d.m - 1;
  const double c[5] = {1.0, d.tg[i], d.th[i], d.tg[i + 1], d.th[i + 1]};
  double v = 0.0;
  for (int r = 0; r < 5; ++r) v += c[r] * d.rD[((i * 5 + r) * d.MD + k) * 2];
  return v;
}

// Cross-lane moves of the interface iteration: the neighbours' values (lane
// q - 1 and q + 1, zero past the ends) and the maximum over the lanes holding
// interfaces, broadcast to every lane.  With N0 <= 16 the interfaces sit in
// the first row of 16 lanes and the moves are DPP row shifts (no round trip
// through the LDS crossbar); else cross-lane shuffles.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <bool DPP>
__device__ __forceinline__ double dd1_left(double v, int q) {
  if constexpr (DPP) return dpp_f64<0x111>(v);     // row_shr:1
  else return __shfl(v, (q + 63) & 63, 64);
}
template <bool DPP>
__device__ __forceinline__ double dd1_right(double v, int q) {
  if constexpr (DPP) return dpp_f64<0x101>(v);     // row_shl:1
  else return __shfl(v, (q + 1) & 63, 64);
}
// v >= 0 on every lane (zero off the interfaces)
template <bool DPP>
__device__ __forceinline__ double dd1_max(double v, int N0) {
  if constexpr (DPP) {
    // prefix maxima along row 0 by zero-filled shifts: lane 15 ends with the row's
    v = fmax(v, dpp_f64<0x111>(v));
    v = fmax(v, dpp_f64<0x112>(v));
    v = fmax(v, dpp_f64<0x114>(v));
    v = fmax(v, dpp_f64<0x118>(v));
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 15),
                            __builtin_amdgcn_readlane(__double2loint(v), 15));
  } else {
    int W = 1;                            // power of two >= N0 (<= 64)
    while (W < N0) W <<= 1;
    for (int o = 1; o < W; o <<= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return __shfl(v, 0, 64);
  }
}

// The Neumann-Neumann iteration on the traces (g, h) of interface q, one lane
// each (wave 0; the other lanes carry zeros).  Returns the iterations.
template <bool DPP>
__device__ __forceinline__ int dd1_iterate(const DD1& d, const InstDev& P, int q, bool on,
                                           double up, double cp, double& g, double& h,
                                           const double (&RL)[5][2], const double (&RR)[5][2],
                                           const double (&NL)[4][2], const double (&NRt)[4][2],
                                           int& status) {
  const double th = P.dd_theta;
  int it = 0;
  while (d.N0 > 1) {
    // Dirichlet states next to the interface from the current traces
    const double gl = dd1_left<DPP>(g, q), hl = dd1_left<DPP>(h, q);
    const double gr = dd1_right<DPP>(g, q), hr = dd1_right<DPP>(h, q);
    double Lv[2], Rv[2];
    for (int s = 0; s < 2; ++s) {
      Lv[s] = RL[0][s] + gl * RL[1][s] + hl * RL[2][s] + g * RL[3][s] + h * RL[4][s];
      Rv[s] = RR[0][s] + g * RR[1][s] + h * RR[2][s] + gr * RR[3][s] + hr * RR[4][s];
    }
    // residual of the global equations at p_q: the jump of the Neumann traces
    double ru = up - (g - d.a * (Lv[1] - 2.0 * h + Rv[1]));
    double rv = d.fvs * up - (d.b * (Lv[0] - 2.0 * g + Rv[0]) - cp * g + h);
    if (!on) ru = rv = 0.0;
    const double rul = dd1_left<DPP>(ru, q), rvl = dd1_left<DPP>(rv, q);
    const double rur = dd1_right<DPP>(ru, q), rvr = dd1_right<DPP>(rv, q);
    // Neumann corrections of both neighbours at p_q, relaxed by theta
    double dg = 0.0, dh = 0.0;
    if (on) {
      dg = th * (NL[0][0] * rul + NL[1][0] * rvl + NL[2][0] * ru + NL[3][0] * rv +
                 NRt[0][0] * ru + NRt[1][0] * rv + NRt[2][0] * rur + NRt[3][0] * rvr);
      dh = th * (NL[0][1] * rul + NL[1][1] * rvl + NL[2][1] * ru + NL[3][1] * rv +
                 NRt[0][1] * ru + NRt[1][1] * rv + NRt[2][1] * rur + NRt[3][1] * rvr);
    }
    g += dg;
    h += dh;
    ++it;
    // max over the interfaces of max(|dg|, |dh|) (both traces meet the
    // tolerance iff it does; a non-finite change counts as infinite)
    const double mx =
        dd1_max<DPP>((dg == dg && dh == dh) ? fmax(fabs(dg), fabs(dh)) : INFINITY, d.N0);
    if (!(mx < INFINITY)) { status |= 1; break; }
    if (mx <= P.dd_tol) break;
    if (it >= P.dd_max) { status |= 1; break; }
  }
  return it;
}

// One Neumann-Neumann step (2.4) of the thread's node value u; iters counts
// the iterations, status bit 1 flags the cap or a non-finite update.
__device__ double dd1_step(double u, const InstDev& P, double tau, double* L, int& iters,
                           int& status) {
  const DD1 d = dd1_layout(P, P.dd_sub, tau, L, true);
  const int tid = threadIdx.x, N0 = d.N0, m = d.m;
  dd1_prepare(d, u, true);
  if (tid < 64) {
    // lane q: interface q (1..N0-1); the other lanes carry zeros
    const int q = tid;
    const bool on = q >= 1 && q < N0;
    double g = 0.0, h = 0.0, up = 0.0, cp = 0.0;
    double RL[5][2], RR[5][2], NL[4][2], NRt[4][2];
    if (on) {
      const int p = q * m;
      up = d.ub[p];
      cp = d.cz ? 0.0 : up * up;
      // initial traces: the mixed variables of u_n (v = -eps^2 Lap u + c u + f_v)
      g = up;
      h = -d.b * (d.ub[p - 1] - 2.0 * up + d.ub[p + 1]) + cp * up + d.fvs * up;
      dd1_near(d, q, RL, RR);
      for (int e = 0; e < 4; ++e)
        for (int s = 0; s < 2; ++s) {
          NL[e][s] = d.nr[((q - 1) * 4 + e) * 4 + 2 + s];
          NRt[e][s] = d.nr[(q * 4 + e) * 4 + s];
        }
    } else {
      for (int k = 0; k < 5; ++k) RL[k][0] = RL[k][1] = RR[k][0] = RR[k][1] = 0.0;
      for (int e = 0; e < 4; ++e) NL[e][0] = NL[e][1] = NRt[e][0] = NRt[e][1] = 0.0;
    }
    const int it = N0 <= 16 ? dd1_iterate<true>(d, P, q, on, up, cp, g, h, RL, RR, NL, NRt, status)
                            : dd1_iterate<false>(d, P, q, on, up, cp, g, h, RL, RR, NL, NRt, status);
    iters += it;
    if (on) { d.tg[q] = g; d.th[q] = h; }
    if (tid == 0) { d.tg[0] = d.th[0] = d.tg[N0] = d.th[N0] = 0.0; }
  }
  __syncthreads();
  return dd1_result(d);
}

// 2x2 helpers (row-major)
__device__ __forceinline__ void m2_inv(const double* A, double* R) {
  const double id = 1.0 / (A[0] * A[3] - A[1] * A[2]);
  const double r0 = A[3] * id, r1 = -A[1] * id, r2 = -A[2] * id, r3 = A[0] * id;
  R[0] = r0; R[1] = r1; R[2] = r2; R[3] = r3;
}
__device__ __forceinline__ void m2_mul(const double* A, const double* B, double* R) {
  const double r0 = A[0] * B[0] + A[1] * B[2], r1 = A[0] * B[1] + A[1] * B[3];
  const double r2 = A[2] * B[0] + A[3] * B[2], r3 = A[2] * B[1] + A[3] * B[3];
  R[0] = r0; R[1] = r1; R[2] = r2; R[3] = r3;
}

// One (2.4) step solved directly by substructuring on P.direct_sub equal
// subdomains: the global equations at the interface nodes, written with the
// subdomains' responses, are block tridiagonal in the traces x_q = (g_q, h_q):
// A_q x_{q-1} + B_q x_q + C_q x_{q+1} = D_q.  One lane per interface forms
// its blocks, one lane eliminates them (block Thomas), then every node takes
// its subdomain's state.
__device__ double dd1_direct_step(double u, const InstDev& P, double tau, double* L) {
  const DD1 d = dd1_layout(P, P.direct_sub, tau, L, false);
  const int tid = threadIdx.x, N0 = d.N0;
  dd1_prepare(d, u, false);
  const int q = tid;
  if (q >= 1 && q < N0) {
    double RL[5][2], RR[5][2];
    dd1_near(d, q, RL, RR);
    const double up = d.ub[q * d.m], cp = d.cz ? 0.0 : up * up;
    const double a = d.a, b = d.b;
    // r_u = f_u - [g - a (v_L - 2 h + v_R)], r_v = f_v - [b (u_L - 2 g + u_R)
    // - c g + h], with (u, v)_L, (u, v)_R affine in the traces; r = 0
    double* e = d.ib + 14 * q;       // A (4), B (4), C (4), D (2)
    e[0] = a * RL[1][1];  e[1] = a * RL[2][1];  e[2] = -b * RL[1][0];  e[3] = -b * RL[2][0];
    e[4] = -1.0 + a * (RL[3][1] + RR[1][1]);
    e[5] = a * (RL[4][1] + RR[2][1] - 2.0);
    e[6] = -b * (RL[3][0] + RR[1][0] - 2.0) + cp;
    e[7] = -b * (RL[4][0] + RR[2][0]) - 1.0;
    e[8] = a * RR[3][1];  e[9] = a * RR[4][1];  e[10] = -b * RR[3][0];  e[11] = -b * RR[4][0];
    e[12] = -(up + a * (RL[0][1] + RR[0][1]));
    e[13] = -(d.fvs * up - b * (RL[0][0] + RR[0][0]));
  }
  __syncthreads();
  if (tid == 0) {
    // forward: B'_q = B_q - A_q B'^-1_{q-1} C_{q-1}, D'_q = D_q - A_q B'^-1_{q-1} D'_{q-1}
    // (B'^-1 kept in place of B, D' in place of D)
    for (int k = 1; k < N0; ++k) {
      double* e = d.ib + 14 * k;
      if (k > 1) {
        const double* f = d.ib + 14 * (k - 1);
        double W[4], WC[4];
        m2_mul(e, f + 4, W);          // A_q B'^-1_{q-1}
        m2_mul(W, f + 8, WC);
        for (int r = 0; r < 4; ++r) e[4 + r] -= WC[r];
        e[12] -= W[0] * f[12] + W[1] * f[13];
        e[13] -= W[2] * f[12] + W[3] * f[13];
      }
      m2_inv(e + 4, e + 4);
    }
    double xg = 0.0, xh = 0.0;
    for (int k = N0 - 1; k >= 1; --k) {
      const double* e = d.ib + 14 * k;
      const double r0 = e[12] - (e[8] * xg + e[9] * xh), r1 = e[13] - (e[10] * xg + e[11] * xh);
      xg = e[4] * r0 + e[5] * r1;
      xh = e[6] * r0 + e[7] * r1;
      d.tg[k] = xg;
      d.th[k] = xh;
    }
    d.tg[0] = d.th[0] = d.tg[N0] = d.th[N0] = 0.0;
  }
  __syncthreads();
  return dd1_result(d);
}

// Fine propagator of one work item with the Neumann-Neumann step: J steps;
// the iterations of the J steps go to iters[2 slice].
__global__ void __launch_bounds__(128)
k_fine_dd_1d(const WorkItem* __restrict__ items, const InstDev* __restrict__ inst,
             const double* __restrict__ U_in, double* __restrict__ F_out,
             const uint8_t* __restrict__ mask, const int32_t* __restrict__ active,
             const int32_t* __restrict__ kmin, int in_iter) {
  extern __shared__ double smem[];
  const WorkItem it = items[blockIdx.x];
  const InstDev P = inst[it.inst];
  if (mask && !mask[P.slice_base + it.slice]) return;
  if ((kmin && it.slice < *kmin) || (active && !active[it.inst])) return;
  const int n = P.n;
  const int64_t in0 = (in_iter ? P.off_iter : P.off_slices) + (int64_t)it.slice * n;
  double u = (int)threadIdx.x < n ? U_in[in0 + threadIdx.x] : 0.0;
  int status = 0, iters = 0;
  for (int s = 0; s < P.j_fine; ++s) u = dd1_step(u, P, P.dt, smem, iters, status);
  if ((int)threadIdx.x < n) F_out[P.off_slices + (int64_t)it.slice * n + threadIdx.x] = u;
  if (threadIdx.x == 0) {
    P.iters[2 * it.slice] = iters;
    P.iters[2 * it.slice + 1] = 0;
    if (status) atomicOr(P.status, status);
  }
}

// Scheme (2.4) steps of tau solved directly (dd1_direct_step); the chains
// are the subdomains' m-node eliminations and the N0-long interface
// elimination instead of one 2n-pivot elimination, and far shorter than the
// transforms and reductions of CG iterations in the sine basis.
__device__ double approx2_direct1(const Ctx1& c, double u, const InstDev& P, double tau,
                                  int steps) {
  for (int m = 0; m < steps; ++m) u = dd1_direct_step(u, P, tau, c.dl);
  return u;
}

// Linear stabilised steps: (I + tau eps^2 L^2 - s tau L) v = u + tau L (f(u) - s u),
// diagonal on the sine modes with 1 / sigma = rsig[i].
__device__ double stab1(const Ctx1& c, double u, const InstDev& P, double tau, int steps,
                        const double* rsig) {
  const double coef = tau / (P.h * P.h), s = P.s_fine;
  const double rs = c.on ? rsig[c.i] : 0.0;
  for (int m = 0; m < steps; ++m) {
    const double w = P.f_zero ? (-s * u) : (u * u * u - (1.0 + s) * u);
    const double r = lap_rhs1(c, u, w, coef);
    u = sine1(c, sine1(c, r) * rs);
  }
  return u;
}

// PCG in sine coordinates for K x = b, K = diag(d) + tau S diag(q) S (SPD),
// preconditioner 1 / (d + tau cshift), from x = 0, stopped when
// ||r|| <= rtol ||b||.  Returns false on the cap or a non-finite residual.
__device__ bool cg1(const Ctx1& c, double b, double d, double q, double tau, double cshift,
                    double rtol, int maxit, double& x) {
  const double mi = c.on ? 1.0 / (d + tau * cshift) : 0.0;
  x = 0.0;
  double r = b, p = b * mi;
  double rz = bsum1(c, r * p);
  const double bb = bsum1(c, b * b);
  if (!(bb > 0.0)) return true;
  const double stop2 = rtol * rtol * bb;
  for (int it = 1; it <= maxit; ++it) {
    const double kp = d * p + tau * sine1(c, q * sine1(c, p));
    const double alpha = rz / bsum1(c, p * kp);
    x += alpha * p;
    r -= alpha * kp;
    const double rr = bsum1(c, r * r);
    const double rzn = bsum1(c, r * (r * mi));
    if (rr <= stop2) return true;
    if (!(rr == rr)) return false;
    p = r * mi + (rzn / rz) * p;
    rz = rzn;
  }
  return false;
}

// Scheme (2.3) (be = false) or backward Euler (true) with step tau, by
// Newton's method from Y_0 = u in sine coordinates (as newton_step in 2D):
// A^{-1} H(Y) = d Yh + tau S(Y^3) - (1/mu + tau) uh (2.3) or
// d Yh + tau S(Y^3) - tau Yh - uh/mu (BE), the Newton matrix
// diag(d) + tau S diag(q) S with q = 3Y^2 (2.3) or 3Y^2 - 1 (BE); stop when
// ||Y_{m+1} - Y_m||_h <= newton_tol.  Returns the new state.
__device__ double newton1(const Ctx1& c, double u, const InstDev& P, const double* lam,
                          double tau, bool be, int& status) {
  const double mu = c.on ? -lam[c.i] : 1.0;
  const double im = c.on ? 1.0 / mu : 0.0;
  const double d = im + tau * P.eps * P.eps * mu;
  const double uh = sine1(c, u);
  double yh = uh;
  bool conv = false;
  for (int it = 0; it < P.newton_max; ++it) {
    const double y = sine1(c, yh);
    const double q = (P.f_zero || !c.on) ? 0.0 : 3.0 * y * y + (be ? -1.0 : 0.0);
    const double cs = bmid1(c, q);
    const double y3h = sine1(c, P.f_zero ? 0.0 : y * y * y);
    double g;
    if (P.f_zero) g = d * yh - im * uh;
    else if (be) g = d * yh + tau * y3h - tau * yh - im * uh;
    else g = d * yh + tau * y3h - (im + tau) * uh;
    if (!c.on) g = 0.0;
    double dx;
    if (!cg1(c, -g, d, q, tau, cs, P.nl_krylov_rtol, P.krylov_max, dx)) status |= 1;
    yh += dx;
    const double step = sqrt(P.h * bsum1(c, dx * dx));   // ||S dYh||_h = sqrt(h) ||dYh||
    if (step <= P.newton_tol) { conv = true; break; }
    if (!(step == step)) break;
  }
  if (!conv) status |= 1;
  return sine1(c, yh);
}

// Fine propagator of one work item: J steps of the instance's fine scheme.
__global__ void k_fine_1d(const WorkItem* __restrict__ items, const InstDev* __restrict__ inst,
                          const double* __restrict__ S, const double* __restrict__ lam,
                          const double* __restrict__ U_in, double* __restrict__ F_out,
                          const uint8_t* __restrict__ mask, const int32_t* __restrict__ active,
                          const int32_t* __restrict__ kmin, int in_iter) {
  extern __shared__ double smem[];
  const WorkItem it = items[blockIdx.x];
  const InstDev P = inst[it.inst];
  if (mask && !mask[P.slice_base + it.slice]) return;
  if ((kmin && it.slice < *kmin) || (active && !active[it.inst])) return;
  const int n = P.n;
  // the direct (2.4) solve needs no sine matrix: its launch holds none
  const int so = P.fine_kind != 2 ? n * n : 0;
  Ctx1 c{smem, smem + so, smem + so + n, n, (int)threadIdx.x, (int)threadIdx.x < n,
         smem + so + n + 64};
  if (so)
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) smem[idx] = S[idx];
  const int64_t in0 = (in_iter ? P.off_iter : P.off_slices) + (int64_t)it.slice * n;
  double u = c.on ? U_in[in0 + c.i] : 0.0;
  int status = 0;
  if (P.fine_kind == 0) {
    u = stab1(c, u, P, P.dt, P.j_fine, P.rsig_fine);
  } else if (P.fine_kind == 2) {
    u = approx2_direct1(c, u, P, P.dt, P.j_fine);
  } else {
    for (int m = 0; m < P.j_fine; ++m) u = newton1(c, u, P, lam, P.dt, P.nl_variant == 1, status);
  }
  if (c.on) F_out[P.off_slices + (int64_t)it.slice * n + c.i] = u;
  if (status && threadIdx.x == 0) atomicOr(P.status, status);
}

// One coarse propagation: m_coarse steps of tau = dT/m_coarse of the
// instance's coarse scheme.
__device__ double coarse_apply_1d(const Ctx1& c, double u, const InstDev& P, const double* lam,
                                  int& status) {
  const double tau = P.dT / P.m_coarse;
  if (P.coarse_kind == 1) return stab1(c, u, P, tau, P.m_coarse, P.rsig_stab);
  if (P.coarse_kind == 3) {
    for (int m = 0; m < P.m_coarse; ++m) u = newton1(c, u, P, lam, tau, false, status);
    return u;
  }
  return approx2_direct1(c, u, P, tau, P.m_coarse);
}

__global__ void k_coarse_1d(int mode, const int32_t* __restrict__ insts,
                            const WorkItem* __restrict__ items, const InstDev* __restrict__ inst,
                            const double* __restrict__ S, const double* __restrict__ lam,
                            const double* __restrict__ U_in, double* __restrict__ G_out,
                            const uint8_t* __restrict__ mask, double* U,
                            const double* __restrict__ F, double* G_old, double* delta,
                            int32_t* status_out, const int32_t* __restrict__ active, int k,
                            const int32_t* __restrict__ kdev) {
  extern __shared__ double smem[];
  if (kdev) k = *kdev;
  int status = 0;
  const bool par = mode == 0;
  const WorkItem it = par ? items[blockIdx.x] : WorkItem{insts[blockIdx.x], 0};
  const int ii = it.inst;
  const InstDev P = inst[ii];
  if (par && mask && !mask[P.slice_base + it.slice]) return;
  if (!par && active && !active[ii]) return;
  const int n = P.n;
  Ctx1 c{smem, smem + n * n, smem + n * n + n, n, (int)threadIdx.x, (int)threadIdx.x < n,
         smem + n * n + n + 64};
  if (P.coarse_kind != 0)   // the direct (2.4) solve needs no sine matrix
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) smem[idx] = S[idx];
  const int i = c.i;
  if (par) {
    const int64_t off = P.off_slices + (int64_t)it.slice * n;
    const double g = coarse_apply_1d(c, c.on ? U_in[off + i] : 0.0, P, lam, status);
    if (c.on) G_out[off + i] = g;
    if (status && threadIdx.x == 0) atomicOr(P.status, status);
    return;
  }
  double* Ui = U + P.off_iter;
  const double* Fi = F + P.off_slices;
  double* Gi = G_old + P.off_slices;
  if (mode == 1) {
    double u = c.on ? Ui[i] : 0.0;
    for (int s = 0; s < P.n_slices; ++s) {
      u = coarse_apply_1d(c, u, P, lam, status);
      if (c.on) {
        Ui[(s + 1) * n + i] = u;
        Gi[s * n + i] = u;
      }
    }
    if (threadIdx.x == 0) status_out[ii] = status | *P.status;
    return;
  }
  if (k >= P.n_slices) {
    if (threadIdx.x == 0) delta[ii] = 0.0;
    return;
  }
  double u = c.on ? Fi[k * n + i] : 0.0;
  double dd = c.on ? u - Ui[(k + 1) * n + i] : 0.0;
  double dmax = bsum1(c, dd * dd);
  if (c.on) Ui[(k + 1) * n + i] = u;
  for (int s = k + 1; s < P.n_slices; ++s) {
    const double g = coarse_apply_1d(c, u, P, lam, status);
    const double un = c.on ? Fi[s * n + i] + (g - Gi[s * n + i]) : 0.0;
    dd = c.on ? un - Ui[(s + 1) * n + i] : 0.0;
    dmax = fmax(dmax, bsum1(c, dd * dd));
    if (c.on) {
      Ui[(s + 1) * n + i] = un;
      Gi[s * n + i] = g;
    }
    u = un;
  }
  if (threadIdx.x == 0) {
    const double dlt = sqrt(P.h * dmax);
    delta[ii] = dlt;
    if (!(dlt == dlt) || dlt > 1e300) status |= 2;
    status_out[ii] |= status | *P.status;
  }
}

// --------------------------------------------------------------- energy
// E_h = h^d sum (u^2-1)^2/4 + (eps^2/2) h^d sum u (-Lap_h u); one block per state.
// Per-slice distance ||A_n - B_n||_h (h^d-weighted L2, the norm of the update
// norm) for the work items of one class, slice layout; one block per item,
// summed in a fixed order.  Streams both states once: 16 bytes per point.
__global__ void __launch_bounds__(256)
k_slice_dist(const WorkItem* __restrict__ items, const InstDev* __restrict__ inst,
             const double* __restrict__ A, const double* __restrict__ B, double* __restrict__ out) {
  __shared__ double red[4];
  const WorkItem it = items[blockIdx.x];
  const InstDev& P = inst[it.inst];
  const int64_t pts = P.dim == 2 ? (int64_t)P.n * P.n : P.n;
  const int64_t off = P.off_slices + (int64_t)it.slice * pts;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < pts; i += 256) {
    const double d = A[off + i] - B[off + i];
    acc += d * d;
  }
  double v[1] = {acc};
  block_sum<4, 1>(v, red);
  if (threadIdx.x == 0) {
    const double hd = P.dim == 2 ? P.h * P.h : P.h;
    out[P.slice_base + it.slice] = sqrt(hd * v[0]);
  }
}

hipError_t launch_slice_dist(const WorkItem* items, int n_items, const InstDev* inst,
                             const double* A, const double* B, double* out, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slice_dist, dim3(n_items), dim3(256), 0, s, items, inst, A, B, out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
k_energy(int n, int dim, const double* __restrict__ u, double eps, double* __restrict__ E) {
  __shared__ double red[8];
  const double* s = u + (int64_t)blockIdx.x * (dim == 2 ? (int64_t)n * n : n);
  const double h = 1.0 / (n + 1), ih2 = 1.0 / (h * h);
  double bulk = 0.0, grad = 0.0;
  const int tot = dim == 2 ? n * n : n;
  // 2D grids have n = 2^ln (32 .. 256): row and column by shift and mask
  const int ln = 31 - __builtin_clz(n);
#pragma unroll 4
  for (int idx = threadIdx.x; idx < tot; idx += 256) {
    const double c = s[idx];
    double lap;
    if (dim == 2) {
      const int iy = idx >> ln, ix = idx & (n - 1);
      const double a = iy > 0 ? s[idx - n] : 0.0, b = iy < n - 1 ? s[idx + n] : 0.0;
      const double l = ix > 0 ? s[idx - 1] : 0.0, r = ix < n - 1 ? s[idx + 1] : 0.0;
      lap = ((a + b) + (l + r) - 4.0 * c) * ih2;
    } else {
      const double l = idx > 0 ? s[idx - 1] : 0.0, r = idx < n - 1 ? s[idx + 1] : 0.0;
      lap = ((l + r) - 2.0 * c) * ih2;
    }
    const double t = c * c - 1.0;
    bulk += 0.25 * t * t;
    grad += -c * lap;
  }
  double v[2] = {bulk, grad};
  v[0] = wave_sum<4>(v[0]);
  v[1] = wave_sum<4>(v[1]);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) { red[w] = v[0]; red[4 + w] = v[1]; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double hd = dim == 2 ? h * h : h;
    const double b = (red[0] + red[1]) + (red[2] + red[3]);
    const double g = (red[4] + red[5]) + (red[6] + red[7]);
    E[blockIdx.x] = hd * b + 0.5 * eps * eps * hd * g;
  }
}

// first != 0: every instance active.  Otherwise instances whose last update
// norm fell below tol stop, once at least one correction has been made
// (device iteration counter *kdev > 0).
__global__ void k_flag_active(const double* __restrict__ delta, int32_t* __restrict__ active,
                              int n_inst, double tol, int first, const int32_t* __restrict__ kdev) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inst) return;
  if (first) active[i] = 1;
  else if (*kdev > 0 && active[i] && delta[i] < tol) active[i] = 0;
}
// *kdev = value (add == 0) or *kdev += value
__global__ void k_counter(int32_t* kdev, int value, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *kdev = add ? *kdev + value : value;
}
hipError_t launch_counter(int32_t* kdev, int value, int add, hipStream_t s) {
  hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, s, kdev, value, add);
  return hipGetLastError();
}

// ------------------------------------------------------------ launchers
template <int N, int NW>
static hipError_t fine2d(const WorkItem* items, int n_items, const InstDev* inst,
                         const double* Tg, const double* U_in, double* F_out,
                         const uint8_t* mask, const int32_t* active, const int32_t* kmin, int in_iter,
                         hipStream_t s, int j_steps = 0) {
  const size_t lds = (size_t)(Geo<N, NW>::XSZ + Geo<N, NW>::P2) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_fine_linear_2d<N, NW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fine_linear_2d<N, NW>), dim3(n_items), dim3(NW * 64), lds, s, items, inst,
                     Tg, U_in, F_out, mask, active, kmin, in_iter, j_steps);
  return hipGetLastError();
}

template <int N, int NW>
static hipError_t fine_stream(const WorkItem* items, int n_items, const InstDev* inst,
                              const double* Tg, const double* U_in, double* F_out,
                              const uint8_t* mask, const int32_t* active, const int32_t* kmin, int in_iter,
                              hipStream_t s, int j_steps) {
  const size_t lds = (size_t)(2 * GeoS<N, NW>::CHUNK + GeoS<N, NW>::P2) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_fine_linear_stream<N, NW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fine_linear_stream<N, NW>), dim3(n_items), dim3(NW * 64), lds, s, items,
                     inst, Tg, U_in, F_out, mask, active, kmin, in_iter, j_steps);
  return hipGetLastError();
}

// Tunable variants of the on-chip linear fine kernel: waves per workgroup.
int fine_wave_options(int n, int* out) {
  switch (n) {
    case 32: out[0] = 2; out[1] = 1; return 2;
    case 64: out[0] = 4; out[1] = 2; out[2] = 8; return 3;
    case 128: out[0] = 8; out[1] = 16; return 2;
    default: out[0] = 8; return 1;
  }
}

hipError_t launch_fine_2d(int n, const WorkItem* items, int n_items, const InstDev* inst,
                          const double* Tg, const double* U_in, double* F_out,
                          const uint8_t* mask, const int32_t* active, const int32_t* kmin, int in_iter,
                          hipStream_t s, int waves, int j_steps) {
  if (n_items <= 0) return hipSuccess;
  const int key = n * 100 + waves;
  switch (key) {
    case 25608: case 25600: return fine_stream<256, 8>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s, j_steps);
    case 3202: case 3200: return fine2d<32, 2>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s, j_steps);
    case 3201: return fine2d<32, 1>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s, j_steps);
    case 6404: case 6400: return fine2d<64, 4>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s, j_steps);
    case 6402: return fine2d<64, 2>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s, j_steps);
    case 6408: return fine2d<64, 8>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s, j_steps);
    case 12808: case 12800: return fine2d<128, 8>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s, j_steps);
    case 12816: return fine2d<128, 16>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s, j_steps);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int NW>
static hipError_t newton2d(const WorkItem* items, int n_items, const InstDev* inst,
                           const double* Tg, const double* U_in, double* F_out,
                           const uint8_t* mask, const int32_t* active, const int32_t* kmin, int in_iter,
                           hipStream_t s) {
  const size_t lds = ((size_t)Geo<N, NW>::XSZ + Geo<N, NW>::P2 + 4 * NW) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_fine_newton_2d<N, NW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fine_newton_2d<N, NW>), dim3(n_items), dim3(NW * 64), lds, s, items, inst,
                     Tg, U_in, F_out, mask, active, kmin, in_iter);
  return hipGetLastError();
}

template <int N, int NW>
static hipError_t newton_stream(const WorkItem* items, int n_items, const InstDev* inst,
                                const double* Tg, const double* U_in, double* F_out,
                                const uint8_t* mask, const int32_t* active, const int32_t* kmin,
                                int in_iter, hipStream_t s) {
  const size_t lds =
      ((size_t)2 * GeoS<N, NW>::CHUNK + GeoS<N, NW>::P2 + 4 * NW) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_fine_newton_stream<N, NW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fine_newton_stream<N, NW>), dim3(n_items), dim3(NW * 64), lds, s, items,
                     inst, Tg, U_in, F_out, mask, active, kmin, in_iter);
  return hipGetLastError();
}

template <int N, int NW>
static hipError_t approx2f_2d(const WorkItem* items, int n_items, const InstDev* inst,
                              const double* Tg, const double* U_in, double* F_out,
                              const uint8_t* mask, const int32_t* active, const int32_t* kmin,
                              int in_iter, hipStream_t s) {
  const size_t lds = ((size_t)Geo<N, NW>::XSZ + Geo<N, NW>::P2 + 4 * NW) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_fine_approx2_2d<N, NW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fine_approx2_2d<N, NW>), dim3(n_items), dim3(NW * 64), lds, s, items,
                     inst, Tg, U_in, F_out, mask, active, kmin, in_iter);
  return hipGetLastError();
}

template <int N, int NW>
static hipError_t approx2f_stream(const WorkItem* items, int n_items, const InstDev* inst,
                                  const double* Tg, const double* U_in, double* F_out,
                                  const uint8_t* mask, const int32_t* active, const int32_t* kmin,
                                  int in_iter, hipStream_t s) {
  const size_t lds =
      ((size_t)2 * GeoS<N, NW>::CHUNK + GeoS<N, NW>::P2 + 4 * NW) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_fine_approx2_stream<N, NW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fine_approx2_stream<N, NW>), dim3(n_items), dim3(NW * 64), lds, s, items,
                     inst, Tg, U_in, F_out, mask, active, kmin, in_iter);
  return hipGetLastError();
}

hipError_t launch_fine_approx2_2d(int n, const WorkItem* items, int n_items, const InstDev* inst,
                                  const double* Tg, const double* U_in, double* F_out,
                                  const uint8_t* mask, const int32_t* active, const int32_t* kmin,
                                  int in_iter, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  switch (n) {
    case 256: return approx2f_stream<256, 8>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s);
    case 32: return approx2f_2d<32, 2>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s);
    case 64: return approx2f_2d<64, 4>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s);
    case 128: return approx2f_2d<128, 8>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fine_newton_2d(int n, const WorkItem* items, int n_items, const InstDev* inst,
                                 const double* Tg, const double* U_in, double* F_out,
                                 const uint8_t* mask, const int32_t* active, const int32_t* kmin,
                                 int in_iter, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  switch (n) {
    case 256: return newton_stream<256, 8>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s);
    case 32: return newton2d<32, 2>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s);
    case 64: return newton2d<64, 4>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s);
    case 128: return newton2d<128, 8>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fine_1d(int n, const WorkItem* items, int n_items, const InstDev* inst,
                          const double* S, const double* U_in, double* F_out,
                          const uint8_t* mask, const int32_t* active, const int32_t* kmin, int in_iter,
                          hipStream_t s, int sine) {
  if (n_items <= 0) return hipSuccess;
  // lam for 1D is stored right after S (n x n) in the table block
  const double* lam = S + (size_t)n * n;
  const size_t lds = ((sine ? (size_t)n * n : 0) + n + 64 + direct1_lds_doubles(n)) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_fine_1d,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fine_1d, dim3(n_items), dim3((n + 63) / 64 * 64), lds, s, items, inst, S,
                     lam, U_in, F_out, mask, active, kmin, in_iter);
  return hipGetLastError();
}

hipError_t launch_fine_dd_1d(int n, const WorkItem* items, int n_items, const InstDev* inst,
                             const double* U_in, double* F_out, const uint8_t* mask,
                             const int32_t* active, const int32_t* kmin, int in_iter,
                             hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (n < 1 || n > 128) return hipErrorInvalidValue;
  const size_t lds = dd1_lds_doubles(n) * sizeof(double);
  hipLaunchKernelGGL(k_fine_dd_1d, dim3(n_items), dim3(128), lds, s, items, inst, U_in, F_out,
                     mask, active, kmin, in_iter);
  return hipGetLastError();
}

template <int N, int NW>
static hipError_t coarse2d(int mode, const int32_t* insts, int n_insts, const WorkItem* items,
                           int n_items, const InstDev* inst, const double* Tg,
                           const double* U_in, double* G_out, const uint8_t* mask, double* U,
                           const double* F, double* G_old, double* delta, int32_t* status,
                           const int32_t* active, int k, const int32_t* kdev, hipStream_t s,
                           const int32_t* gate) {
  const size_t lds = ((size_t)Geo<N, NW>::XSZ + Geo<N, NW>::P2 + 4 * NW) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_coarse_2d<N, NW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int grid = (mode == 0 || mode >= 3) ? n_items : n_insts;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_coarse_2d<N, NW>), dim3(grid), dim3(NW * 64), lds, s, mode, insts, items,
                     inst, Tg, U_in, G_out, mask, U, F, G_old, delta, status, active, k, kdev,
                     gate);
  return hipGetLastError();
}

template <int N, int NW>
static hipError_t coarse_stream(int mode, const int32_t* insts, int n_insts, const WorkItem* items,
                                int n_items, const InstDev* inst, const double* Tg,
                                const double* U_in, double* G_out, const uint8_t* mask, double* U,
                                const double* F, double* G_old, double* delta, int32_t* status,
                                const int32_t* active, int k, const int32_t* kdev, hipStream_t s,
                                const int32_t* gate) {
  const size_t lds =
      ((size_t)2 * GeoS<N, NW>::CHUNK + GeoS<N, NW>::P2 + 4 * NW) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_coarse_stream<N, NW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int grid = (mode == 0 || mode >= 3) ? n_items : n_insts;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_coarse_stream<N, NW>), dim3(grid), dim3(NW * 64), lds, s, mode, insts,
                     items, inst, Tg, U_in, G_out, mask, U, F, G_old, delta, status, active, k, kdev,
                     gate);
  return hipGetLastError();
}

hipError_t launch_coarse_2d(int n, int mode, const int32_t* insts, int n_insts,
                            const WorkItem* items, int n_items, const InstDev* inst,
                            const double* Tg, const double* U_in,
                            double* G_out, const uint8_t* mask, double* U, const double* F,
                            double* G_old, double* delta, int32_t* status,
                            const int32_t* active, int k, const int32_t* kdev, hipStream_t s,
                            const int32_t* gate) {
  switch (n) {
    case 256: return coarse_stream<256, 8>(mode, insts, n_insts, items, n_items, inst, Tg, U_in, G_out, mask, U, F, G_old, delta, status, active, k, kdev, s, gate);
    case 32: return coarse2d<32, 2>(mode, insts, n_insts, items, n_items, inst, Tg, U_in, G_out, mask, U, F, G_old, delta, status, active, k, kdev, s, gate);
    case 64: return coarse2d<64, 4>(mode, insts, n_insts, items, n_items, inst, Tg, U_in, G_out, mask, U, F, G_old, delta, status, active, k, kdev, s, gate);
    case 128: return coarse2d<128, 8>(mode, insts, n_insts, items, n_items, inst, Tg, U_in, G_out, mask, U, F, G_old, delta, status, active, k, kdev, s, gate);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_coarse_1d(int n, int mode, const int32_t* insts, int n_insts,
                            const WorkItem* items, int n_items, const InstDev* inst,
                            const double* S, const double* U_in, double* G_out,
                            const uint8_t* mask, double* U, const double* F, double* G_old,
                            double* delta, int32_t* status, const int32_t* active, int k,
                            const int32_t* kdev, hipStream_t s) {
  // lam for 1D is stored right after S (n x n) in the table block
  const double* lam = S + (size_t)n * n;
  const size_t lds = ((size_t)n * n + n + 64 + direct1_lds_doubles(n)) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_coarse_1d,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int grid = mode == 0 ? n_items : n_insts;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarse_1d, dim3(grid), dim3((n + 63) / 64 * 64), lds, s, mode, insts, items, inst, S, lam,
                     U_in, G_out, mask, U, F, G_old, delta, status, active, k, kdev);
  return hipGetLastError();
}

// ------------------------------------------ judge of the learned propagator
// Per learned-propagator instance t (global index insts[t]): live[i] = the
// instance is active and still uses the learned propagator (the gate of its
// network passes and of the plain propagator's judge pass).
__global__ void k_judge_live(const int32_t* __restrict__ insts, int n, const InstDev* __restrict__ inst,
                             const int32_t* __restrict__ active, int32_t* __restrict__ live) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= n) return;
  const int i = insts[t];
  live[i] = (!active || active[i]) && inst[i].coarse_kind == 2;
}
// A new run: the learned propagator again, no fallback, no previous norm.
__global__ void k_judge_reset(const int32_t* __restrict__ insts, int n, InstDev* __restrict__ inst,
                              JudgeDev* __restrict__ J, double* __restrict__ ratios, int rstride,
                              int32_t* __restrict__ refresh) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= n) return;
  const int i = insts[t];
  if (J[t].enabled) inst[i].coarse_kind = 2;
  J[t].delta_prev = __builtin_huge_val();
  J[t].fallback_at = -1;
  refresh[i] = 0;
  for (int k = 0; k < rstride; ++k) ratios[(int64_t)t * rstride + k] = __builtin_nan("");
}
// The judge's ratio of iteration k = *kdev: the mean over the slices n >= k
// with d_plain > 0 of d_learned / d_plain, d = ||G(U_n^k) - F_n||_h (NaN if
// no slice qualifies); one thread per instance, slices summed in order.
__global__ void k_judge_ratio(const int32_t* __restrict__ insts, int n,
                              const InstDev* __restrict__ inst, const int32_t* __restrict__ live,
                              const double* __restrict__ d_learned,
                              const double* __restrict__ d_plain, const int32_t* __restrict__ kdev,
                              double* __restrict__ ratios, int rstride) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= n) return;
  const int i = insts[t];
  if (!live[i]) return;
  const InstDev& P = inst[i];
  const int k = *kdev;
  double acc = 0.0;
  int cnt = 0;
  for (int sl = k; sl < P.n_slices; ++sl) {
    const double dp = d_plain[P.slice_base + sl];
    if (dp > 0.0) {
      acc += d_learned[P.slice_base + sl] / dp;
      ++cnt;
    }
  }
  if (k < rstride) ratios[(int64_t)t * rstride + k] = cnt ? acc / cnt : __builtin_nan("");
}
// After the correction of iteration k = *kdev: fall back to the plain
// propagator when the update norm is not finite, or no smaller than the
// previous one, or the judge's ratios of iterations k - 1 and k both exceed
// 1 (unless the norm is already below tol).  A fallback switches the
// instance's kind on the device and asks for G_old to be recomputed with the
// plain propagator at the new iterate (refresh).
__global__ void k_judge_decide(const int32_t* __restrict__ insts, int n, InstDev* __restrict__ inst,
                               const int32_t* __restrict__ live, const double* __restrict__ delta,
                               double tol, const int32_t* __restrict__ kdev,
                               JudgeDev* __restrict__ J, const double* __restrict__ ratios,
                               int rstride, int32_t* __restrict__ refresh) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= n) return;
  const int i = insts[t];
  refresh[i] = 0;
  if (!live[i]) return;
  const int k = *kdev;
  const double d = delta[i];
  const double* r = ratios + (int64_t)t * rstride;
  const bool worse = k >= 1 && k < rstride && r[k] > 1.0 && r[k - 1] > 1.0;
  if (!(d < tol) && (!(d == d) || d > 1e300 || d >= J[t].delta_prev || worse)) {
    inst[i].coarse_kind = 0;
    J[t].fallback_at = k + 1;
    refresh[i] = 1;
  }
  J[t].delta_prev = d;
}
hipError_t launch_judge(int what, const int32_t* insts, int n, InstDev* inst, const int32_t* active,
                        int32_t* live, JudgeDev* J, double* ratios, int rstride, int32_t* refresh,
                        const double* d_learned, const double* d_plain, const double* delta,
                        double tol, const int32_t* kdev, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((n + 63) / 64), blk(64);
  switch (what) {
    case 0: hipLaunchKernelGGL(k_judge_reset, grid, blk, 0, s, insts, n, inst, J, ratios, rstride, refresh); break;
    case 1: hipLaunchKernelGGL(k_judge_live, grid, blk, 0, s, insts, n, inst, active, live); break;
    case 2: hipLaunchKernelGGL(k_judge_ratio, grid, blk, 0, s, insts, n, inst, live, d_learned, d_plain, kdev, ratios, rstride); break;
    case 3: hipLaunchKernelGGL(k_judge_decide, grid, blk, 0, s, insts, n, inst, live, delta, tol, kdev, J, ratios, rstride, refresh); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ void k_zero_i32(int32_t* p, int count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = 0;
}
hipError_t launch_zero_i32(int32_t* p, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i32, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
  return hipGetLastError();
}
__global__ void k_status_merge(int32_t* __restrict__ dst, const int32_t* __restrict__ src,
                               int count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < count) dst[i] |= src[i];
}
hipError_t launch_status_merge(int32_t* dst, const int32_t* src, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_status_merge, dim3((count + 255) / 256), dim3(256), 0, s, dst, src, count);
  return hipGetLastError();
}

template <int N, int G, int NW, bool OPQ>
static hipError_t chain_coop(int mode, const int32_t* insts, int n_insts, const InstDev* inst,
                             const double* Tg, const double* lam, double* U, const double* F,
                             double* G_old, double* delta, int32_t* status, const int32_t* active,
                             int k, const int32_t* kdev, int32_t* sync, hipStream_t s) {
  using C = GeoC<N, G, NW>;
  const size_t lds =
      ((size_t)N * C::LDB + C::P2 + N + 4 * NW + 3 * (size_t)C::OWN * C::NT) * sizeof(double);
  const void* fn = (const void*)k_chain_coop<N, G, NW, OPQ>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  // every workgroup of the grid must be resident at once
  int dev = 0, cus = 0, per_cu = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NW * 64, lds)) != hipSuccess)
    return e;
  const int groups = (n_insts + 7) / 8;
  const int grid = 8 * G * groups;
  if (grid > cus * per_cu) return hipErrorCooperativeLaunchTooLarge;
  const int words = 64 * 8 * groups;
  hipLaunchKernelGGL(k_zero_i32, dim3((words + 255) / 256), dim3(256), 0, s, sync, words);
  hipLaunchKernelGGL((k_chain_coop<N, G, NW, OPQ>), dim3(grid), dim3(NW * 64), lds, s, mode, insts,
                     n_insts, inst, Tg, lam, U, F, G_old, delta, status, active, k, kdev, sync);
  return hipGetLastError();
}

template <int N, int G, int NW, bool OPQ>
static hipError_t fine_group(const WorkItem* items, int n_items, const InstDev* inst,
                             const double* Tg, const double* U_in, double* F_out,
                             const uint8_t* mask, const int32_t* active, const int32_t* kmin,
                             int in_iter, int j_steps, int32_t* sync, hipStream_t s) {
  using C = GeoC<N, G, NW>;
  const size_t lds = ((size_t)N * C::LDB + C::P2 + N + (size_t)C::OWN * C::NT) * sizeof(double);
  const void* fn = (const void*)k_fine_group<N, G, NW, OPQ>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0, per_cu = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NW * 64, lds)) != hipSuccess)
    return e;
  // groups in multiples of eight (one per XCD), as many as fit at once, at
  // most one per work item (rounded up to eight)
  const int fit8 = cus * per_cu / (8 * G);
  if (fit8 < 1) return hipErrorCooperativeLaunchTooLarge;
  const int groups8 = std::min((n_items + 7) / 8, fit8);
  const int grid = 8 * G * groups8;
  const int words = 64 * 8 * groups8;
  hipLaunchKernelGGL(k_zero_i32, dim3((words + 255) / 256), dim3(256), 0, s, sync, words);
  const double* lam = Tg + 2 * (N + 1);
  hipLaunchKernelGGL((k_fine_group<N, G, NW, OPQ>), dim3(grid), dim3(NW * 64), lds, s, items, n_items,
                     inst, Tg, lam, U_in, F_out, mask, active, kmin, in_iter, j_steps, sync);
  return hipGetLastError();
}

template <int N, int G, int NW, bool OPQ>
static hipError_t newton_group(const WorkItem* items, int n_items, const InstDev* inst,
                               const double* Tg, const double* U_in, double* F_out,
                               const uint8_t* mask, const int32_t* active, const int32_t* kmin,
                               int in_iter, int32_t* sync, hipStream_t s) {
  using C = GeoC<N, G, NW>;
  const size_t lds =
      ((size_t)N * C::LDB + C::P2 + N + 4 * NW + 3 * (size_t)C::OWN * C::NT) * sizeof(double);
  const void* fn = (const void*)k_fine_newton_group<N, G, NW, OPQ>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0, per_cu = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NW * 64, lds)) != hipSuccess)
    return e;
  const int fit8 = cus * per_cu / (8 * G);
  if (fit8 < 1) return hipErrorCooperativeLaunchTooLarge;
  const int groups8 = std::min((n_items + 7) / 8, fit8);
  const int grid = 8 * G * groups8;
  const int words = 64 * 8 * groups8;
  hipLaunchKernelGGL(k_zero_i32, dim3((words + 255) / 256), dim3(256), 0, s, sync, words);
  const double* lam = Tg + 2 * (N + 1);
  hipLaunchKernelGGL((k_fine_newton_group<N, G, NW, OPQ>), dim3(grid), dim3(NW * 64), lds, s, items,
                     n_items, inst, Tg, lam, U_in, F_out, mask, active, kmin, in_iter, sync);
  return hipGetLastError();
}

// Implicit fine sweep on groups of workgroups (2D; n = 128: G = 8, n = 256:
// G = 16); hipErrorNotSupported for other shapes, hipErrorCooperativeLaunchTooLarge
// when no group fits on the device.
hipError_t launch_fine_newton_group(int n, int groups, const WorkItem* items, int n_items,
                                    const InstDev* inst, const double* Tg, const double* U_in,
                                    double* F_out, const uint8_t* mask, const int32_t* active,
                                    const int32_t* kmin, int in_iter, int32_t* sync,
                                    hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  switch (n * 100 + groups) {
    case 12808: return newton_group<128, 8, 4, true>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, sync, s);
    case 25616: return newton_group<256, 16, 8, true>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, sync, s);
    default: return hipErrorNotSupported;
  }
}

// Largest work-item count for which the multi-workgroup fine sweep is the
// default for class size n (0: never).  The kernel is persistent and takes
// any count; at n = 128 one workgroup per slice is faster once the slices
// alone fill the device, at n = 256 the group kernel (state on chip in the
// members' slabs) beats the streamed one-workgroup kernel at any count.
// Group sizes of the linear fine sweep for class size n (tuning candidates).
int fine_group_options(int n, int* out) {
  switch (n) {
    case 128: out[0] = 8; out[1] = 4; return 2;
    case 256: out[0] = 8; return 1;
    default: return 0;
  }
}

int fine_group_capacity(int n) {
  switch (n) {
    case 128: return 64;
    case 256: return 1 << 30;
    default: return 0;
  }
}

// Default group size for class size n: eight at both sizes (at n = 128 two
// groups share a CU; measured 3% faster than four per slice with the
// coherent exchange protocol).
int fine_group_default(int) { return 8; }

// Fine sweep of the linear FP64 step on groups of workgroups (2D, n = 128:
// G = 4 or 8; n = 256: G = 8); hipErrorNotSupported for other shapes,
// hipErrorCooperativeLaunchTooLarge when no group fits on the device.
hipError_t launch_fine_group(int n, int groups, const WorkItem* items, int n_items,
                             const InstDev* inst, const double* Tg, const double* U_in,
                             double* F_out, const uint8_t* mask, const int32_t* active,
                             const int32_t* kmin, int in_iter, int32_t* sync, hipStream_t s,
                             int j_steps) {
  if (n_items <= 0) return hipSuccess;
  switch (n * 100 + groups) {
    // eight waves per workgroup at G = 4 (two per SIMD hide LDS and exchange
    // latency; measured 9% faster than four); G = 8 allows only four at n = 128
    case 12804: return fine_group<128, 4, 8, false>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, j_steps, sync, s);
    case 12808: return fine_group<128, 8, 4, false>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, j_steps, sync, s);
    case 25608: return fine_group<256, 8, 8, false>(items, n_items, inst, Tg, U_in, F_out, mask, active, kmin, in_iter, j_steps, sync, s);
    default: return hipErrorNotSupported;
  }
}

// Largest instance count the cooperative chain takes for class size n (0: none).
int chain_coop_capacity(int n) {
  switch (n) {
    case 128: return 64;
    default: return 0;
  }
}

// Coarse chain on a group of workgroups per instance (2D, n = 128, scheme
// (2.4) only); hipErrorNotSupported for other sizes.
hipError_t launch_chain_coop(int n, int groups, int mode, const int32_t* insts, int n_insts,
                             const InstDev* inst, const double* Tg, double* U, const double* F,
                             double* G_old, double* delta, int32_t* status, const int32_t* active,
                             int k, const int32_t* kdev, int32_t* sync, hipStream_t s) {
  if (n_insts <= 0) return hipSuccess;
  if (n_insts > chain_coop_capacity(n)) return hipErrorNotSupported;
  const double* lam = Tg + 2 * (n + 1);
  switch (n * 100 + groups) {
    case 12804: return chain_coop<128, 4, 4, false>(mode, insts, n_insts, inst, Tg, lam, U, F, G_old, delta, status, active, k, kdev, sync, s);
    case 12808: return chain_coop<128, 8, 4, false>(mode, insts, n_insts, inst, Tg, lam, U, F, G_old, delta, status, active, k, kdev, sync, s);
    default: return hipErrorNotSupported;
  }
}

template <int N, int G, int NW>
static hipError_t parareal_pipe(PipeArgs A, int n_slices, int32_t* sync, hipStream_t s) {
  using C = GeoC<N, G, NW>;
  const size_t lds =
      ((size_t)N * C::LDB + C::P2 + N + 4 * NW + 3 * (size_t)C::OWN * C::NT) * sizeof(double);
  const void* fn = (const void*)k_parareal_pipe<N, G, NW>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0, per_cu = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NW * 64, lds)) != hipSuccess)
    return e;
  // one coarse-sweep group and up to N - 1 fine groups, all resident at once
  const int max_groups = 8 * (cus * per_cu / (8 * G));
  const int groups = std::min(max_groups, 8 * ((n_slices + 1 + 7) / 8));
  const int grid = G * groups;
  // With more workgroups than CUs the dispatcher gives block b + cus the CU of
  // block b (measured: every block of a 512-block launch on a 256-CU device
  // shares its CU with the block 256 later).  The group holding the partners
  // of the coarse-sweep group (blocks 8m, m < G) is left idle, so the sweep,
  // the latency-bound part, has its CUs to itself.  Only speed depends on this.
  int idle = -1;
  if (grid > cus && (cus / 8) % G == 0 && (cus / 8) / G * 8 < groups) idle = (cus / 8) / G * 8;
  const int n_fine = std::min(groups - 1 - (idle >= 0 ? 1 : 0), n_slices - 1);
  if (n_fine < 1) return hipErrorCooperativeLaunchTooLarge;
  const int bar_words = 64 * 8 * ((n_slices + 7) / 8);
  A.bar = sync;
  A.ucnt = sync + bar_words;
  A.fcnt = A.ucnt + n_slices;
  A.ctl = A.fcnt + n_slices;
  A.n_fine = n_fine;
  A.idle = idle;
  const int words = pipe_sync_words(n_slices);
  hipLaunchKernelGGL(k_zero_i32, dim3((words + 255) / 256), dim3(256), 0, s, sync, words);
  const int64_t count = (int64_t)n_slices * N * N;   // U_0..U_{N-1} into both input buffers
  hipLaunchKernelGGL(k_copy2, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, A.U, A.Uin,
                     A.Uin + count, count);
  hipLaunchKernelGGL((k_parareal_pipe<N, G, NW>), dim3(grid), dim3(NW * 64), lds, s, A);
  hipLaunchKernelGGL(k_pipe_finish, dim3(1), dim3(64), 0, s, const_cast<int32_t*>(A.kdev), A.ctl);
  return hipGetLastError();
}

// Sync words of the pipelined launch: barrier counters of up to N groups,
// the two hand-off counters per slice, two control words.
int pipe_sync_words(int n_slices) { return 64 * 8 * ((n_slices + 7) / 8) + 2 * n_slices + 2; }

bool pipe_supported(int n) { return n == 128; }

// Pipelined Parareal iterations of one instance (2D, n = 128, scheme (2.4),
// linear FP64 fine step, groups of eight workgroups).  U is the instance's
// iterate layout, F0 its slice layout; F1 (N n^2) and Uin (2 N n^2) are
// scratch; sync holds pipe_sync_words(N) ints.  hipErrorNotSupported for other
// shapes, hipErrorCooperativeLaunchTooLarge when the groups cannot all be
// resident.
hipError_t launch_parareal_pipe(int n, const InstDev* inst, int ii, int n_slices,
                                const double* Tsin, double* U, double* F0, double* F1,
                                double* Uin, double* G_old, double* delta, int32_t* status,
                                const int32_t* active, int32_t* kdev, int K, int sweep_all,
                                double tol, int32_t* sync, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  if (!pipe_supported(n) || n_slices < 2) return hipErrorNotSupported;
  PipeArgs A{};
  A.inst = inst;
  A.Tg = Tsin;
  A.lam = Tsin + 2 * (n + 1);
  A.U = U;
  A.F0 = F0;
  A.F1 = F1;
  A.Uin = Uin;
  A.G_old = G_old;
  A.delta = delta;
  A.status_out = status;
  A.active = active;
  A.kdev = kdev;
  A.ii = ii;
  A.K = K;
  A.sweep_all = sweep_all;
  A.tol = tol;
  return parareal_pipe<128, 8, 4>(A, n_slices, sync, s);
}

hipError_t launch_cg_tables(int n, int dim, const int32_t* insts, int n_insts, const InstDev* inst,
                            const double* lam, hipStream_t s) {
  if (dim != 2 || n_insts <= 0) return hipSuccess;
  switch (n) {
    case 256:
      hipLaunchKernelGGL(k_cg_tables_natural, dim3((256 * 256 + 255) / 256, n_insts), dim3(256), 0, s,
                         insts, inst, lam);
      break;
    case 32: hipLaunchKernelGGL((k_cg_tables_2d<32, 2>), dim3(n_insts), dim3(128), 0, s, insts, inst, lam); break;
    case 64: hipLaunchKernelGGL((k_cg_tables_2d<64, 4>), dim3(n_insts), dim3(256), 0, s, insts, inst, lam); break;
    case 128: hipLaunchKernelGGL((k_cg_tables_2d<128, 8>), dim3(n_insts), dim3(512), 0, s, insts, inst, lam); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_energy(int n, int dim, const double* u, int count, double eps, double* E,
                         hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_energy, dim3(count), dim3(256), 0, s, n, dim, u, eps, E);
  return hipGetLastError();
}

hipError_t launch_flag_active(const double* delta, int32_t* active, int n_inst, double tol,
                              int first, const int32_t* kdev, hipStream_t s) {
  hipLaunchKernelGGL(k_flag_active, dim3((n_inst + 255) / 256), dim3(256), 0, s, delta, active,
                     n_inst, tol, first, kdev);
  return hipGetLastError();
}

}  // namespace chk
