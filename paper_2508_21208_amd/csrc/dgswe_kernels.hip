// gfx950 kernels of one SSP-RK(2,2) discontinuous Galerkin shallow-water
// step (arXiv 2508.21208, Sec. 2.2 and Sec. 5.2).
//
// One fused kernel per RK stage.  A workgroup owns a chunk of C consecutive
// elements (Hilbert order, so a compact patch of the mesh) and works in four
// phases separated by barriers, all intermediates in LDS:
//   L  load the chunk and its ring-1 halo (full state) and the ring-2 halo
//      (means) of the previous stage's UNLIMITED result, and issue the loads
//      of phases P and E (bathymetry, neighbour lists, edge records) so they
//      arrive while L completes (phase A's inputs - geometry, nodal forcing,
//      RK base - are requested after phase P or in phase A: registers held
//      from L through E would cost the third wave per SIMD);
//   P  slope limiter + wet/dry of the chunk and ring 1 (the paper's SLOPELIM
//      and WETDRY kernels), so every state the edges need is post-processed;
//   E  each edge touching the chunk: traces of both sides at the three
//      Gauss-Lobatto points, local Lax-Friedrichs flux with the wet/dry
//      rules, computed once per edge (Algorithm 2) into two flux moments;
//   A  one lane per element: volume and source integrals at the three area
//      points (Algorithm 1), fixed-order gather of its three edges
//      (Algorithm 3), inverse diagonal mass matrix and the Shu-Osher RK
//      combination; the result is written unlimited.
// Edges on a chunk border and ring-1 post-processing are computed by both
// neighbouring chunks, identically, instead of being exchanged.  The CFL
// candidate of the next step comes from the unlimited stage-2 result: the
// post-processing leaves the mean depth and, in wet elements, the mean
// momentum unchanged.  No floating-point atomics: results are deterministic.
// k_forcing evaluates the Holland vortex once per mesh node and stage (the
// paper's WIND node loops).  With the vertex-based limiter, k_vbounds
// first forms per mesh node the range of the unlimited element means around
// it, and phase P limits each element against the ranges at its vertices.
//
// Precision.  The kernels are templated on QT, the storage type of the
// momentum modes and the arithmetic type of the flux, volume and source
// terms; QT = double is the FP64 path.  QT = float is the mixed path (the
// paper runs everything in FP32): zeta modes, bathymetry, element areas,
// every limiter and wet/dry decision of the post-processing, the hydrostatic
// term g/2 zeta (zeta + 2 h_b), the zeta jump of the numerical flux, the
// zeta right-hand side and its RK update stay FP64.  Each FP32 edge mass
// moment is added to one element and subtracted from the other in FP64, so
// mass is conserved to FP64 rounding in both paths.
#include "dgswe_p1.h"

namespace dgswe {

#undef HD

// ---------------------------------------------------------------- kernels

// Forcing blocks are numbered member by member (members without a moving
// vortex have none); block b finds its member by bisection of fblk_off.
__global__ __launch_bounds__(kBlock) void k_forcing(DevMesh m, DevState s, Params p, int slot, double c) {
  const int b = blockIdx.x;
  int lo = 0, hi = m.nmem;  // fblk_off[lo] <= b < fblk_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (m.fblk_off[mid] <= b) lo = mid;
    else hi = mid;
  }
  const Member &f = m.mem[lo];
  const Ctrl *ctl = s.ctrl + lo;
  const int i = (b - m.fblk_off[lo]) * kBlock + threadIdx.x;
  if (i >= f.nn || ctl->status) return;
  double dt;
  if (!step_dt(ctl, p, slot, dt)) return;
  const int n = f.n0 + i;
  double out[3];
  holland(f, m.node_x[n], m.node_y[n], ctl->t[slot] + c * dt, out);
  ((double2 *)s.nodal)[n] = make_double2(out[0], out[1]);
  s.nodal[2 * (size_t)m.nn + n] = out[2];
}

// One RK stage (stage1_chunk): one chunk per workgroup, or (PERSIST)
// workgroup b takes the chunks of items b, b + gridDim.x, ...  The loop
// costs registers (the compiler keeps loop-invariant kernel arguments live
// across iterations), which is why it is a separate instantiation.
template <int NT, int WPE, class QT, int STAGE, bool VL, bool PERSIST>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void k_stage(
    DevMesh m, DevState s, Params p, CSt<QT> win, CSt<QT> wbase, St<QT> wout, St<QT> wpp, StageCoef sc, int slot,
    int want_dt) {
  extern __shared__ double lds_raw[];
  __shared__ double red[NT / 64];
  if constexpr (PERSIST) {
    for (int b = blockIdx.x; b < m.nch; b += gridDim.x) {
      stage1_chunk<NT, QT, STAGE, VL>(m, s, p, win, wbase, wout, wpp, sc, slot, want_dt, chunk_of_block(b, m.nch),
                                      lds_raw, red);
      __syncthreads();  // the next chunk overwrites the LDS
    }
  } else {
    const int c = chunk_of_block(blockIdx.x, m.nch);
    if (c < 0) return;  // the same for every lane of the block
    stage1_chunk<NT, QT, STAGE, VL>(m, s, p, win, wbase, wout, wpp, sc, slot, want_dt, c, lds_raw, red);
  }
}

// elements [e0, e0 + count) of a state (post-processed if pp) as FP64
// [9][count], for read-back
template <class QT>
__global__ __launch_bounds__(kBlock) void k_post_only(DevMesh m, Params p, const double *vb, CSt<QT> win, int pp,
                                                      int e0, int count, double *__restrict__ wout,
                                                      const int *__restrict__ perm) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  double u[9];
  load_pp_global<QT>(m, p, vb, win, e0 + i, pp != 0, u);
  const int c = perm ? perm[e0 + i] : i;
  for (int j = 0; j < 9; ++j) wout[(size_t)j * count + c] = u[j];
}

// Vertex-based limiter: per mesh node (range slot n), the smallest and
// largest unlimited mean of zeta, Qx, Qy over the elements having the node
// as a vertex.
template <class QT>
__global__ __launch_bounds__(kBlock) void k_vbounds(DevMesh m, CSt<QT> w, double *__restrict__ vb) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= m.nn) return;
  const int2 r = m.nd_rng[n];
  const size_t ne = (size_t)m.ne;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int j = 0; j < r.y; ++j) {
    const int e = m.nd_el[r.x + j];
    const double v[3] = {w.z[e], (double)w.q[e], (double)w.q[3 * ne + e]};
    for (int q = 0; q < 3; ++q) {
      lo[q] = fmin(lo[q], v[q]);
      hi[q] = fmax(hi[q], v[q]);
    }
  }
  double2 *o = (double2 *)vb + 3 * (size_t)n;
  for (int q = 0; q < 3; ++q) o[q] = make_double2(lo[q], hi[q]);
}

__global__ void k_ctrl_reset(Ctrl *c, double t, int pp_in) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->t[0] = t;
    c->t[1] = t;
    c->dt_last = 0.0;
    c->dtmin[0] = double_to_bits(INFINITY);
    c->dtmin[1] = double_to_bits(INFINITY);
    c->steps = 0;
    c->status = 0;
    c->pp_in = pp_in;
  }
}

// CFL candidates of elements [e0, e0 + count) into ctl->dtmin[slot]
template <class QT>
__global__ __launch_bounds__(kBlock) void k_init(DevMesh m, Ctrl *ctl, Params p, CSt<QT> w, int e0, int count,
                                                 int slot, int nm) {
  __shared__ double red[kBlock / 64];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double cand = INFINITY;
  if (i < count) {
    const size_t ne = (size_t)m.ne;
    const int e = e0 + i;
    const double h[3] = {m.hbv[e], m.hbv[ne + e], m.hbv[2 * ne + e]};
    cand = cfl_candidate(w.z[e], (double)w.q[e], (double)w.q[(size_t)nm * ne + e], mean3(h), m.inr2[e], p);
  }
  const double bm = block_min<kBlock>(cand, red);
  if (threadIdx.x == 0 && bm < INFINITY) atomicMin(&ctl->dtmin[slot], double_to_bits(bm));
}

// Diagnostics: per-block partial sums (mass, volume, wet count), then one
// block adds the partials in a fixed order: deterministic.  Mean depth and
// zeta mean are unchanged by the post-processing, so the unlimited state
// gives the same values; z is the zeta block of a state buffer.
__global__ __launch_bounds__(kBlock) void k_diag1(DevMesh m, Params p, const double *__restrict__ z, int e0,
                                                  int count, double *__restrict__ partial) {
  __shared__ double sm[3][kBlock];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int e = e0 + i;
  const size_t ne = (size_t)m.ne;
  double a = 0.0, b = 0.0, c = 0.0;
  if (i < count) {
    const double h[3] = {m.hbv[e], m.hbv[ne + e], m.hbv[2 * ne + e]};
    const double hmean = mean3(h);
    const double z0 = z[e];
    a = m.area[e] * z0;
    b = m.area[e] * (z0 + hmean);
    c = (p.wetdry ? (z0 + hmean > p.h0) : true) ? 1.0 : 0.0;
  }
  sm[0][threadIdx.x] = a; sm[1][threadIdx.x] = b; sm[2][threadIdx.x] = c;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int q = 0; q < 3; ++q) sm[q][threadIdx.x] += sm[q][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int nb = gridDim.x;
    partial[blockIdx.x] = sm[0][0];
    partial[nb + blockIdx.x] = sm[1][0];
    partial[2 * nb + blockIdx.x] = sm[2][0];
  }
}

__global__ __launch_bounds__(kBlock) void k_diag2(const double *__restrict__ partial, int nb, double *out) {
  __shared__ double sm[3][kBlock];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nb; i += kBlock)
    for (int q = 0; q < 3; ++q) acc[q] += partial[(size_t)q * nb + i];
  for (int q = 0; q < 3; ++q) sm[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int q = 0; q < 3; ++q) sm[q][threadIdx.x] += sm[q][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sm[0][0];
    out[1] = sm[1][0];
    out[2] = sm[2][0];
  }
}

// One member's diagnostics as 8 doubles: t, dt_last, mass, volume, steps,
// n_wet, n_dry, status.
__global__ void k_diag_pack(const Ctrl *__restrict__ ctl, int slot, int count, const double *__restrict__ sums,
                            double *__restrict__ out) {
  if (threadIdx.x != 0) return;
  out[0] = ctl->t[slot];
  out[1] = ctl->dt_last;
  out[2] = sums[0];
  out[3] = sums[1];
  out[4] = (double)ctl->steps;
  out[5] = sums[2];
  out[6] = (double)count - sums[2];
  out[7] = (double)ctl->status;
}

// ---------------------------------------------------------------- launchers
static inline unsigned nblk(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

int diag_blocks(int ne) { return (int)nblk(ne); }

size_t stage_lds_bytes(const DevMesh &m, int precision) {
  return precision == DGSWE_MIXED ? lds_bytes<float>(m) : lds_bytes<double>(m);
}

size_t state_bytes(size_t ne, int precision, int order) {
  const size_t nm = order == 2 ? 6 : 3;
  return ne * nm * (precision == DGSWE_MIXED ? sizeof(double) + 2 * sizeof(float) : 3 * sizeof(double));
}

bool stage_block_ok(int block) {
  for (int b : kStageBlocks)
    if (b == block) return true;
  return false;
}


hipError_t launch_forcing(const DevMesh &m, const DevState &s, const Params &p, int nfblk, int slot, double c,
                          hipStream_t st) {
  if (nfblk > 0) hipLaunchKernelGGL(k_forcing, dim3(nfblk), dim3(kBlock), 0, st, m, s, p, slot, c);
  return hipGetLastError();
}

template <class QT>
static void stage_qt(const DevMesh &m, const DevState &s, const Params &p, const void *win, const void *wbase,
                     void *wout, void *wpp, int slot, int first, const StageCoef &sc, int want_dt, int block,
                     hipStream_t st) {
  const size_t ne = (size_t)m.ne;
  const size_t lds = lds_bytes<QT>(m);
  const CSt<QT> a = csplit<QT>(win, ne);
  const CSt<QT> b = wbase ? csplit<QT>(wbase, ne) : CSt<QT>{nullptr, nullptr};
  const St<QT> o = split<QT>(wout, ne);
  const St<QT> q = wpp ? split<QT>(wpp, ne) : St<QT>{nullptr, nullptr};
#define DGSWE_STAGE(NT, W, S, V)                                                                             \
  do {                                                                                                       \
    if (p.persistent > 0)                                                                                    \
      hipLaunchKernelGGL((k_stage<NT, W, QT, S, V, true>), dim3(stage_grid(p, m.nch)), dim3(NT), lds, st, m, s, \
                         p, a, b, o, q, sc, slot, want_dt);                                                  \
    else                                                                                                     \
      hipLaunchKernelGGL((k_stage<NT, W, QT, S, V, false>), dim3(m.nch), dim3(NT), lds, st, m, s, p, a, b, o, q, \
                         sc, slot, want_dt);                                                                 \
  } while (0)
  (void)block;  // 256 lanes (the local ids and edge codes are packed for it)
  if (p.limiter == 2) {
    if (!first) DGSWE_STAGE(256, 2, 1, true);
    else DGSWE_STAGE(256, 2, 0, true);
  } else {
    if (!first) DGSWE_STAGE(256, 2, 1, false);
    else DGSWE_STAGE(256, 2, 0, false);
  }
#undef DGSWE_STAGE
}

hipError_t launch_stage(const DevMesh &m, const DevState &s, const Params &p, const void *win, const void *wbase,
                        void *wout, void *wpp, int slot, int first, const StageCoef &sc, int want_dt, int block,
                        int precision, hipStream_t st) {
  if (precision == DGSWE_MIXED)
    stage_qt<float>(m, s, p, win, wbase, wout, wpp, slot, first, sc, want_dt, block, st);
  else
    stage_qt<double>(m, s, p, win, wbase, wout, wpp, slot, first, sc, want_dt, block, st);
  return hipGetLastError();
}

hipError_t launch_vbounds(const DevMesh &m, const DevState &s, const void *win, int precision, hipStream_t st) {
  const size_t ne = (size_t)m.ne;
  if (precision == DGSWE_MIXED)
    hipLaunchKernelGGL(k_vbounds<float>, dim3(nblk(m.nn)), dim3(kBlock), 0, st, m, csplit<float>(win, ne), s.vb);
  else
    hipLaunchKernelGGL(k_vbounds<double>, dim3(nblk(m.nn)), dim3(kBlock), 0, st, m, csplit<double>(win, ne), s.vb);
  return hipGetLastError();
}

hipError_t launch_post_only(const DevMesh &m, const DevState &s, const Params &p, const void *win, int pp, int e0,
                            int count, double *wout, const int *perm, int precision, hipStream_t st) {
  const size_t ne = (size_t)m.ne;
  if (count <= 0) return hipSuccess;
  if (pp && p.limiter == 2) {
    const hipError_t e = launch_vbounds(m, s, win, precision, st);
    if (e != hipSuccess) return e;
  }
  if (precision == DGSWE_MIXED)
    hipLaunchKernelGGL(k_post_only<float>, dim3(nblk(count)), dim3(kBlock), 0, st, m, p, (const double *)s.vb,
                       csplit<float>(win, ne), pp, e0, count, wout, perm);
  else
    hipLaunchKernelGGL(k_post_only<double>, dim3(nblk(count)), dim3(kBlock), 0, st, m, p, (const double *)s.vb,
                       csplit<double>(win, ne), pp, e0, count, wout, perm);
  return hipGetLastError();
}

hipError_t launch_init_state(const DevMesh &m, const DevState &s, const Params &p, const void *w, int mb, int e0,
                             int count, double t, int slot, int pp_in, int precision, int order, hipStream_t st) {
  const size_t ne = (size_t)m.ne;
  Ctrl *ctl = s.ctrl + mb;
  const int nm = order == 2 ? 6 : 3;
  hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, st, ctl, t, pp_in);
  if (count <= 0) return hipGetLastError();
  if (precision == DGSWE_MIXED)
    hipLaunchKernelGGL(k_init<float>, dim3(nblk(count)), dim3(kBlock), 0, st, m, ctl, p, CSt<float>{(const double *)w, (const float *)((const double *)w + nm * ne)},
                       e0, count, slot, nm);
  else
    hipLaunchKernelGGL(k_init<double>, dim3(nblk(count)), dim3(kBlock), 0, st, m, ctl, p, CSt<double>{(const double *)w, (const double *)w + nm * ne},
                       e0, count, slot, nm);
  return hipGetLastError();
}

hipError_t launch_diag(const DevMesh &m, const Params &p, const void *w, int e0, int count, double *partial,
                       double *out4, hipStream_t st) {
  const int nb = (int)nblk(count > 0 ? count : 1);
  hipLaunchKernelGGL(k_diag1, dim3(nb), dim3(kBlock), 0, st, m, p, (const double *)w, e0, count, partial);
  hipLaunchKernelGGL(k_diag2, dim3(1), dim3(kBlock), 0, st, (const double *)partial, nb, out4);
  return hipGetLastError();
}

hipError_t launch_diag_pack(const Ctrl *ctl, int slot, int count, const double *sums3, double *out8,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_diag_pack, dim3(1), dim3(64), 0, st, ctl, slot, count, sums3, out8);
  return hipGetLastError();
}

}  // namespace dgswe
