// gfx950 kernels of the p = 2 DG step (six modes per variable): the same
// SSP-RK(2,2) scheme, fluxes and source terms as the p = 1 path (arXiv
// 2508.21208, Sec. 2.2), with the Dubiner basis carried to degree 2 and the
// quadratures raised to match (degree-4 area rule, 4-point Gauss-Lobatto
// edges).
//
// Two kernels per RK stage, one workgroup per chunk of 256 consecutive
// (Hilbert-ordered) elements:
//   k_pp2   slope limiter + wet/dry of the stage input (raw state, structure
//           of arrays) into a post-processed copy, one 16-byte-aligned record
//           per element (144 B in FP64), so a neighbour's state is a few
//           contiguous 16-byte loads;
//   k_rhs2  first every edge touching the chunk, once, one lane per edge:
//           both sides' traces at the four Gauss-Lobatto points from the
//           records, the wet/dry edge rules and the numerical flux, into
//           LDS (Algorithm 2's edge pass); then one lane per element: the
//           volume and source integrals at the six area points, its three
//           edges' fluxes from LDS in a fixed order (Algorithms 1 and 3),
//           inverse mass diagonal and the Shu-Osher RK combination, written
//           raw.
// An edge on a chunk border is evaluated by both chunks it touches, with the
// same instructions on the same records, so both get bitwise the same flux:
// no edge buffer in HBM, no atomics, mass conserved to rounding.  The
// post-processed stage-1 input (the RK base of stage 2) is kept as the first
// stage's record buffer.
//
// Precision as in the p = 1 path: QT is the storage type of the momentum
// modes and the arithmetic type of flux, volume and source terms; zeta,
// bathymetry, the post-processing and the zeta update stay FP64.
#include <algorithm>
#include <cstdlib>

#include "dgswe_p2.h"

namespace dgswe {

// ---------------------------------------------------------------- kernels
// Post-processing of one stage input into records (pp2_chunk): one chunk
// per workgroup, or (PERSIST) workgroup b takes items b, b + gridDim.x, ...
template <class QT, int STAGE, bool PERSIST>
__global__ __launch_bounds__(kBlock) void k_pp2(DevMesh m, DevState s, Params p, CSt<QT> win,
                                                Rec2<QT> *__restrict__ out, int slot) {
  if constexpr (PERSIST) {
    for (int b = blockIdx.x; b < m.nch; b += gridDim.x)
      pp2_chunk<QT, STAGE>(m, s, p, win, out, slot, chunk_of_block(b, m.nch));
  } else {
    const int c = chunk_of_block(blockIdx.x, m.nch);
    if (c < 0) return;
    pp2_chunk<QT, STAGE>(m, s, p, win, out, slot, c);
  }
}

// One RK stage (rhs2_chunk), one chunk per workgroup or persistent as
// k_pp2; WPE: minimum waves per SIMD the register allocation is held to.
template <class QT, int WPE, bool PERSIST, bool MF = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WPE))) void k_rhs2(
    DevMesh m, DevState s, Params p, const Rec2<QT> *__restrict__ u, const Rec2<QT> *__restrict__ base, St<QT> wout,
    StageCoef sc, int slot, int want_dt) {
  extern __shared__ double lds2_raw[];
  __shared__ double red[kBlock / 64];
  if constexpr (PERSIST) {
    for (int b = blockIdx.x; b < m.nch; b += gridDim.x) {
      rhs2_chunk<QT>(m, s, p, u, base, wout, sc, slot, want_dt, chunk_of_block(b, m.nch), lds2_raw, red);
      __syncthreads();  // the next chunk overwrites the LDS
    }
  } else {
    const int c = chunk_of_block(blockIdx.x, m.nch);
    if (c < 0) return;
    rhs2_chunk<QT, MF>(m, s, p, u, base, wout, sc, slot, want_dt, c, lds2_raw, red);
  }
}

// elements [e0, e0 + count) of a state (post-processed if pp) as FP64
// [18][count], for read-back
template <class QT>
__global__ __launch_bounds__(kBlock) void k_post_only2(DevMesh m, Params p, CSt<QT> win, int pp, int e0, int count,
                                                       double *__restrict__ wout, const int *__restrict__ perm) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  double u[18];
  load_pp2<QT>(m, p, win, e0 + i, pp != 0, u);
  const int c = perm ? perm[e0 + i] : i;
  for (int j = 0; j < 18; ++j) wout[(size_t)j * count + c] = u[j];
}

// ---------------------------------------------------------------- launchers
// register budget of k_rhs2 (waves per SIMD), overridable with the
// environment variable DGSWE_RHS2_WPE = 1..4
constexpr int kRhs2WpeFp64 = 3, kRhs2WpeMixed = 2;

static inline unsigned nblk2(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <class QT>
static void stage2_qt(const DevMesh &m, const DevState &s, const Params &p, const void *win, void *rec,
                      const void *rbase, void *wout, int slot, int stage, const StageCoef &sc, int want_dt,
                      hipStream_t st, bool pp_only, bool rhs_only) {
  const size_t ne = (size_t)m.ne;
  const CSt<QT> a = {(const double *)win, (const QT *)((const double *)win + 6 * ne)};
  const St<QT> o = {(double *)wout, (QT *)((double *)wout + 6 * ne)};
  Rec2<QT> *r = (Rec2<QT> *)rec;
  const Rec2<QT> *b = (const Rec2<QT> *)rbase;
  if (!rhs_only) {
    const dim3 g(stage_grid(p, m.nch));
    if (p.persistent > 0) {
      if (stage) hipLaunchKernelGGL((k_pp2<QT, 1, true>), g, dim3(kBlock), 0, st, m, s, p, a, r, slot);
      else hipLaunchKernelGGL((k_pp2<QT, 0, true>), g, dim3(kBlock), 0, st, m, s, p, a, r, slot);
    } else {
      if (stage) hipLaunchKernelGGL((k_pp2<QT, 1, false>), g, dim3(kBlock), 0, st, m, s, p, a, r, slot);
      else hipLaunchKernelGGL((k_pp2<QT, 0, false>), g, dim3(kBlock), 0, st, m, s, p, a, r, slot);
    }
  }
  if (!pp_only) {
    static const int wpe_env = [] {
      const char *ev = std::getenv("DGSWE_RHS2_WPE");
      const int w = ev ? std::atoi(ev) : 0;
      return (w >= 1 && w <= 4) ? w : 0;
    }();
    const int wpe = wpe_env ? wpe_env : (p.waves ? p.waves : (sizeof(QT) == 8 ? kRhs2WpeFp64 : kRhs2WpeMixed));
    // the momentum at the area points on the matrix cores (a measured
    // variant; one workgroup per chunk only)
    const bool mf = p.rhs2_mfma != 0 && p.persistent <= 0;
    const size_t lds = mf ? std::max(lds2_bytes<QT>(m.ed_max), mfma_scratch_bytes<QT>()) : lds2_bytes<QT>(m.ed_max);
#define DGSWE_RHS2(W)                                                                                           \
  do {                                                                                                          \
    if (p.persistent > 0)                                                                                       \
      hipLaunchKernelGGL((k_rhs2<QT, W, true>), dim3(stage_grid(p, m.nch)), dim3(kBlock), lds, st, m, s, p, r, b, o, \
                         sc, slot, want_dt);                                                                    \
    else if (mf)                                                                                                \
      hipLaunchKernelGGL((k_rhs2<QT, W, false, true>), dim3(m.nch), dim3(kBlock), lds, st, m, s, p, r, b, o, sc,    \
                         slot, want_dt);                                                                        \
    else                                                                                                        \
      hipLaunchKernelGGL((k_rhs2<QT, W, false>), dim3(m.nch), dim3(kBlock), lds, st, m, s, p, r, b, o, sc, slot,   \
                         want_dt);                                                                              \
  } while (0)
    switch (wpe) {
      case 1: DGSWE_RHS2(1); break;
      case 2: DGSWE_RHS2(2); break;
      case 3: DGSWE_RHS2(3); break;
      default: DGSWE_RHS2(4); break;
    }
#undef DGSWE_RHS2
  }
}

hipError_t launch_pp2(const DevMesh &m, const DevState &s, const Params &p, const void *win, void *rec, int slot,
                      int stage, int precision, hipStream_t st) {
  const StageCoef none{0.0, 1.0, 1.0, 0.0, 0};
  if (precision == DGSWE_MIXED)
    stage2_qt<float>(m, s, p, win, rec, nullptr, nullptr, slot, stage, none, 0, st, true, false);
  else
    stage2_qt<double>(m, s, p, win, rec, nullptr, nullptr, slot, stage, none, 0, st, true, false);
  return hipGetLastError();
}

hipError_t launch_rhs2(const DevMesh &m, const DevState &s, const Params &p, const void *rec, const void *rbase,
                       void *wout, int slot, int first, const StageCoef &sc, int want_dt, int precision,
                       hipStream_t st) {
  // the RK base is read only by stages that combine with it
  const void *b = sc.a != 0.0 ? rbase : nullptr;
  if (precision == DGSWE_MIXED)
    stage2_qt<float>(m, s, p, nullptr, (void *)rec, b, wout, slot, first ? 0 : 1, sc, want_dt, st, false, true);
  else
    stage2_qt<double>(m, s, p, nullptr, (void *)rec, b, wout, slot, first ? 0 : 1, sc, want_dt, st, false, true);
  return hipGetLastError();
}

hipError_t launch_post_only2(const DevMesh &m, const Params &p, const void *win, int pp, int e0, int count,
                             double *wout, const int *perm, int precision, hipStream_t st) {
  const size_t ne = (size_t)m.ne;
  if (count <= 0) return hipSuccess;
  if (precision == DGSWE_MIXED)
    hipLaunchKernelGGL(k_post_only2<float>, dim3(nblk2(count)), dim3(kBlock), 0, st, m, p,
                       CSt<float>{(const double *)win, (const float *)((const double *)win + 6 * ne)}, pp, e0, count,
                       wout, perm);
  else
    hipLaunchKernelGGL(k_post_only2<double>, dim3(nblk2(count)), dim3(kBlock), 0, st, m, p,
                       CSt<double>{(const double *)win, (const double *)win + 6 * ne}, pp, e0, count, wout, perm);
  return hipGetLastError();
}

}  // namespace dgswe
