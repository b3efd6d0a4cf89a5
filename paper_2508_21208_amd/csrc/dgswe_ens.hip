// One launch per RK stage for an ensemble whose members have both orders:
// a p = 1 batch and a p = 2 batch (Sec. 2.2: the method carries to higher
// degrees; the members are independent meshes) advanced by the same kernel.
// A work item is a chunk of the p = 1 batch (its whole stage, the fused LDS
// kernel's work) or of the p = 2 batch (its edge pass and element
// integrals; the p = 2 records of the stage input are made by k_pp2
// before).  Each XCD takes the same share of both kinds (item12_of_block);
// with persistent workgroups each takes items b, b + gridDim.x, ...  Each
// chunk's arithmetic is that of its own batch's kernel, so every member's
// result is bitwise the one of its batch stepped alone.
#include "dgswe_p1.h"
#include "dgswe_p2.h"

namespace dgswe {

// Work items of both batches per XCD: XCD x (workgroups b with b % 8 = x)
// takes its contiguous eighth of the p = 1 chunks, then its eighth of the
// p = 2 chunks, so every XCD gets the same mix of the two kinds of work
// (whose costs differ about 2.6x) and neighbouring chunks share its L2.
__host__ __device__ __forceinline__ int stage12_items(int n1, int n2) {
  return 8 * ((n1 + 7) / 8 + (n2 + 7) / 8);
}
__device__ __forceinline__ int item12_of_block(int b, int n1, int n2, int &c) {
  const int x = b % 8, r = b / 8;
  const int per1 = n1 / 8, rem1 = n1 % 8, per2 = n2 / 8, rem2 = n2 % 8;
  const int len1 = per1 + (x < rem1 ? 1 : 0), len2 = per2 + (x < rem2 ? 1 : 0);
  if (r < len1) {
    c = x * per1 + (x < rem1 ? x : rem1) + r;
    return 1;
  }
  if (r < len1 + len2) {
    c = x * per2 + (x < rem2 ? x : rem2) + r - len1;
    return 2;
  }
  return 0;  // no item: a workgroup of the last row of an XCD with fewer items
}

template <class QT, int STAGE, int WPE, bool PERSIST>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WPE))) void k_stage12(
    DevMesh m1, DevState s1, Params p1, CSt<QT> win1, CSt<QT> wbase1, St<QT> wout1, St<QT> wpp1, int slot1,
    int want_dt1, DevMesh m2, DevState s2, Params p2, const Rec2<QT> *__restrict__ rec2,
    const Rec2<QT> *__restrict__ base2, St<QT> wout2, int slot2, int want_dt2, StageCoef sc) {
  extern __shared__ double lds_raw[];
  __shared__ double red[kBlock / 64];
  const int nw = stage12_items(m1.nch, m2.nch);
  auto item = [&](int b) {
    int c = 0;
    const int which = item12_of_block(b, m1.nch, m2.nch, c);
    if (which == 1)
      // (phase A's nodal forcing loaded in phase A: the p = 2 work shares
      // the registers)
      stage1_chunk<kBlock, QT, STAGE, false, false>(m1, s1, p1, win1, wbase1, wout1, wpp1, sc, slot1, want_dt1, c,
                                                    lds_raw, red);
    else if (which == 2)
      rhs2_chunk<QT>(m2, s2, p2, rec2, base2, wout2, sc, slot2, want_dt2, c, lds_raw, red);
  };
  if constexpr (PERSIST) {
    for (int b = blockIdx.x; b < nw; b += gridDim.x) {
      item(b);
      __syncthreads();  // the next item overwrites the LDS
    }
  } else {
    item(blockIdx.x);
  }
}

// The other split of a stage of both orders: the p = 1 stage of every p = 1
// chunk together with the post-processing of every p = 2 chunk (k_pp2's
// work: independent of each other, so the streaming post-processing shares
// the compute units with the p = 1 stage), then the p = 2 right-hand side
// alone (k_rhs2).
template <class QT, int STAGE, int WPE, bool PERSIST>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WPE))) void k_stage1pp2(
    DevMesh m1, DevState s1, Params p1, CSt<QT> win1, CSt<QT> wbase1, St<QT> wout1, St<QT> wpp1, int slot1,
    int want_dt1, DevMesh m2, DevState s2, Params p2, CSt<QT> win2, Rec2<QT> *__restrict__ rec2, int slot2,
    StageCoef sc) {
  extern __shared__ double lds_raw[];
  __shared__ double red[kBlock / 64];
  const int nw = stage12_items(m1.nch, m2.nch);
  auto item = [&](int b) {
    int c = 0;
    const int which = item12_of_block(b, m1.nch, m2.nch, c);
    if (which == 1)
      // (phase A's nodal forcing loaded in phase A: the p = 2 work shares
      // the registers)
      stage1_chunk<kBlock, QT, STAGE, false, false>(m1, s1, p1, win1, wbase1, wout1, wpp1, sc, slot1, want_dt1, c,
                                                    lds_raw, red);
    else if (which == 2)
      pp2_chunk<QT, STAGE>(m2, s2, p2, win2, rec2, slot2, c);
  };
  if constexpr (PERSIST) {
    for (int b = blockIdx.x; b < nw; b += gridDim.x) {
      item(b);
      __syncthreads();  // the next item overwrites the LDS
    }
  } else {
    item(blockIdx.x);
  }
}

template <class QT>
static hipError_t stage1pp2_qt(const DevMesh &m1, const DevState &s1, const Params &p1, const void *win1,
                               const void *wbase1, void *wout1, void *wpp1, int slot1, int want_dt1,
                               const DevMesh &m2, const DevState &s2, const Params &p2, const void *win2, void *rec2,
                               int slot2, int first, const StageCoef &sc, hipStream_t st) {
  const size_t lds = lds_bytes<QT>(m1);
  const CSt<QT> a = csplit<QT>(win1, (size_t)m1.ne);
  const CSt<QT> b = wbase1 ? csplit<QT>(wbase1, (size_t)m1.ne) : CSt<QT>{nullptr, nullptr};
  const St<QT> o = split<QT>(wout1, (size_t)m1.ne);
  const St<QT> q = wpp1 ? split<QT>(wpp1, (size_t)m1.ne) : St<QT>{nullptr, nullptr};
  const size_t ne2 = (size_t)m2.ne;
  const CSt<QT> a2 = {(const double *)win2, (const QT *)((const double *)win2 + 6 * ne2)};
  Rec2<QT> *r2 = (Rec2<QT> *)rec2;
  const unsigned grid = stage_grid(p1, stage12_items(m1.nch, m2.nch));
#define DGSWE_S1PP2(S, P)                                                                                          \
  hipLaunchKernelGGL((k_stage1pp2<QT, S, 2, P>), dim3(grid), dim3(kBlock), lds, st, m1, s1, p1, a, b, o, q, slot1, \
                     want_dt1, m2, s2, p2, a2, r2, slot2, sc)
  if (p1.persistent > 0) {
    if (first) DGSWE_S1PP2(0, true);
    else DGSWE_S1PP2(1, true);
  } else {
    if (first) DGSWE_S1PP2(0, false);
    else DGSWE_S1PP2(1, false);
  }
#undef DGSWE_S1PP2
  return hipGetLastError();
}

hipError_t launch_stage1pp2(const DevMesh &m1, const DevState &s1, const Params &p1, const void *win1,
                            const void *wbase1, void *wout1, void *wpp1, int slot1, int want_dt1, const DevMesh &m2,
                            const DevState &s2, const Params &p2, const void *win2, void *rec2, int slot2, int first,
                            const StageCoef &sc, int precision, hipStream_t st) {
  if (precision == DGSWE_MIXED)
    return stage1pp2_qt<float>(m1, s1, p1, win1, wbase1, wout1, wpp1, slot1, want_dt1, m2, s2, p2, win2, rec2, slot2,
                               first, sc, st);
  return stage1pp2_qt<double>(m1, s1, p1, win1, wbase1, wout1, wpp1, slot1, want_dt1, m2, s2, p2, win2, rec2, slot2,
                              first, sc, st);
}

template <class QT>
static hipError_t stage12_qt(const DevMesh &m1, const DevState &s1, const Params &p1, const void *win1,
                             const void *wbase1, void *wout1, void *wpp1, int slot1, int want_dt1, const DevMesh &m2,
                             const DevState &s2, const Params &p2, const void *rec2, const void *base2, void *wout2,
                             int slot2, int want_dt2, int first, const StageCoef &sc, hipStream_t st) {
  const size_t lds = std::max(lds_bytes<QT>(m1), lds2_bytes<QT>(m2.ed_max));
  const CSt<QT> a = csplit<QT>(win1, (size_t)m1.ne);
  const CSt<QT> b = wbase1 ? csplit<QT>(wbase1, (size_t)m1.ne) : CSt<QT>{nullptr, nullptr};
  const St<QT> o = split<QT>(wout1, (size_t)m1.ne);
  const St<QT> q = wpp1 ? split<QT>(wpp1, (size_t)m1.ne) : St<QT>{nullptr, nullptr};
  const size_t ne2 = (size_t)m2.ne;
  const St<QT> o2 = {(double *)wout2, (QT *)((double *)wout2 + 6 * ne2)};
  const Rec2<QT> *r2 = (const Rec2<QT> *)rec2, *b2 = (const Rec2<QT> *)base2;
  const unsigned grid = stage_grid(p1, stage12_items(m1.nch, m2.nch));
#define DGSWE_STAGE12(S, P)                                                                                       \
  hipLaunchKernelGGL((k_stage12<QT, S, 2, P>), dim3(grid), dim3(kBlock), lds, st, m1, s1, p1, a, b, o, q, slot1,  \
                     want_dt1, m2, s2, p2, r2, b2, o2, slot2, want_dt2, sc)
  if (p1.persistent > 0) {
    if (first) DGSWE_STAGE12(0, true);
    else DGSWE_STAGE12(1, true);
  } else {
    if (first) DGSWE_STAGE12(0, false);
    else DGSWE_STAGE12(1, false);
  }
#undef DGSWE_STAGE12
  return hipGetLastError();
}

hipError_t launch_stage12(const DevMesh &m1, const DevState &s1, const Params &p1, const void *win1,
                          const void *wbase1, void *wout1, void *wpp1, int slot1, int want_dt1, const DevMesh &m2,
                          const DevState &s2, const Params &p2, const void *rec2, const void *base2, void *wout2,
                          int slot2, int want_dt2, int first, const StageCoef &sc, int precision, hipStream_t st) {
  if (precision == DGSWE_MIXED)
    return stage12_qt<float>(m1, s1, p1, win1, wbase1, wout1, wpp1, slot1, want_dt1, m2, s2, p2, rec2, base2, wout2,
                             slot2, want_dt2, first, sc, st);
  return stage12_qt<double>(m1, s1, p1, win1, wbase1, wout1, wpp1, slot1, want_dt1, m2, s2, p2, rec2, base2, wout2,
                            slot2, want_dt2, first, sc, st);
}

}  // namespace dgswe
