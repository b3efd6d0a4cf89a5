// Device code of the p = 2 stage (basis, records, post-processing, the edge
// pass and the element integrals, and the two kernels' work on one chunk),
// shared by the p = 2 kernels and the kernel that advances members of both
// orders in one launch.  See dgswe_p2.hip for the design.
#pragma once
#include "dgswe_device.h"

namespace dgswe {

// ---------------------------------------------------------------- basis
// Dubiner p = 2 in the order [phi00, phi10, phi01, phi20, phi11, phi02] with
// A = (1 + 2 xi + eta)/2, B = (1 - eta)/2: phi10 = A, phi01 = (1 + 3 eta)/2,
// phi20 = (3 A^2 - B^2)/2, phi11 = A (3 + 5 eta)/2, phi02 = (5 eta^2 + 2 eta - 1)/2.
HD void basis2(double xi, double eta, double f[6]) {
  const double A = 0.5 * (1.0 + 2.0 * xi + eta), B = 0.5 * (1.0 - eta);
  f[0] = 1.0;
  f[1] = A;
  f[2] = 0.5 * (1.0 + 3.0 * eta);
  f[3] = 0.5 * (3.0 * A * A - B * B);
  f[4] = 0.5 * A * (3.0 + 5.0 * eta);
  f[5] = 0.5 * (5.0 * eta * eta + 2.0 * eta - 1.0);
}
// reference gradients (d/dxi, d/deta)
HD void basis2_grad(double xi, double eta, double d[6][2]) {
  const double A = 0.5 * (1.0 + 2.0 * xi + eta), B = 0.5 * (1.0 - eta);
  d[0][0] = 0.0; d[0][1] = 0.0;
  d[1][0] = 1.0; d[1][1] = 0.5;
  d[2][0] = 0.0; d[2][1] = 1.5;
  d[3][0] = 3.0 * A; d[3][1] = 0.5 * (3.0 * A + B);
  d[4][0] = 0.5 * (3.0 + 5.0 * eta); d[4][1] = 0.25 * (3.0 + 5.0 * eta) + 2.5 * A;
  d[5][0] = 0.0; d[5][1] = 5.0 * eta + 1.0;
}

// mass diagonal / area and its inverse
constexpr double kMu2Inv[6] = {1.0, 6.0, 2.0, 15.0, 9.0, 3.0};

// values of the six modes at the vertices V0 (-1,-1), V1 (1,-1), V2 (-1,1)
// and at the midpoints of local edges 0, 1, 2 (opposite V0, V1, V2)
constexpr double kPt6[6][6] = {
    {1.0, -1.0, -1.0, 1.0, 1.0, 1.0},   {1.0, 1.0, -1.0, 1.0, -1.0, 1.0},   {1.0, 0.0, 2.0, 0.0, 0.0, 3.0},
    {1.0, 0.5, 0.5, 0.25, 0.75, -0.5}, {1.0, -0.5, 0.5, 0.25, -0.75, -0.5}, {1.0, 0.0, -1.0, -0.5, 0.0, 1.0}};

// degree-4 symmetric area rule: barycentric (a, b, b) and permutations,
// weights as fractions of the area
constexpr double kD4A1 = 0.10810301816807022736, kD4B1 = 0.44594849091596488632, kD4W1 = 0.22338158967801146570;
constexpr double kD4A2 = 0.81684757298045851308, kD4B2 = 0.09157621350977074346, kD4W2 = 0.10995174365532186764;
HD void area_point2(int q, double L[3], double &w) {
  const bool o1 = q < 3;
  const int r = o1 ? q : q - 3;
  const double a = o1 ? kD4A1 : kD4A2, b = o1 ? kD4B1 : kD4B2;
  for (int v = 0; v < 3; ++v) L[v] = v == r ? a : b;
  w = o1 ? kD4W1 : kD4W2;
}

// 4-point Gauss-Lobatto rule on [-1, 1]: nodes -1, -1/sqrt5, 1/sqrt5, 1,
// weights 1/6, 5/6, 5/6, 1/6
constexpr double kGL4S = 0.44721359549995793928;
HD double gl4_s(int g) { return g == 0 ? -1.0 : (g == 1 ? -kGL4S : (g == 2 ? kGL4S : 1.0)); }
HD double gl4_w(int g) { return (g == 0 || g == 3) ? (1.0 / 6.0) : (5.0 / 6.0); }

// reference point at parameter s of local edge l (from vertex l+1 at s = -1
// to vertex l+2 at s = +1)
HD void edge_point2(int l, double s, double &xi, double &eta) {
  const int a = l == 2 ? 0 : l + 1, b = l == 0 ? 2 : l - 1;
  const double ax = a == 1 ? 1.0 : -1.0, ay = a == 2 ? 1.0 : -1.0;
  const double bx = b == 1 ? 1.0 : -1.0, by = b == 2 ? 1.0 : -1.0;
  xi = ax * 0.5 * (1.0 - s) + bx * 0.5 * (1.0 + s);
  eta = ay * 0.5 * (1.0 - s) + by * 0.5 * (1.0 + s);
}

// packed ids stored in the low bits of a double / in a float
HD uint32_t info_bits(double v) {
  union { double d; unsigned long long u; } x;
  x.d = v;
  return (uint32_t)x.u;
}
HD uint32_t info_bits(float v) {
  union { float f; uint32_t u; } x;
  x.f = v;
  return x.u;
}

// ---------------------------------------------------------------- records
// post-processed state of one element: zeta modes (FP64), Qx modes, Qy modes
template <class QT>
struct alignas(16) Rec2 {
  double z[6];
  QT q[12];
};
static_assert(sizeof(Rec2<double>) == 144, "FP64 record");
static_assert(sizeof(Rec2<float>) == 96, "mixed record");

template <class QT>
HD void load_rec(const Rec2<QT> *__restrict__ r, int e, double z[6], QT q[12]) {
  const double2 *d = (const double2 *)(r + e);
  for (int j = 0; j < 3; ++j) {
    const double2 v = d[j];
    z[2 * j] = v.x;
    z[2 * j + 1] = v.y;
  }
  if constexpr (sizeof(QT) == 8) {
    for (int j = 0; j < 6; ++j) {
      const double2 v = d[3 + j];
      q[2 * j] = (QT)v.x;
      q[2 * j + 1] = (QT)v.y;
    }
  } else {
    const float4 *f = (const float4 *)(d + 3);
    for (int j = 0; j < 3; ++j) {
      const float4 v = f[j];
      q[4 * j] = (QT)v.x; q[4 * j + 1] = (QT)v.y; q[4 * j + 2] = (QT)v.z; q[4 * j + 3] = (QT)v.w;
    }
  }
}

template <class QT>
HD void store_rec(Rec2<QT> *__restrict__ r, int e, const double u[18]) {
  double2 *d = (double2 *)(r + e);
  for (int j = 0; j < 3; ++j) d[j] = make_double2(u[2 * j], u[2 * j + 1]);
  if constexpr (sizeof(QT) == 8) {
    for (int j = 0; j < 6; ++j) d[3 + j] = make_double2(u[6 + 2 * j], u[7 + 2 * j]);
  } else {
    float4 *f = (float4 *)(d + 3);
    for (int j = 0; j < 3; ++j)
      f[j] = make_float4((float)u[6 + 4 * j], (float)u[7 + 4 * j], (float)u[8 + 4 * j], (float)u[9 + 4 * j]);
  }
}

// ---------------------------------------------------------------- post-processing
// Reference coordinates of the points at which a stage evaluates an
// element's state: i = 0..2 the vertices, 3..8 the two interior
// Gauss-Lobatto points of each edge (edge (i-3)/2, s = -+1/sqrt5), 9..14
// the six area points.  With constant i (unrolled loops) it folds away.
HD void depth_point2(int i, double &xi, double &eta) {
  if (i < 3) {
    xi = i == 1 ? 1.0 : -1.0;
    eta = i == 2 ? 1.0 : -1.0;
  } else if (i < 9) {
    edge_point2((i - 3) >> 1, ((i - 3) & 1) ? kGL4S : -kGL4S, xi, eta);
  } else {
    double L[3], w;
    area_point2(i - 9, L, w);
    xi = -L[0] + L[1] - L[2];
    eta = -L[0] - L[1] + L[2];
  }
}

// Post-processing of one element, FP64: u[18] = zeta, Qx, Qy modes
// [var * 6 + mode] of the raw state; nbm[v][k] the raw mean of variable v of
// neighbour k.  Both steps keep the means and are continuous in their
// inputs, so rounding-level input changes (FP32 momentum) move the output
// at rounding level only.
//   Limiter, per variable: with [lo, hi] the range of the element's and its
//   neighbours' means and d the deviations of the field from its mean at
//   the vertices and the edge midpoints, modes 1-5 are scaled by the
//   largest theta <= 1 that keeps mean + theta d inside [lo, hi] (a linear
//   field gives the p = 1 Barth-Jespersen factor).
//   Wet/dry: mean depth <= H0 -> flat at the mean depth, momentum 0; else
//   if the depth falls below H0 at a vertex, an interior edge quadrature
//   point or an area point, the depth's deviation from its mean (modes 1-5
//   of zeta plus the bed's linear modes) is scaled by (Hm - H0)/(Hm - Hmin),
//   which lifts the lowest of those points to H0; momentum unchanged.
HD void postprocess2(double u[18], const double nbm[3][3], const bool has[3], const double h[3], double hmean,
                     const Params &p) {
  if (p.limiter) {
    for (int v = 0; v < 3; ++v) {
      double *w = u + 6 * v;
      const double mean = w[0];
      double hi = mean, lo = mean;
      for (int k = 0; k < 3; ++k)
        if (has[k]) { hi = fmax(hi, nbm[v][k]); lo = fmin(lo, nbm[v][k]); }
      double dmax = 0.0, dmin = 0.0;
      for (int i = 0; i < 6; ++i) {
        double d = 0.0;
        for (int k = 1; k < 6; ++k) d += w[k] * kPt6[i][k];
        dmax = fmax(dmax, d);
        dmin = fmin(dmin, d);
      }
      double theta = 1.0;
      if (dmax > 0.0 && hi - mean < dmax) theta = fmin(theta, (hi - mean) / dmax);
      if (dmin < 0.0 && lo - mean > dmin) theta = fmin(theta, (lo - mean) / dmin);
      if (theta < 1.0)
        for (int k = 1; k < 6; ++k) w[k] *= theta;
    }
  }
  if (p.wetdry) {
    const double Hm = u[0] + hmean;
    const double b1 = 0.5 * (h[1] - h[0]), b2 = 0.5 * (h[2] - hmean);
    if (Hm <= p.h0) {
      u[1] = -b1; u[2] = -b2;
      u[3] = 0.0; u[4] = 0.0; u[5] = 0.0;
      for (int j = 6; j < 18; ++j) u[j] = 0.0;
    } else {
      const double H[6] = {0.0, u[1] + b1, u[2] + b2, u[3], u[4], u[5]};
      double dmin = 0.0;
#pragma unroll
      for (int i = 0; i < 15; ++i) {
        double xi, eta, f[6];
        depth_point2(i, xi, eta);
        basis2(xi, eta, f);
        double d = 0.0;
        for (int k = 1; k < 6; ++k) d += H[k] * f[k];
        dmin = fmin(dmin, d);
      }
      if (Hm + dmin < p.h0) {
        const double theta = (Hm - p.h0) / (-dmin);
        u[1] = theta * H[1] - b1;
        u[2] = theta * H[2] - b2;
        for (int k = 3; k < 6; ++k) u[k] = theta * H[k];
      }
    }
  }
}

// raw element e of a state (structure of arrays: zeta [6][ne], Qx [6][ne],
// Qy [6][ne]) as FP64 u[18], post-processed if pp with raw neighbour means
template <class QT>
HD void load_pp2(const DevMesh &m, const Params &p, CSt<QT> w, int e, bool pp, double u[18]) {
  const size_t ne = (size_t)m.ne;
  for (int k = 0; k < 6; ++k) u[k] = w.z[k * ne + e];
  for (int k = 0; k < 12; ++k) u[6 + k] = (double)w.q[k * ne + e];
  if (!pp) return;
  double h[3], nbm[3][3];
  bool has[3];
  for (int k = 0; k < 3; ++k) h[k] = m.hbv[k * ne + e];
  for (int k = 0; k < 3; ++k) {
    const int f = m.el_nb[k * ne + e];
    has[k] = f >= 0;
    const int fi = has[k] ? f : e;
    nbm[0][k] = w.z[fi];
    nbm[1][k] = (double)w.q[fi];
    nbm[2][k] = (double)w.q[6 * ne + fi];
  }
  postprocess2(u, nbm, has, h, mean3(h), p);
}

// ---------------------------------------------------------------- edge
// Traces of an element's modes (z, q) at the four points of its local edge
// l; rev: the points in the opposite direction (the e- side of an edge).
template <class QT>
HD void traces_from(const double z[6], const QT q[12], int l, bool rev, double tz[4], QT tx[4], QT ty[4]) {
  for (int g = 0; g < 4; ++g) {
    double xi, eta, f[6];
    edge_point2(l, rev ? -gl4_s(g) : gl4_s(g), xi, eta);
    basis2(xi, eta, f);
    double sz = 0.0;
    QT sx = (QT)0, sy = (QT)0;
    for (int k = 0; k < 6; ++k) {
      const QT fk = (QT)f[k];
      sz += z[k] * f[k];
      sx += q[k] * fk;
      sy += q[6 + k] * fk;
    }
    tz[g] = sz; tx[g] = sx; ty[g] = sy;
  }
}

// bathymetry at point g of an edge with end values hA (s = -1), hB (s = +1)
HD double edge_hb(double hA, double hB, int g) {
  return hA * 0.5 * (1.0 - gl4_s(g)) + hB * 0.5 * (1.0 + gl4_s(g));
}

// Flux kinds of an edge (wet/dry rules as for p = 1): LLF to both sides (e+
// gets F, e- gets -F), LLF to e+ only (ocean ghost), land or no-flood wall
// of e+, no-flood wall of e- (normal -n), nothing.
enum EdgeKind { EK_LLF = 0, EK_LLF_P, EK_WALL_P, EK_WALL_M, EK_NONE };

// ---------------------------------------------------------------- edges in LDS
// The right-hand side works per chunk: every chunk-local edge (the edges
// touching the chunk's elements, chunk-border edges included) is evaluated
// once, by one lane, into LDS; then each chunk element integrates its three
// edges from there.  A border edge is evaluated by both chunks it touches,
// with the same instructions on the same records, so both sides get bitwise
// the same flux.  Per edge: the flux at the four Gauss-Lobatto points that
// its receiving side(s) integrate, in the edge's orientation (zeta part
// FP64 holding the QT value, momentum in QT), half its length, its kind.
template <class QT>
struct Lds2 {
  double *fz;           // [4][eds]
  double *hl;           // [eds]
  QT *fq;               // [8][eds]: x flux at g = 0..3, then y
  unsigned char *kind;  // [eds]
  int eds;
};

template <class QT>
HD size_t lds2_bytes(int ed_max) {
  return (size_t)ed_max * (5 * sizeof(double) + 8 * sizeof(QT) + 1);
}

template <class QT>
HD Lds2<QT> lds2_view(int ed_max, void *base) {
  Lds2<QT> L;
  L.eds = ed_max;
  L.fz = (double *)base;
  L.hl = L.fz + 4 * (size_t)ed_max;
  L.fq = (QT *)(L.hl + (size_t)ed_max);
  L.kind = (unsigned char *)(L.fq + 8 * (size_t)ed_max);
  return L;
}

// the record of chunk-local edge j: normal, half length, packed ids and
// the global ids of its two sides
template <class QT>
struct Edge2In {
  QT nx, ny;
  double hl;
  uint32_t ids;
  int gp, gm;
};

template <class QT>
HD Edge2In<QT> load_edge2(const DevMesh &m, const ChunkInfo &k, int j) {
  const size_t r = (size_t)(k.leo + j);
  Edge2In<QT> E;
  if constexpr (sizeof(QT) == 8) {
    const double2 a = m.le_a[r], b = m.le_b[r];
    E.nx = a.x; E.ny = a.y; E.hl = b.x;
    E.ids = info_bits(b.y);
  } else {
    const float4 a = m.le_f[r];
    E.nx = a.x; E.ny = a.y; E.hl = (double)a.z;
    E.ids = info_bits(a.w);
  }
  const int2 g = m.le_g[r];
  E.gp = g.x;
  E.gm = g.y;  // = gp on a boundary edge
  return E;
}

// Chunk-local edge j (record E): both sides' traces from the records, the
// wet/dry rules (as for p = 1), the flux at the four points into LDS.
template <class QT>
HD void edge_phase2(const DevMesh &m, const Params &p, const ChunkInfo &k, const Rec2<QT> *__restrict__ u,
                    double zb, int j, const Edge2In<QT> &E, const Lds2<QT> &L) {
  using R = QT;
  const R nx = E.nx, ny = E.ny;
  const double hl = E.hl;
  const uint32_t ids = E.ids;
  const int info = (int)(ids >> 24);
  const int lp = info & 3, lm = (info >> 2) & 3, type = info >> 4;
  const int ip = (int)(ids & 0xFFFu);
  const bool ghost = type != 0;
  const int gp = E.gp, gm = E.gm;
  // bathymetry at the edge ends: vertices lp+1 (s = -1) and lp+2 (s = +1) of e+
  // every load of the edge at once: both records (gm = gp on a boundary
  // edge, whose second copy goes unused), mean bathymetries, edge-end
  // bathymetry; one wait for memory instead of one per dependent step
  double zp6[6], zm6[6];
  R qp12[12], qm12[12];
  load_rec<QT>(u, gp, zp6, qp12);
  load_rec<QT>(u, gm, zm6, qm12);
  const double hmp = m.hmean[gp], hmm = m.hmean[gm];
  const double2 h01 = m.lhb01[k.lo + ip];
  const double h2 = m.lhb2[k.lo + ip];
#ifdef __HIP_DEVICE_COMPILE__
  // FP64: keep every load above the arithmetic (measured faster; in the
  // mixed path the scheduler's own order measured faster)
  if constexpr (sizeof(QT) == 8) __builtin_amdgcn_sched_barrier(0);
#endif
  const int va = lp == 2 ? 0 : lp + 1, vb = lp == 0 ? 2 : lp - 1;
  const double hA = va == 0 ? h01.x : (va == 1 ? h01.y : h2);
  const double hB = vb == 0 ? h01.x : (vb == 1 ? h01.y : h2);
  // (both candidates of wetm formed unconditionally: a select, so the
  // mean-bathymetry load is not sunk into a branch that then waits for
  // every outstanding load)
  const bool wm_in = zm6[0] + hmm > p.h0, wm_ghost = zb + 0.5 * (hA + hB) > p.h0;
  const bool wetp = p.wetdry ? (zp6[0] + hmp > p.h0) : true;
  const bool wetm = p.wetdry ? (ghost ? wm_ghost : wm_in) : true;
  // e+ and e- traces; a ghost e- side is (zeta_b, momentum of e+)
  double pz[4], mz[4];
  R px[4], py[4], mx[4], my[4];
  traces_from<QT>(zp6, qp12, lp, false, pz, px, py);
  if (ghost) {
    for (int g = 0; g < 4; ++g) { mz[g] = zb; mx[g] = px[g]; my[g] = py[g]; }
  } else {
    traces_from<QT>(zm6, qm12, lm, true, mz, mx, my);
  }
  int kind;
  if (type == DGSWE_BC_LAND) kind = EK_WALL_P;
  else if (!wetp && !wetm) kind = EK_NONE;
  else if (wetp && wetm) kind = ghost ? EK_LLF_P : EK_LLF;
  else {
    // one side dry: the sign of the LLF mass flux decides
    R mf = (R)0;
    for (int g = 0; g < 4; ++g) {
      R Fg[3];
      llf<R>(p.g, pz[g], px[g], py[g], mz[g], mx[g], my[g], edge_hb(hA, hB, g), nx, ny, wetp, wetm, Fg);
      mf += (R)gl4_w(g) * Fg[0];
    }
    const bool flood = wetp ? (mf > (R)0) : (mf < (R)0);
    kind = flood ? (ghost ? EK_LLF_P : EK_LLF) : (wetp ? EK_WALL_P : (ghost ? EK_NONE : EK_WALL_M));
  }
  for (int g = 0; g < 4; ++g) {
    R Fg[3] = {(R)0, (R)0, (R)0};
    const double hq = edge_hb(hA, hB, g);
    if (kind == EK_WALL_P) wall<R>(p.g, pz[g], px[g], py[g], hq, nx, ny, wetp, Fg);
    else if (kind == EK_WALL_M) wall<R>(p.g, mz[g], mx[g], my[g], hq, -nx, -ny, wetm, Fg);
    else if (kind == EK_NONE) {
    } else if (p.flux == 1 && wetp && wetm) roe<R>(p.g, pz[g], px[g], py[g], mz[g], mx[g], my[g], hq, nx, ny, Fg);
    else llf<R>(p.g, pz[g], px[g], py[g], mz[g], mx[g], my[g], hq, nx, ny, wetp, wetm, Fg);
    L.fz[g * L.eds + j] = (double)Fg[0];
    L.fq[g * L.eds + j] = Fg[1];
    L.fq[(4 + g) * L.eds + j] = Fg[2];
  }
  L.hl[j] = hl;
  L.kind[j] = (unsigned char)kind;
}

// ---------------------------------------------------------------- MFMA variant
// The momentum at the six area points of the 64 elements of a wavefront as
// matrix products on the matrix cores (16x16x4 MFMA, FP32 in the mixed path,
// FP64 otherwise): for each group of 16 elements, D = A B with A[point][mode]
// the basis values (6 of 16 rows, 6 of 8 modes used) and B[mode][element] the
// modes, two K-steps of 4 modes.  Lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and receives, for i = 0..3, D[4 (l / 16) + i][l % 16]
// (FP32) or D[l / 16 + 4 i][l % 16] (FP64) - the two builtins' result
// layouts differ (checked on the device) - so the modes go to the lanes
// through LDS and the point values come back the same way (S: the wave's
// modes [6][64], T: the four groups' results [4][64][4]).  Called by every
// lane of the workgroup (it has barriers).
template <class QT>
struct AreaQ {
  QT qx[6], qy[6];
};

template <class QT>
HD size_t mfma_scratch_bytes() {
  return (size_t)(kBlock / 64) * (6 * 64 + 4 * 64 * 4) * sizeof(QT);
}

template <class QT>
__device__ __forceinline__ void area_points_mfma(const Rec2<QT> *__restrict__ u, int e, void *scratch, AreaQ<QT> &P) {
#ifdef __HIP_DEVICE_COMPILE__
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  QT *S = (QT *)scratch + (size_t)wv * (6 * 64 + 4 * 64 * 4);
  QT *T = S + 6 * 64;
  double z[6];
  QT q[12];
  load_rec<QT>(u, e, z, q);
  // A values of this lane: basis mode 4 kk + r at area point c
  const int r = lane >> 4, c = lane & 15;
  double f[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (c < 6) {
    double L[3], w;
    area_point2(c, L, w);
    basis2(-L[0] + L[1] - L[2], -L[0] - L[1] + L[2], f);
  }
  const QT a0 = (QT)f[r], a1 = r < 2 ? (QT)f[4 + r] : (QT)0;
  for (int v = 0; v < 2; ++v) {
    for (int k = 0; k < 6; ++k) S[k * 64 + lane] = q[6 * v + k];
    __syncthreads();
    for (int g = 0; g < 4; ++g) {
      const int n = 16 * g + c;
      const QT b0 = S[r * 64 + n], b1 = r < 2 ? S[(4 + r) * 64 + n] : (QT)0;
      if constexpr (sizeof(QT) == 8) {
        typedef double d4 __attribute__((ext_vector_type(4)));
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc, 0, 0, 0);
        for (int i = 0; i < 4; ++i) T[(g * 64 + lane) * 4 + i] = acc[i];
      } else {
        typedef float f4 __attribute__((ext_vector_type(4)));
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc, 0, 0, 0);
        for (int i = 0; i < 4; ++i) T[(g * 64 + lane) * 4 + i] = acc[i];
      }
    }
    __syncthreads();
    // this lane's element is n = lane of group g = lane / 16, column lane % 16
    const int g = lane >> 4, j = lane & 15;
    QT *out = v == 0 ? P.qx : P.qy;
    for (int pt = 0; pt < 6; ++pt) {
      // the lane and register holding row pt, column j of this group's D
      const int src = sizeof(QT) == 8 ? j + 16 * (pt & 3) : j + 16 * (pt >> 2);
      const int reg = sizeof(QT) == 8 ? pt >> 2 : pt & 3;
      out[pt] = T[(g * 64 + src) * 4 + reg];
    }
    __syncthreads();
  }
#else
  (void)u; (void)e; (void)scratch; (void)P;
#endif
}

// ---------------------------------------------------------------- one chunk
// Post-processing of one stage input into records.  The first stage also
// does the step's bookkeeping: ALLDRY when no time step is defined, and the
// reset of the next step's CFL minimum.
template <class QT, int STAGE>
__device__ __forceinline__ void pp2_chunk(DevMesh m, DevState s, Params p, CSt<QT> win, Rec2<QT> *__restrict__ out,
                                          int slot, int c) {
  const ChunkInfo k = chunk_info(m, c);
  Ctrl *ctl = s.ctrl + k.member;
  const int i = threadIdx.x;
  const int status = ctl->status;
  const unsigned long long dtbits = ctl->dtmin[slot];
  const int pp_in = STAGE == 0 ? ctl->pp_in : 1;
  double dt;
  if (status != 0) return;
  if (!dt_from_bits(p, dtbits, dt)) {
    if (STAGE == 0 && k.first && i == 0) atomicCAS(&ctl->status, 0, (int)DGSWE_E_ALLDRY);
    return;
  }
  if (STAGE == 0 && k.first && i == 0) ctl->dtmin[slot ^ 1] = double_to_bits(INFINITY);
  if (i >= k.cc) return;
  const int e = k.c0 + i;
  double u[18];
  load_pp2<QT>(m, p, win, e, pp_in != 0, u);
  store_rec<QT>(out, e, u);
}

// One RK stage of chunk element i from the post-processed records u (and,
// in the second stage, the RK base records): out = u + dt L(u), or
// 1/2 base + 1/2 (u + dt L(u)); zeta modes in out, momentum modes in oqv,
// the CFL candidate of the result in cand.  Returns false on a non-finite
// result.
template <class QT, bool MF = false>
HD bool rhs2_element(const DevMesh &m, const DevState &s, const Params &p, const ChunkInfo &k, const Member &F,
                     const Rec2<QT> *__restrict__ u, const Rec2<QT> *__restrict__ base, const StageCoef &sc, int i,
                     const Lds2<QT> &L, double out[6], QT oqv[12], double &cand, double dt,
                     const AreaQ<QT> *AQ = nullptr) {
  using R = QT;
  const size_t ne = (size_t)m.ne;
  const int e = k.c0 + i;

  // every load that needs no index first (own record, vertex bathymetry,
  // area, gradients, node ids and edge codes, Manning n), then the nodal
  // forcing through the node ids: two waits for memory
  double z[6];
  R q[12];
  load_rec<QT>(u, e, z, q);
  double h[3];
  for (int j = 0; j < 3; ++j) h[j] = m.hbv[j * ne + e];
  const double2 ai = m.eai[e];
  R g1x, g1y, g2x, g2y;
  if constexpr (sizeof(QT) == 8) {
    const double2 a = m.eg1[e], b = m.eg2[e];
    g1x = a.x; g1y = a.y; g2x = b.x; g2y = b.y;
  } else {
    const float4 a = m.egf[e];
    g1x = a.x; g1y = a.y; g2x = a.z; g2y = a.w;
  }
  const int4 nd = m.enode[e];
  const R man = manning_of(m, k, i, (QT)0);
#ifdef __HIP_DEVICE_COMPILE__
  if constexpr (sizeof(QT) == 8) __builtin_amdgcn_sched_barrier(0);
#endif
  const double hm = mean3(h);
  const bool wet = p.wetdry ? (z[0] + hm > p.h0) : true;
  const double iA = rcp_nr(ai.x);

  // physical gradients of the reference coordinates from those of phi_10
  // and phi_01: J^-T e1 = g1 - g2/3, J^-T e2 = 2/3 g2
  const R c1x = g1x - g2x * (R)(1.0 / 3.0), c1y = g1y - g2y * (R)(1.0 / 3.0);
  const R c2x = g2x * (R)(2.0 / 3.0), c2y = g2y * (R)(2.0 / 3.0);

  // nodal forcing: wind stress at the vertices, pressure gradient from
  // vertex differences (FP64, large common offset)
  const int node[3] = {nd.x, nd.y, nd.z};
  R tx[3], ty[3];
  double pa[3];
  {
    const double2 *tau = (const double2 *)s.nodal;
    for (int j = 0; j < 3; ++j) {
      const double2 t = tau[node[j]];
      tx[j] = (R)t.x;
      ty[j] = (R)t.y;
      pa[j] = s.nodal[2 * (size_t)m.nn + node[j]];
    }
  }
  const double dh1 = h[1] - h[0], dh2 = h[2] - h[0];
  const R hm1 = (R)(0.5 * dh1), hm2 = (R)((2.0 * dh2 - dh1) * (1.0 / 6.0));
  const R dhx = hm1 * g1x + hm2 * g2x, dhy = hm1 * g1y + hm2 * g2y;
  const double dp1 = pa[1] - pa[0], dp2 = pa[2] - pa[0];
  const R pm1 = (R)(0.5 * dp1), pm2 = (R)((2.0 * dp2 - dp1) * (1.0 / 6.0));
  const R dpx = pm1 * g1x + pm2 * g2x, dpy = pm1 * g1y + pm2 * g2y;

  // chunk-local edge codes of the three local edges (edge << 1 | 1 on the
  // e- side)
  int ecode[3];
  for (int l = 0; l < 3; ++l) ecode[l] = (nd.w >> (10 * l)) & 0x3FF;

  // area part: rz[k] = (1/A) sum_q w_q A grad phi_k . F_zeta (FP64 sums of
  // R terms), rq[v][k] likewise for the momentum rows with the sources
  double rz[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  R rq[12];
  for (int j = 0; j < 12; ++j) rq[j] = (R)0;
  {
    const R gr = (R)p.g, gn2 = gr * man * man, irho = (R)(1.0 / p.rho0), h0 = (R)p.h0;
#pragma unroll 1
    for (int qd = 0; qd < 6; ++qd) {
      double L[3], wq;
      area_point2(qd, L, wq);
      const double xi = -L[0] + L[1] - L[2], eta = -L[0] - L[1] + L[2];
      double f[6], d[6][2];
      basis2(xi, eta, f);
      basis2_grad(xi, eta, d);
      double ze = 0.0;
      R qx = (R)0, qy = (R)0;
      for (int j = 0; j < 6; ++j) ze += z[j] * f[j];
      if constexpr (MF) {
        // selects, not an indexed load: the values stay in registers
        for (int j = 0; j < 6; ++j) {
          qx = qd == j ? AQ->qx[j] : qx;
          qy = qd == j ? AQ->qy[j] : qy;
        }
      } else {
        for (int j = 0; j < 6; ++j) {
          qx += q[j] * (R)f[j];
          qy += q[6 + j] * (R)f[j];
        }
      }
      const double hb = L[0] * h[0] + L[1] * h[1] + L[2] * h[2];
      const R H = (R)(ze + hb);
      const R ph = (R)p_hydro(p.g, ze, hb);
      R uu = (R)0, vv = (R)0;
      if (wet) {
        const R iH = rcp_nr(H);
        uu = qx * iH;
        vv = qy * iH;
      }
      const R w = (R)wq;
      const R Fz[2] = {qx * w, qy * w};
      const R Fx[2] = {(qx * uu + ph) * w, qx * vv * w};
      const R Fy[2] = {qy * uu * w, (qy * vv + ph) * w};
      // grad phi_j . F = d_j0 (J^-T e1 . F) + d_j1 (J^-T e2 . F): the flux in
      // reference components, then the reference gradients
      const R Gz1 = c1x * Fz[0] + c1y * Fz[1], Gz2 = c2x * Fz[0] + c2y * Fz[1];
      const R Gx1 = c1x * Fx[0] + c1y * Fx[1], Gx2 = c2x * Fx[0] + c2y * Fx[1];
      const R Gy1 = c1x * Fy[0] + c1y * Fy[1], Gy2 = c2x * Fy[0] + c2y * Fy[1];
      for (int j = 1; j < 6; ++j) {
        const R d0 = (R)d[j][0], d1 = (R)d[j][1];
        rz[j] += (double)(d0 * Gz1 + d1 * Gz2);
        rq[j] += d0 * Gx1 + d1 * Gx2;
        rq[6 + j] += d0 * Gy1 + d1 * Gy2;
      }
      if (wet) {
        const R Hf = fmax(H, h0);
        const R qm = sqrt_nr(qx * qx + qy * qy);
        const R fr = gn2 * qm * rcp_nr(Hf * Hf * cbrt_nr(Hf));
        const R txq = (R)L[0] * tx[0] + (R)L[1] * tx[1] + (R)L[2] * tx[2];
        const R tyq = (R)L[0] * ty[0] + (R)L[1] * ty[1] + (R)L[2] * ty[2];
        const R gz = (R)(p.g * ze);
        const R cor = (R)F.coriolis;
        const R sx = (gz * dhx - fr * qx + txq * irho - H * irho * dpx + cor * qy) * w;
        const R sy = (gz * dhy - fr * qy + tyq * irho - H * irho * dpy - cor * qx) * w;
        for (int j = 0; j < 6; ++j) {
          rq[j] += (R)f[j] * sx;
          rq[6 + j] += (R)f[j] * sy;
        }
      }
    }
  }

  rz[0] += F.rain;  // uniform rain projects on mode 0 alone
  // mixed: the RK base (later stages) is loaded here, so its latency
  // overlaps the edge integrals instead of following them; without a base
  // the element's own record stands in (unused), so the load is
  // unconditional and nothing waits for it before its use.  FP64 loads it
  // after the edge integrals (early, its registers spill at 3 waves per
  // SIMD: measured slower).
  constexpr bool kEarlyBase = sizeof(QT) == 4;
  double bz[6];
  R bq[12];
  const bool use_base = base != nullptr;
  if constexpr (kEarlyBase) load_rec<QT>(use_base ? base : u, e, bz, bq);
  // edges, from LDS: the side takes the flux its kind gives it, e- with the
  // opposite sign for a flux both sides share, integrated with its own basis
  // (e- runs the edge backwards)
#pragma unroll 1
  for (int l = 0; l < 3; ++l) {
    const int j = ecode[l] >> 1;
    const bool minus = (ecode[l] & 1) != 0;
    const int kind = L.kind[j];
    const bool take = minus ? (kind == EK_LLF || kind == EK_WALL_M) : (kind == EK_LLF || kind == EK_LLF_P || kind == EK_WALL_P);
    if (!take) continue;
    const R sg = (minus && kind == EK_LLF) ? (R)-1 : (R)1;
    const double hlA = L.hl[j] * iA;
#pragma unroll 1
    for (int g = 0; g < 4; ++g) {
      double xi, eta, fb[6];
      edge_point2(l, minus ? -gl4_s(g) : gl4_s(g), xi, eta);
      basis2(xi, eta, fb);
      const double wg = hlA * gl4_w(g);
      const double fz = (double)sg * L.fz[g * L.eds + j] * wg;
      const R fx = sg * L.fq[g * L.eds + j] * (R)wg, fy = sg * L.fq[(4 + g) * L.eds + j] * (R)wg;
      for (int jj = 0; jj < 6; ++jj) {
        rz[jj] -= fz * fb[jj];
        rq[jj] -= fx * (R)fb[jj];
        rq[6 + jj] -= fy * (R)fb[jj];
      }
    }
  }

  // inverse mass diagonal and the RK combination
  if constexpr (!kEarlyBase) {
    if (use_base) load_rec<QT>(base, e, bz, bq);
    else {
      for (int j = 0; j < 6; ++j) bz[j] = 0.0;
      for (int j = 0; j < 12; ++j) bq[j] = (R)0;
    }
  }
  const double hdt = sc.h * dt;
  bool fin = true;
  for (int j = 0; j < 6; ++j) {
    const double dw = rz[j] * kMu2Inv[j];
    out[j] = use_base ? sc.a * bz[j] + sc.b * (z[j] + hdt * dw) : z[j] + hdt * dw;
    fin = fin && __builtin_isfinite(out[j]);
  }
  const R dtq = (R)hdt;
  for (int j = 0; j < 12; ++j) {
    R dw = rq[j] * (R)kMu2Inv[j % 6];
    if (!wet) dw = (R)0;
    oqv[j] = use_base ? (R)sc.a * bq[j] + (R)sc.b * (q[j] + dtq * dw) : q[j] + dtq * dw;
    fin = fin && __builtin_isfinite(oqv[j]);
  }
  cand = cfl_candidate(out[0], (double)oqv[0], (double)oqv[6], hm, ai.y, p);
  return fin;
}

// One RK stage of chunk c from the post-processed records u (and the RK
// base records): the edge pass into LDS (lds2_raw, lds2_bytes(ed_max)),
// then the elements.
template <class QT, bool MF = false>
__device__ __forceinline__ void rhs2_chunk(DevMesh m, DevState s, Params p, const Rec2<QT> *__restrict__ u,
                                           const Rec2<QT> *__restrict__ base, St<QT> wout, StageCoef sc, int slot,
                                           int want_dt, int c, double *lds2_raw, double *red) {
  const ChunkInfo k = chunk_info(m, c);
  const Member &F = m.mem[k.member];
  Ctrl *ctl = s.ctrl + k.member;
  const int tid = threadIdx.x;
  const size_t ne = (size_t)m.ne;
  const int status = ctl->status;
  const unsigned long long dtbits = ctl->dtmin[slot];
  const double t0 = ctl->t[slot];
  double dt = 0.0;
  // No lane leaves early (the barriers must match): an inactive workgroup
  // computes and stores nothing.
  const bool active = status == 0 && dt_from_bits(p, dtbits, dt);
  const bool act = active && tid < k.cc;
  const Lds2<QT> L = lds2_view<QT>(m.ed_max, lds2_raw);
  // MFMA variant: the momentum at the area points first, through the same
  // LDS (every lane takes part; the edge pass overwrites the LDS after it)
  AreaQ<QT> AQ;
  if constexpr (MF) area_points_mfma<QT>(u, k.c0 + (tid < k.cc ? tid : k.cc - 1), lds2_raw, AQ);
  // edges of the chunk at the stage time (ocean tide), two per lane at most
  if (active) {
    const double ts = t0 + sc.c * dt;
    const bool tide = F.n_tide > 0 || F.tide_offset != 0.0;
    const int j0 = tid < k.ne_loc ? tid : k.ne_loc - 1;
    const int j1 = tid + kBlock < k.ne_loc ? tid + kBlock : k.ne_loc - 1;
    if constexpr (sizeof(QT) == 4) {
      // mixed: both records first, so the second edge's record is in
      // registers when the first edge's flux is done (in FP64 the extra
      // registers spill at 3 waves per SIMD: measured slower there)
      const double zb = tide ? tide_level(F, ts) : 0.0;
      const Edge2In<QT> E0 = load_edge2<QT>(m, k, j0), E1 = load_edge2<QT>(m, k, j1);
      if (tid < k.ne_loc) edge_phase2<QT>(m, p, k, u, zb, tid, E0, L);
      if (tid + kBlock < k.ne_loc) edge_phase2<QT>(m, p, k, u, zb, tid + kBlock, E1, L);
    } else {
      // FP64: the first record is requested before the ocean tide is formed
      // (measured faster; in the mixed path the other order was)
      const Edge2In<QT> E0 = load_edge2<QT>(m, k, j0);
      const double zb = tide ? tide_level(F, ts) : 0.0;
      if (tid < k.ne_loc) edge_phase2<QT>(m, p, k, u, zb, tid, E0, L);
      if (tid + kBlock < k.ne_loc) edge_phase2<QT>(m, p, k, u, zb, tid + kBlock, load_edge2<QT>(m, k, j1), L);
    }
  }
  __syncthreads();
  double out[6], cand = INFINITY;
  QT oqv[12];
  bool fin = true;
  if (act) fin = rhs2_element<QT, MF>(m, s, p, k, F, u, base, sc, tid, L, out, oqv, cand, dt, &AQ);
  const int e = k.c0 + tid;
  if (act) {
    for (int j = 0; j < 6; ++j) wout.z[j * ne + e] = out[j];
    for (int j = 0; j < 12; ++j) wout.q[j * ne + e] = oqv[j];
    if (!fin) atomicCAS(&ctl->status, 0, (int)DGSWE_E_NONFINITE);
  }
  if (want_dt) {
    const double bm = block_min<kBlock>(act ? cand : (double)INFINITY, red);
    if (tid == 0 && bm < INFINITY) atomicMin(&ctl->dtmin[slot ^ 1], double_to_bits(bm));
  }
  if (sc.last && active && k.first && tid == 0) {
    ctl->t[slot ^ 1] = t0 + dt;
    ctl->dt_last = dt;
    ctl->steps = ctl->steps + 1;
    ctl->pp_in = 1;
  }
}

}  // namespace dgswe
