// Device code of the p = 1 stage (per-element math, the LDS phases and the
// whole stage of one chunk), shared by the stage kernel and the kernel that
// advances members of both orders in one launch.  See dgswe_kernels.hip for
// the design.
#pragma once
#include "dgswe_device.h"

namespace dgswe {


// ---------------------------------------------------------------- per-item math
// Post-processing of one element (slope limiter, then wet/dry), FP64 in
// both paths.  u[9] is the unlimited state [var*3 + mode].

// Face-neighbour limiter: nbm[v][k] the unlimited mean of variable v of
// neighbour k (has[k] false: no neighbour).
HD void limit_face(double u[9], const double nbm[3][3], const bool has[3]) {
  for (int v = 0; v < 3; ++v) {
    const double mean = u[3 * v];
    double hi = mean, lo = mean;
    for (int k = 0; k < 3; ++k)
      if (has[k]) { hi = fmax(hi, nbm[v][k]); lo = fmin(lo, nbm[v][k]); }
    const double a = u[3 * v + 1], b = u[3 * v + 2];
    const double d0 = (mean - a - b) - mean, d1 = (mean + a - b) - mean, d2 = (mean + 2.0 * b) - mean;
    // the smallest vertex ratio belongs to the largest excursion on each side
    const double dmax = fmax(d0, fmax(d1, d2)), dmin = fmin(d0, fmin(d1, d2));
    double alpha = 1.0;
    if (dmax > 0.0 && hi - mean < dmax) alpha = fmin(alpha, (hi - mean) / dmax);
    if (dmin < 0.0 && lo - mean > dmin) alpha = fmin(alpha, (lo - mean) / dmin);
    u[3 * v + 1] = a * alpha;
    u[3 * v + 2] = b * alpha;
  }
}

// Vertex-based limiter: lo[v][i], hi[v][i] the range of the unlimited means
// of variable v over the elements sharing the element's vertex i; alpha is
// the largest value in [0, 1] that keeps every vertex value inside.
HD void limit_vertex(double u[9], const double lo[3][3], const double hi[3][3]) {
  for (int v = 0; v < 3; ++v) {
    const double mean = u[3 * v], a = u[3 * v + 1], b = u[3 * v + 2];
    const double d[3] = {(mean - a - b) - mean, (mean + a - b) - mean, (mean + 2.0 * b) - mean};
    double alpha = 1.0;
    for (int i = 0; i < 3; ++i) {
      if (d[i] > 0.0) alpha = fmin(alpha, (hi[v][i] - mean) / d[i]);
      else if (d[i] < 0.0) alpha = fmin(alpha, (lo[v][i] - mean) / d[i]);
    }
    u[3 * v + 1] = a * alpha;
    u[3 * v + 2] = b * alpha;
  }
}

// Wet/dry treatment; h[3] the vertex bathymetry.
HD void wetdry_fix(double u[9], const double h[3], double hmean, const Params &p) {
  if (p.wetdry) {
    const double z0 = u[0] - u[1] - u[2], z1 = u[0] + u[1] - u[2], z2 = u[0] + 2.0 * u[2];
    double H[3] = {z0 + h[0], z1 + h[1], z2 + h[2]};
    const double Hm = u[0] + hmean;
    bool changed = false;
    if (Hm <= p.h0) {
      H[0] = H[1] = H[2] = Hm;
      for (int j = 3; j < 9; ++j) u[j] = 0.0;
      changed = true;
    } else if (fmin(H[0], fmin(H[1], H[2])) < p.h0) {
      double D = 0.0, S = 0.0;
      for (int i = 0; i < 3; ++i) {
        if (H[i] < p.h0) D += p.h0 - H[i];
        else S += H[i] - p.h0;
      }
      if (S > D) {
        for (int i = 0; i < 3; ++i) H[i] = (H[i] < p.h0) ? p.h0 : H[i] - D * (H[i] - p.h0) / S;
      } else {
        // S - D = 3 (Hm - H0) > 0 exactly; if rounding cancels it: flat at Hm
        H[0] = H[1] = H[2] = Hm;
      }
      changed = true;
    }
    if (changed) {
      const double y0 = H[0] - h[0], y1 = H[1] - h[1], y2 = H[2] - h[2];
      u[1] = 0.5 * (y1 - y0);
      u[2] = 0.5 * (y2 - u[0]);
    }
  }
}

HD void postprocess(double u[9], const double nbm[3][3], const bool has[3], const double h[3],
                    double hmean, const Params &p) {
  if (p.limiter == 1) limit_face(u, nbm, has);
  wetdry_fix(u, h, hmean, p);
}

// vertex bounds of an element whose vertices have the range slots nd
HD void load_vbounds(const double *vb, int4 nd, double lo[3][3], double hi[3][3]) {
  const int n[3] = {nd.x, nd.y, nd.z};
  for (int i = 0; i < 3; ++i)
    for (int v = 0; v < 3; ++v) {
      const double2 r = ((const double2 *)vb)[3 * (size_t)n[i] + v];
      lo[v][i] = r.x;
      hi[v][i] = r.y;
    }
}

// Trace coefficients, bathymetry and normal of one edge at its three
// Gauss-Lobatto points s = -1, 0, 1 in the e+ orientation.
template <class R>
struct EdgeGeo {
  double cp1[3], cp2[3], cm1[3], cm2[3];  // trace coefficients per point, e+ and e-
  double hq[3];                           // bathymetry at the points
  R nx, ny;
};

// One pass over the three points (weights 1/3, 4/3, 1/3), accumulating the
// flux moments m0 = sum_g w_g F_g and m1 = sum_g w_g s_g F_g (before the
// factor len/2) and the mass-flux integral.  kind 0: LLF between the two
// sides; 1: land wall seen from e+ (wet flag wetp); 2: wall seen from e-
// (normal -n); 3: Roe between the two (wet) sides.  States: zeta modes (FP64) and momentum modes (R) of e+ and
// e-; ghost: the e- trace is (zb, momentum of e+).
template <class R>
HD void edge_pass(int kind, const double zp[3], const R qp[6], const double zm[3], const R qm[6], bool ghost,
                  double zb, bool wetp, bool wetm, const EdgeGeo<R> &G, const Params &p, R m0[3], R m1[3],
                  R &mflux) {
  const R wq[3] = {(R)(1.0 / 3.0), (R)(4.0 / 3.0), (R)(1.0 / 3.0)};
  for (int v = 0; v < 3; ++v) { m0[v] = (R)0; m1[v] = (R)0; }
  mflux = (R)0;
  for (int g = 0; g < 3; ++g) {
    const R c1 = (R)G.cp1[g], c2 = (R)G.cp2[g];
    const double zpg = zp[0] + G.cp1[g] * zp[1] + G.cp2[g] * zp[2];
    const R qxp = qp[0] + c1 * qp[1] + c2 * qp[2];
    const R qyp = qp[3] + c1 * qp[4] + c2 * qp[5];
    double zmg;
    R qxm, qym;
    if (ghost) {
      zmg = zb; qxm = qxp; qym = qyp;
    } else {
      const R d1 = (R)G.cm1[g], d2 = (R)G.cm2[g];
      zmg = zm[0] + G.cm1[g] * zm[1] + G.cm2[g] * zm[2];
      qxm = qm[0] + d1 * qm[1] + d2 * qm[2];
      qym = qm[3] + d1 * qm[4] + d2 * qm[5];
    }
    R F[3];
    if (kind == 0) llf<R>(p.g, zpg, qxp, qyp, zmg, qxm, qym, G.hq[g], G.nx, G.ny, wetp, wetm, F);
    else if (kind == 3) roe<R>(p.g, zpg, qxp, qyp, zmg, qxm, qym, G.hq[g], G.nx, G.ny, F);
    else if (kind == 1) wall<R>(p.g, zpg, qxp, qyp, G.hq[g], G.nx, G.ny, wetp, F);
    else wall<R>(p.g, zmg, qxm, qym, G.hq[g], -G.nx, -G.ny, true, F);
    const R sg = (R)(g - 1);
    for (int v = 0; v < 3; ++v) {
      m0[v] += wq[g] * F[v];
      m1[v] += (wq[g] * sg) * F[v];
    }
    mflux += wq[g] * F[0];
  }
}

// Edge flux moments: M0 = len/2 sum_g w_g F_g, M1 = len/2 sum_g w_g s_g F_g
// in the e+ frame.  e+ receives (M0, M1), e- receives (-M0, M1) in its own
// frame; the returned mode says which sides receive anything (0 both, 1 e+
// only, 2 e- only, 3 none).  Wet/dry rules: both sides dry -> nothing; one
// side dry -> LLF with u = 0 on the dry side if its mass flux runs into the
// dry side, else a wall for the wet side and nothing for the dry side.
// Ocean edges: ghost state (zeta_b, Q+), wet iff zeta_b + mean h_b > h0.
template <class R>
HD int edge_flux(const double zp[3], const R qp[6], const double zm[3], const R qm[6], int lp, int lm, int type,
                 bool wetp, bool wetm_in, double hA, double hB, R nx, R ny, R hl, double zb, const Params &p,
                 R mom[6]) {
  EdgeGeo<R> G;
  const int va = lp == 2 ? 0 : lp + 1, vb = lp == 0 ? 2 : lp - 1;
  G.cp1[0] = c1v(va); G.cp2[0] = c2v(va);
  G.cp1[1] = c1m(lp); G.cp2[1] = c2m(lp);
  G.cp1[2] = c1v(vb); G.cp2[2] = c2v(vb);
  // e- runs the edge backwards: its vertex (lm+2) sits at s = -1
  const int ma = lm == 2 ? 0 : lm + 1, mb = lm == 0 ? 2 : lm - 1;
  G.cm1[0] = c1v(mb); G.cm2[0] = c2v(mb);
  G.cm1[1] = c1m(lm); G.cm2[1] = c2m(lm);
  G.cm1[2] = c1v(ma); G.cm2[2] = c2v(ma);
  G.hq[0] = hA; G.hq[1] = hA * 0.5 + hB * 0.5; G.hq[2] = hB;
  G.nx = nx; G.ny = ny;
  const bool ghost = type != 0;
  const bool wetm = ghost ? (p.wetdry ? (zb + 0.5 * (hA + hB) > p.h0) : true) : wetm_in;
  R m0[3], m1[3], mflux;
  int mode;
  bool minus = false;
  if (type == DGSWE_BC_LAND) {
    edge_pass<R>(1, zp, qp, zm, qm, true, zb, wetp, wetm, G, p, m0, m1, mflux);
    mode = 1;
  } else if (!wetp && !wetm) {
    for (int v = 0; v < 6; ++v) mom[v] = (R)0;
    return 3;
  } else {
    edge_pass<R>((p.flux == 1 && wetp && wetm) ? 3 : 0, zp, qp, zm, qm, ghost, zb, wetp, wetm, G, p, m0, m1, mflux);
    mode = ghost ? 1 : 0;
    if (!(wetp && wetm)) {
      const bool flood = wetp ? (mflux > (R)0) : (mflux < (R)0);
      if (!flood) {
        if (wetp) {
          edge_pass<R>(1, zp, qp, zm, qm, ghost, zb, true, wetm, G, p, m0, m1, mflux);
          mode = 1;
        } else if (ghost) {
          mode = 3;
        } else {
          edge_pass<R>(2, zp, qp, zm, qm, false, zb, wetp, true, G, p, m0, m1, mflux);
          mode = 2;
          minus = true;
        }
      }
    }
  }
  // mode 2 holds the e- frame moments (P0, P1) with P1 along e-'s own
  // direction (-s); they are stored so that e- reads (-M0, M1) = (P0, P1)
  const R sgn = minus ? (R)-1 : (R)1;
  for (int v = 0; v < 3; ++v) {
    mom[v] = sgn * hl * m0[v];
    mom[3 + v] = sgn * hl * m1[v];
  }
  return mode;
}

// Per-element inputs of the area integrals and of the RK update: Manning n,
// the member's Coriolis parameter and rain rate and the chunk-local edges
// (loaded in phase L), 2 x inradius (after phase P), wind stress at the
// vertices and the pressure gradient modes (after phase P in the mixed path,
// in phase A in FP64), vertex bathymetry (phase A, from LDS) and (second
// stage) the post-processed RK base (phase A, after the area integrals).
template <class QT>
struct ElemPre {
  double h[3];
  QT tx[3], ty[3];
  QT pm1, pm2;  // modes of grad p_a on grad phi_10, grad phi_01
  double wbz[3];
  QT wbq[6];
  double inr2;
  QT manning;
  QT coriolis;
  double rain;
  int ledge[3];
};

// Volume + source integrals of a post-processed state (zeta FP64, momentum
// R); returns R_k / A (area part) (1/3) [grad phi_k . sum_q F(w_q) + sum_q
// phi_k(q) s(w_q)] in rz[3] (FP64) and rq[6] (R).
template <class R>
HD void area_terms(const double z[3], const R q[6], bool wet, const ElemPre<R> &E, R g1x, R g1y, R g2x, R g2y,
                   const Params &p, double rz[3], R rq[6]) {
  // gradient of a linear nodal field with vertex values f0, f1, f2: modes
  // (f1 - f0)/2 and (2 (f2 - f0) - (f1 - f0))/6 on grad phi_10, grad phi_01,
  // from vertex differences so a large common offset cancels exactly
  const double dh1 = E.h[1] - E.h[0], dh2 = E.h[2] - E.h[0];
  const R hm1 = (R)(0.5 * dh1), hm2 = (R)((2.0 * dh2 - dh1) * (1.0 / 6.0));
  const R dhx = hm1 * g1x + hm2 * g2x, dhy = hm1 * g1y + hm2 * g2y;
  const R dpx = E.pm1 * g1x + E.pm2 * g2x, dpy = E.pm1 * g1y + E.pm2 * g2y;
  const R gr = (R)p.g;
  const R gn2 = gr * E.manning * E.manning;
  const R irho = (R)(1.0 / p.rho0);
  const R h0 = (R)p.h0;
  // area points: barycentric (2/3,1/6,1/6) and permutations; basis values
  // phi_10 = (-1/2, 1/2, 0), phi_01 = (-1/2, -1/2, 1)
  const double C1[3] = {-0.5, 0.5, 0.0}, C2[3] = {-0.5, -0.5, 1.0};
  const double L0[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
  const double L1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
  const double L2[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
  R sF[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  R S0[2] = {0, 0}, S1[2] = {0, 0}, S2[2] = {0, 0};
  for (int qd = 0; qd < 3; ++qd) {
    const R c1 = (R)C1[qd], c2 = (R)C2[qd], l0 = (R)L0[qd], l1 = (R)L1[qd], l2 = (R)L2[qd];
    const double ze = z[0] + C1[qd] * z[1] + C2[qd] * z[2];
    const R qx = q[0] + c1 * q[1] + c2 * q[2];
    const R qy = q[3] + c1 * q[4] + c2 * q[5];
    const double hb = L0[qd] * E.h[0] + L1[qd] * E.h[1] + L2[qd] * E.h[2];
    const R H = (R)(ze + hb);
    const R ph = (R)p_hydro(p.g, ze, hb);
    R uu = (R)0, vv = (R)0;
    if (wet) {
      const R iH = rcp_nr(H);
      uu = qx * iH;
      vv = qy * iH;
    }
    sF[0][0] += qx;            sF[0][1] += qy;
    sF[1][0] += qx * uu + ph;  sF[1][1] += qx * vv;
    sF[2][0] += qy * uu;       sF[2][1] += qy * vv + ph;
    if (wet) {
      const R Hf = fmax(H, h0);
      const R qm = sqrt_nr(qx * qx + qy * qy);
      const R fr = gn2 * qm * rcp_nr(Hf * Hf * cbrt_nr(Hf));
      const R txq = l0 * E.tx[0] + l1 * E.tx[1] + l2 * E.tx[2];
      const R tyq = l0 * E.ty[0] + l1 * E.ty[1] + l2 * E.ty[2];
      const R gz = (R)(p.g * ze);
      const R sx = gz * dhx - fr * qx + txq * irho - H * irho * dpx + E.coriolis * qy;
      const R sy = gz * dhy - fr * qy + tyq * irho - H * irho * dpy - E.coriolis * qx;
      S0[0] += sx;          S0[1] += sy;
      S1[0] += c1 * sx;     S1[1] += c1 * sy;
      S2[0] += c2 * sx;     S2[1] += c2 * sy;
    }
  }
  const R third = (R)(1.0 / 3.0);
  rz[0] = E.rain;  // the only mass source: uniform rain (projects on mode 0 alone)
  rz[1] = (double)((g1x * sF[0][0] + g1y * sF[0][1]) * third);
  rz[2] = (double)((g2x * sF[0][0] + g2y * sF[0][1]) * third);
  for (int v = 0; v < 2; ++v) {
    rq[3 * v + 0] = S0[v] * third;
    rq[3 * v + 1] = (g1x * sF[v + 1][0] + g1y * sF[v + 1][1] + S1[v]) * third;
    rq[3 * v + 2] = (g2x * sF[v + 1][0] + g2y * sF[v + 1][1] + S2[v]) * third;
  }
}



// Element e of a state, post-processed with neighbour means read from the
// same state if pp, as FP64 (read-back)
template <class QT>
HD void load_pp_global(const DevMesh &m, const Params &p, const double *vb, CSt<QT> w, int e, bool pp,
                       double u[9]) {
  const size_t ne = (size_t)m.ne;
  for (int k = 0; k < 3; ++k) u[k] = w.z[k * ne + e];
  for (int k = 0; k < 6; ++k) u[3 + k] = (double)w.q[k * ne + e];
  if (!pp) return;
  if (p.limiter == 2) {
    double h[3], lo[3][3], hi[3][3];
    for (int k = 0; k < 3; ++k) h[k] = m.hbv[k * ne + e];
    load_vbounds(vb, m.evb[e], lo, hi);
    limit_vertex(u, lo, hi);
    wetdry_fix(u, h, mean3(h), p);
    return;
  }
  double h[3], nbm[3][3];
  bool has[3];
  for (int k = 0; k < 3; ++k) h[k] = m.hbv[k * ne + e];
  for (int k = 0; k < 3; ++k) {
    const int f = m.el_nb[k * ne + e];
    has[k] = f >= 0;
    nbm[0][k] = has[k] ? w.z[f] : 0.0;
    nbm[1][k] = has[k] ? (double)w.q[f] : 0.0;
    nbm[2][k] = has[k] ? (double)w.q[3 * ne + f] : 0.0;
  }
  postprocess(u, nbm, has, h, mean3(h), p);
}

// ---------------------------------------------------------------- fused stage phases
// LDS layout of one chunk (sizes from the mesh maxima):
//   SZ[3][nl_max] double, SQ[6][nl_max] QT: states of chunk + ring 1.  Phase
//                 P writes back the post-processed slopes (modes 1, 2) but
//                 never the means, which stay the unlimited means that the
//                 neighbours' limiters read concurrently; a dry element's
//                 momentum is zero after its post-processing, so phases E and
//                 A read its momentum means as 0 (WET = 0)
//   MZ[n2_max]    double, MQ[2][n2_max] QT: unlimited zeta, Qx, Qy means of
//                 ring 2
//   LH[3][nl_max] double: vertex bathymetry of chunk + ring 1
//   EM[6][ed_max] QT: edge moments
//   EMODE[ed_max], WET[nl_max] bytes
// (The chunk elements' geometry is read in phase A, not kept in LDS.)
template <class QT>
struct Lds {
  double *SZ, *MZ, *LH;
  QT *SQ, *MQ, *EM;
  unsigned char *EMODE, *WET;
  int nls, n2s, eds;  // strides
};

template <class QT>
HD size_t lds_bytes(const DevMesh &m) {
  return 8 * (6 * (size_t)m.nl_max + (size_t)m.n2_max) +
         sizeof(QT) * (6 * (size_t)m.nl_max + 2 * (size_t)m.n2_max + 6 * (size_t)m.ed_max) + (size_t)m.ed_max +
         (size_t)m.nl_max;
}

template <class QT>
HD Lds<QT> lds_view(const DevMesh &m, void *base) {
  Lds<QT> L;
  L.nls = m.nl_max; L.n2s = m.n2_max; L.eds = m.ed_max;
  L.SZ = (double *)base;
  L.MZ = L.SZ + 3 * (size_t)L.nls;
  L.LH = L.MZ + (size_t)L.n2s;
  L.SQ = (QT *)(L.LH + 3 * (size_t)L.nls);
  L.MQ = L.SQ + 6 * (size_t)L.nls;
  L.EM = L.MQ + 2 * (size_t)L.n2s;
  L.EMODE = (unsigned char *)(L.EM + 6 * (size_t)L.eds);
  L.WET = L.EMODE + L.eds;
  return L;
}


// bit patterns of the packed ids stored in a double / float slot
HD uint32_t ids_of(double v) {
  union { double d; unsigned long long u; } x;
  x.d = v;
  return (uint32_t)x.u;
}
HD uint32_t ids_of(float v) {
  union { float f; uint32_t u; } x;
  x.f = v;
  return x.u;
}

// one chunk-local edge record, loaded early and kept in registers
template <class QT>
struct EdgeRec {
  uint32_t ids;  // e+ | e- << 12 | (lp | lm << 2 | type << 4) << 24
  QT nx, ny, hl;
};

HD void load_edge_rec(const DevMesh &m, const ChunkInfo &k, int j, EdgeRec<double> &R) {
  const size_t r = (size_t)(k.leo + j);
  const double2 a = ld_once(m.le_a + r), b = ld_once(m.le_b + r);
  R.nx = a.x; R.ny = a.y; R.hl = b.x;
  R.ids = ids_of(b.y);
}
HD void load_edge_rec(const DevMesh &m, const ChunkInfo &k, int j, EdgeRec<float> &R) {
  const size_t r = (size_t)(k.leo + j);
  const float4 a = m.le_f[r];
  R.nx = a.x; R.ny = a.y; R.hl = a.z;
  R.ids = ids_of(a.w);
}

// vertex bathymetry of local element i in [0, nl) of chunk + ring 1
HD void load_local_hb(const DevMesh &m, const ChunkInfo &k, int i, double h[3]) {
  const double2 a = ld_once(m.lhb01 + k.lo + i);
  h[0] = a.x;
  h[1] = a.y;
  h[2] = ld_once(m.lhb2 + k.lo + i);
}

// local neighbour indices of local element i (chunk + ring 1)
HD void load_local_nb(const DevMesh &m, const ChunkInfo &k, int i, uint16_t nb[3]) {
  const unsigned long long v = ld_once(m.lnb + k.lo + i);
  for (int q = 0; q < 3; ++q) nb[q] = (uint16_t)(v >> (16 * q));
}

// Phase L works in three rounds of loads so that each lane waits for
// memory about twice instead of once per dependent gather: first the
// indices later loads depend on (global id of a ring-1 element, of a
// ring-2 element, node ids), then every load that needs no index, then the
// gathers through the indices; LDS is written after all of them.

// global element id of local element i in [0, nl) of chunk + ring 1
HD int local_to_global(const DevMesh &m, const ChunkInfo &k, int i) { return ld_once(m.lgid + k.lo + i); }

// full state of element g
template <class QT>
struct StateReg {
  double z[3];
  QT q[6];
};

template <class QT>
HD void load_state_reg(CSt<QT> w, size_t ne, int g, StateReg<QT> &S) {
  for (int j = 0; j < 3; ++j) S.z[j] = w.z[j * ne + g];
  for (int j = 0; j < 6; ++j) S.q[j] = w.q[j * ne + g];
}

// local element i of chunk + ring 1 into LDS (its state)
template <class QT>
HD void store_state_lds(const Lds<QT> &L, int i, const StateReg<QT> &S) {
  for (int j = 0; j < 3; ++j) L.SZ[j * L.nls + i] = S.z[j];
  for (int j = 0; j < 6; ++j) L.SQ[j * L.nls + i] = S.q[j];
}

// ring-2 element j (local index nl + j): unlimited means only
template <class QT>
HD void load_h2_lds(const Lds<QT> &L, CSt<QT> w, size_t ne, int j, int g) {
  L.MZ[j] = w.z[g];
  L.MQ[j] = w.q[g];
  L.MQ[L.n2s + j] = w.q[3 * ne + g];
}

// geometry of a chunk element
template <class QT>
struct GeoReg {
  QT g[4];
  double area;
};

// gradients, area and 2 x inradius of chunk element i
HD void load_geo(const DevMesh &m, const ChunkInfo &k, int i, GeoReg<double> &G, double &inr2) {
  const int e = k.c0 + i;
  const double2 a = ld_once(m.eg1 + e), b = ld_once(m.eg2 + e), c = ld_once(m.eai + e);
  G.g[0] = a.x; G.g[1] = a.y; G.g[2] = b.x; G.g[3] = b.y;
  G.area = c.x;
  inr2 = c.y;
}
HD void load_geo(const DevMesh &m, const ChunkInfo &k, int i, GeoReg<float> &G, double &inr2) {
  const int e = k.c0 + i;
  const float4 a = m.egf[e];
  const double2 c = m.eai[e];
  G.g[0] = a.x; G.g[1] = a.y; G.g[2] = a.z; G.g[3] = a.w;
  G.area = c.x;
  inr2 = c.y;
}

// node ids and local edge codes of chunk element i
HD void load_elem_node(const DevMesh &m, const ChunkInfo &k, int i, int node[3], int ledge[3]) {
  const int4 v = ld_once(m.enode + k.c0 + i);
  node[0] = v.x; node[1] = v.y; node[2] = v.z;
  for (int q = 0; q < 3; ++q) ledge[q] = (v.w >> (10 * q)) & 0x3FF;
}


// the post-processed slopes of local element i into LDS; the means stay
// (the zeta mean is unchanged by the post-processing; the momentum means of
// a dry element, zeroed by it, are read as 0 through its WET flag)
template <class QT>
HD void write_back_pp(const Lds<QT> &L, int i, const double u[9]) {
  for (int j = 1; j < 3; ++j) L.SZ[j * L.nls + i] = u[j];
  for (int j = 1; j < 3; ++j) {
    L.SQ[j * L.nls + i] = (QT)u[3 + j];
    L.SQ[(3 + j) * L.nls + i] = (QT)u[6 + j];
  }
}

// phase P for local element i of chunk + ring 1 (h: its vertex bathymetry,
// nb: local neighbour indices); the post-processed state of a chunk element
// also goes to wpp if given
// (VL: the vertex-based limiter, with the node ranges vb and the range
// slots ev of the element's vertices)
template <class QT, bool VL>
HD void phase_post(const Params &p, const ChunkInfo &k, const Lds<QT> &L, int pp_in, int i, const double h[3],
                   const uint16_t nb[3], bool to_wpp, const St<QT> &wpp, size_t ne, const double *vb, int4 ev) {
  const int nl = k.nl();
  const double hmean = mean3(h);
  double u[9];
  for (int j = 0; j < 3; ++j) u[j] = L.SZ[j * L.nls + i];
  for (int j = 0; j < 6; ++j) u[3 + j] = (double)L.SQ[j * L.nls + i];
  if (VL && pp_in) {
    double lo[3][3], hi[3][3];
    load_vbounds(vb, ev, lo, hi);
    limit_vertex(u, lo, hi);
    wetdry_fix(u, h, hmean, p);
    write_back_pp<QT>(L, i, u);
  } else if (pp_in) {
    double nbm[3][3];
    bool has[3];
    for (int q = 0; q < 3; ++q) {
      const uint16_t f = nb[q];
      has[q] = f != kNone;
      const int fi = has[q] ? f : 0;
      const bool in = fi < nl;  // chunk + ring 1: unlimited means in SZ, SQ
      nbm[0][q] = in ? L.SZ[fi] : L.MZ[fi - nl];
      nbm[1][q] = (double)(in ? L.SQ[fi] : L.MQ[fi - nl]);
      nbm[2][q] = (double)(in ? L.SQ[3 * L.nls + fi] : L.MQ[L.n2s + fi - nl]);
    }
    postprocess(u, nbm, has, h, hmean, p);
    write_back_pp<QT>(L, i, u);
  }
  L.WET[i] = (p.wetdry ? (u[0] + hmean > p.h0) : true) ? 1 : 0;
  if (to_wpp && i < k.cc) {
    const size_t e = (size_t)(k.c0 + i);
    for (int j = 0; j < 3; ++j) st_out(wpp.z + j * ne + e, u[j]);
    for (int j = 0; j < 6; ++j) st_out(wpp.q + j * ne + e, (QT)u[3 + j]);
  }
}

// phase E for chunk-local edge j with its record
template <class QT>
HD void phase_edge(const Params &p, const Lds<QT> &L, double zb, int j, const EdgeRec<QT> &R) {
  const int info = (int)(R.ids >> 24);
  const int lp = info & 3, lm = (info >> 2) & 3, type = info >> 4;
  const int ip = (int)(R.ids & 0xFFFu), im = (int)((R.ids >> 12) & 0xFFFu);
  double zp[3], zm[3];
  QT qp[6], qm[6];
  for (int q = 0; q < 3; ++q) zp[q] = L.SZ[q * L.nls + ip];
  for (int q = 0; q < 6; ++q) qp[q] = L.SQ[q * L.nls + ip];
  const bool wetp = L.WET[ip] != 0;
  if (!wetp) qp[0] = qp[3] = (QT)0;  // a dry element's momentum is zero
  bool wetm = false;
  if (type == 0) {
    for (int q = 0; q < 3; ++q) zm[q] = L.SZ[q * L.nls + im];
    for (int q = 0; q < 6; ++q) qm[q] = L.SQ[q * L.nls + im];
    wetm = L.WET[im] != 0;
    if (!wetm) qm[0] = qm[3] = (QT)0;
  } else {
    for (int q = 0; q < 3; ++q) zm[q] = 0.0;
    for (int q = 0; q < 6; ++q) qm[q] = (QT)0;
  }
  // bathymetry at the edge ends: vertices lp+1 (s = -1) and lp+2 (s = +1) of e+
  const int va = lp == 2 ? 0 : lp + 1, vb = lp == 0 ? 2 : lp - 1;
  const double hA = L.LH[va * L.nls + ip], hB = L.LH[vb * L.nls + ip];
  QT mom[6];
  const int mode =
      edge_flux<QT>(zp, qp, zm, qm, lp, lm, type, wetp, wetm, hA, hB, R.nx, R.ny, R.hl, zb, p, mom);
  for (int q = 0; q < 6; ++q) L.EM[q * L.eds + j] = mom[q];
  L.EMODE[j] = (unsigned char)mode;
}

// nodal forcing at the element's vertices (node: its node ids); the nodal
// array holds (tau_x, tau_y) pairs [nn], then p_a [nn]
template <class QT>
HD void load_elem_forcing(const DevMesh &m, const DevState &s, const int node[3], ElemPre<QT> &P) {
  const size_t nn = (size_t)m.nn;
  const double2 *tau = (const double2 *)s.nodal;
  double pa[3];
  for (int q = 0; q < 3; ++q) {
    const double2 t = tau[node[q]];
    P.tx[q] = (QT)t.x;
    P.ty[q] = (QT)t.y;
    pa[q] = s.nodal[2 * nn + node[q]];
  }
  // pressure modes from vertex differences in FP64 (large common offset)
  const double dp1 = pa[1] - pa[0], dp2 = pa[2] - pa[0];
  P.pm1 = (QT)(0.5 * dp1);
  P.pm2 = (QT)((2.0 * dp2 - dp1) * (1.0 / 6.0));
}

// phase A for chunk element i (node: its node ids; G: its geometry);
// returns the CFL candidate of the output when want_dt, and sets bad on a
// non-finite output.  base: combine with the post-processed RK base wb, out
// = a base + b (w + hdt L(w)), else out = w + hdt L(w).  The RK base is
// loaded after the area integrals and, unless P0 holds it already (the
// mixed path), the nodal forcing at the start, so they hold no registers
// through the earlier phases (that is what lets the stage kernel run 3
// waves per SIMD in FP64).
template <class QT, bool FORCING_IN_P0>
HD double phase_area(const DevMesh &m, const DevState &s, const Params &p, const ChunkInfo &k, const Lds<QT> &L,
                     const ElemPre<QT> &P0, const int node[3], const GeoReg<QT> &G, const CSt<QT> &wb, bool base,
                     double ca, double cb, St<QT> wout, size_t ne, double dt, int want_dt, int i, bool &bad) {
  const size_t e = (size_t)(k.c0 + i);
  ElemPre<QT> P = P0;
  if (!FORCING_IN_P0) load_elem_forcing<QT>(m, s, node, P);
  for (int q = 0; q < 3; ++q) P.h[q] = L.LH[q * L.nls + i];
  double z[3];
  QT q[6];
  for (int j = 0; j < 3; ++j) z[j] = L.SZ[j * L.nls + i];
  for (int j = 0; j < 6; ++j) q[j] = L.SQ[j * L.nls + i];
  const bool wet = L.WET[i] != 0;
  if (!wet) q[0] = q[3] = (QT)0;  // a dry element's momentum is zero
  double rz[3];
  QT rq[6];
  area_terms<QT>(z, q, wet, P, G.g[0], G.g[1], G.g[2], G.g[3], p, rz, rq);
  if (base) {
    for (int j = 0; j < 3; ++j) P.wbz[j] = wb.z[j * ne + e];
    for (int j = 0; j < 6; ++j) P.wbq[j] = wb.q[j * ne + e];
  }
  // fixed-order gather of the three edges: R_k / A -= edge_k / A (the zeta
  // rows in FP64, so each edge's mass moment cancels between its sides)
  const double iAd = rcp_nr(G.area);
  const QT iA = (QT)iAd;
  for (int l = 0; l < 3; ++l) {
    const int code = P.ledge[l];
    const int j = code >> 1, side = code & 1;
    const int md = L.EMODE[j];
    if (md == 3 || md == 2 - side) continue;  // this side receives nothing
    const double a1 = ga1(l), b1 = gb1(l), a2 = ga2(l), b2 = gb2(l);
    {
      const double P0 = (side ? -iAd : iAd) * (double)L.EM[j];
      const double P1 = iAd * (double)L.EM[3 * L.eds + j];
      rz[0] -= P0;
      rz[1] -= a1 * P0 + b1 * P1;
      rz[2] -= a2 * P0 + b2 * P1;
    }
    const QT sg = side ? -iA : iA;
    for (int v = 0; v < 2; ++v) {
      const QT P0 = sg * L.EM[(v + 1) * L.eds + j];
      const QT P1 = iA * L.EM[(v + 4) * L.eds + j];
      rq[3 * v + 0] -= P0;
      rq[3 * v + 1] -= (QT)a1 * P0 + (QT)b1 * P1;
      rq[3 * v + 2] -= (QT)a2 * P0 + (QT)b2 * P1;
    }
  }
  const double imu[3] = {1.0, 6.0, 2.0};
  bool fin = true;
  double oz[3];
  QT oq[6];
  for (int j = 0; j < 3; ++j) {
    const double dw = rz[j] * imu[j];
    oz[j] = base ? ca * P.wbz[j] + cb * (z[j] + dt * dw) : z[j] + dt * dw;
    st_out(wout.z + j * ne + e, oz[j]);
    fin = fin && __builtin_isfinite(oz[j]);
  }
  const QT dtq = (QT)dt;
  for (int j = 0; j < 6; ++j) {
    QT dw = rq[j] * (QT)imu[j % 3];
    if (!wet) dw = (QT)0;
    oq[j] = base ? (QT)ca * P.wbq[j] + (QT)cb * (q[j] + dtq * dw) : q[j] + dtq * dw;
    st_out(wout.q + j * ne + e, oq[j]);
    fin = fin && __builtin_isfinite(oq[j]);
  }
  bad = !fin;
  return want_dt ? cfl_candidate(oz[0], (double)oq[0], (double)oq[3], mean3(P.h), P.inr2, p) : INFINITY;
}


// ---------------------------------------------------------------- one chunk
// One RK stage (STAGE 0: the first, else a later one; the combination in
// sc) of chunk c by a workgroup of NT lanes
// (chunk size C <= NT, chunk + ring 1 <= 2 NT, chunk-local edges <= 2 NT).
// The chunks of all members of a batch form one grid; each workgroup reads
// its member's forcing and control block.  The first stage also writes the
// post-processed w^n of its chunk to wpp, the RK base that the second stage
// reads.
template <int NT, class QT, int STAGE, bool VL, bool FE = (sizeof(QT) == 4)>
__device__ __forceinline__ void stage1_chunk(DevMesh m, DevState s, Params p, CSt<QT> win, CSt<QT> wbase,
                                             St<QT> wout, St<QT> wpp, StageCoef sc, int slot, int want_dt, int c,
                                             double *lds_raw, double *red) {
  const int tid = threadIdx.x;
  const size_t ne = (size_t)m.ne;
  const ChunkInfo k = chunk_info(m, c);
  const int mb = k.member;
  const Member &F = m.mem[mb];
  Ctrl *ctl = s.ctrl + mb;
  const Lds<QT> L = lds_view<QT>(m, lds_raw);
  const int nl = k.nl();

  // Phase L, round 1: the indices later loads depend on, for lane slots
  // i0 = tid, i1 = tid + NT of chunk + ring 1, ring-2 slot tid and chunk
  // element tid, and the control block.  Inactive slots read clamped, valid
  // positions; their values are never stored.
  const int i0 = tid, i1 = tid + NT;
  const bool a0 = i0 < nl, a1 = i1 < nl, ae = tid < k.cc, a2 = tid < k.n2;
  const int c0i = a0 ? i0 : nl - 1, c1i = a1 ? i1 : nl - 1, cei = ae ? tid : k.cc - 1;
  const int g0 = local_to_global(m, k, c0i);
  const int g1 = local_to_global(m, k, c1i);
  // clamped: a chunk without ring 2 reads the sentinel after the list
  const int g2 = m.h2[k.h2o + (a2 ? tid : (k.n2 > 0 ? k.n2 - 1 : 0))];
  int node[3];
  ElemPre<QT> pre;
  load_elem_node(m, k, cei, node, pre.ledge);
  // Round 2: loads that need no index.
  double h0[3], h1[3];
  uint16_t nb0[3], nb1[3];
  load_local_hb(m, k, c0i, h0);
  load_local_nb(m, k, c0i, nb0);
  load_local_hb(m, k, c1i, h1);
  load_local_nb(m, k, c1i, nb1);
  int4 ev0 = make_int4(0, 0, 0, 0), ev1 = ev0;
  if (VL) {
    ev0 = m.evb[g0];
    ev1 = m.evb[g1];
  }
  EdgeRec<QT> r0, r1;
  const int j0 = tid < k.ne_loc ? tid : k.ne_loc - 1, j1 = tid + NT < k.ne_loc ? tid + NT : k.ne_loc - 1;
  load_edge_rec(m, k, j0, r0);
  load_edge_rec(m, k, j1, r1);
  const bool use_base = STAGE != 0 && sc.a != 0.0;
  pre.manning = manning_of(m, k, cei, (QT)0);
  pre.coriolis = (QT)F.coriolis;
  pre.rain = F.rain;
  // Round 3: gathers through the indices (kept after round 2 in the
  // instruction stream, so the index loads return while round 2 is issued).
#ifdef __HIP_DEVICE_COMPILE__
  __builtin_amdgcn_sched_barrier(0);
#endif
  StateReg<QT> st0, st1;
  load_state_reg<QT>(win, ne, g0, st0);
  load_state_reg<QT>(win, ne, g1, st1);
  const double mz2 = win.z[g2];
  const QT mx2 = win.q[g2], my2 = win.q[3 * ne + g2];
  // Every lane reads its member's status word, dt, time and post-processing
  // flag (issued after the vector loads, whose addresses must not wait for
  // these scalar loads).  No lane leaves early, so the barriers stay
  // matched even if another workgroup changes the status meanwhile; an
  // inactive workgroup only stores nothing.
  const int status = ctl->status;
  const unsigned long long dtbits = ctl->dtmin[slot];
  const double t0 = ctl->t[slot];
  const int pp_in = STAGE == 0 ? ctl->pp_in : 1;
  const bool tide = F.n_tide > 0 || F.tide_offset != 0.0;
  for (int j = tid + NT; j < k.n2; j += NT) load_h2_lds<QT>(L, win, ne, j, m.h2[k.h2o + j]);
  // the go/no-go decision (uniform unless the status changes while the
  // workgroup reads it)
  double dt = 0.0;
  bool active = status == 0;
  if (!dt_from_bits(p, dtbits, dt)) {
    if (active && tid == 0) atomicCAS(&ctl->status, 0, (int)DGSWE_E_ALLDRY);
    active = false;
  }
  if (STAGE == 0 && active && k.first && tid == 0) ctl->dtmin[slot ^ 1] = double_to_bits(INFINITY);
  // the ocean tide at the stage time (its cosine waits for every load in
  // flight; here the state loads are about to be waited for anyway)
  const double ts = t0 + sc.c * dt;
  const double zb = tide ? tide_level(F, ts) : 0.0;
  if (a0) {
    store_state_lds<QT>(L, i0, st0);
    for (int q = 0; q < 3; ++q) L.LH[q * L.nls + i0] = h0[q];
  }
  if (a1) {
    store_state_lds<QT>(L, i1, st1);
    for (int q = 0; q < 3; ++q) L.LH[q * L.nls + i1] = h1[q];
  }
  if (a2) {
    L.MZ[tid] = mz2;
    L.MQ[tid] = mx2;
    L.MQ[L.n2s + tid] = my2;
  }
  __syncthreads();
  const bool to_wpp = STAGE == 0 && active;
  if (a0) phase_post<QT, VL>(p, k, L, pp_in, i0, h0, nb0, to_wpp, wpp, ne, s.vb, ev0);
  if (a1) phase_post<QT, VL>(p, k, L, pp_in, i1, h1, nb1, to_wpp, wpp, ne, s.vb, ev1);
  __syncthreads();
  // phase A's geometry (and with FE - by default in the mixed path, where
  // the registers allow - its nodal forcing) requested now, so it arrives
  // during phase E
  constexpr bool kForcingEarly = FE;
  GeoReg<QT> geo;
  load_geo(m, k, cei, geo, pre.inr2);
  if (kForcingEarly) load_elem_forcing<QT>(m, s, node, pre);
  if (tid < k.ne_loc) phase_edge<QT>(p, L, zb, tid, r0);
  if (tid + NT < k.ne_loc) phase_edge<QT>(p, L, zb, tid + NT, r1);
  __syncthreads();
  double cand = INFINITY;
  bool bad = false;
  if (ae && active)
    cand = phase_area<QT, kForcingEarly>(m, s, p, k, L, pre, node, geo, wbase, use_base, sc.a, sc.b, wout, ne,
                                         sc.h * dt, want_dt, tid, bad);
  if (bad) atomicCAS(&ctl->status, 0, (int)DGSWE_E_NONFINITE);
  if (want_dt) {
    const double bm = block_min<NT>(cand, red);
    if (tid == 0 && bm < INFINITY) atomicMin(&ctl->dtmin[slot ^ 1], double_to_bits(bm));
  }
  if (sc.last && active && k.first && tid == 0) {
    ctl->t[slot ^ 1] = t0 + dt;
    ctl->dt_last = dt;
    ctl->steps = ctl->steps + 1;
    ctl->pp_in = 1;  // the stored result is unlimited
  }
}


}  // namespace dgswe
