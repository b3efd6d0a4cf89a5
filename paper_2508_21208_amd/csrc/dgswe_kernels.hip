// gfx950 kernels of one SSP-RK(2,2) discontinuous Galerkin shallow-water
// step (arXiv 2508.21208, Sec. 2.2 and Sec. 5.2), FP64.
//
// One fused kernel per RK stage.  A workgroup owns a chunk of C consecutive
// elements (Hilbert order, so a compact patch of the mesh) and works in four
// phases separated by barriers, all intermediates in LDS:
//   L  load the chunk and its ring-1 halo (full state) and the ring-2 halo
//      (means) of the previous stage's UNLIMITED result;
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
// paper's WIND node loops).
#include "dgswe_internal.h"
#include "../../include/dgswe.h"

namespace dgswe {

#define HD __host__ __device__ __forceinline__
constexpr uint16_t kNone = 0xFFFF;

// ---------------------------------------------------------------- helpers
HD double bits_to_double(unsigned long long b) {
  union { unsigned long long u; double d; } x;
  x.u = b;
  return x.d;
}
HD unsigned long long double_to_bits(double d) {
  union { unsigned long long u; double d; } x;
  x.d = d;
  return x.u;
}

// Reciprocal, square root and cube root for the flux and source arithmetic:
// the hardware estimates refined by Newton (reciprocal, square root) or
// Halley (cube root) iterations, within about 1 ulp instead of the
// correctly rounded library sequences.  Arguments are finite and in the
// normal range (depths >= h0, lengths and areas of a mesh).
HD double rcp_nr(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
#else
  return 1.0 / x;
#endif
}

// sqrt(x) for x >= 0 (0 for x == 0)
HD double sqrt_nr(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  g = fma(d, h, g);
  return x > 0.0 ? g : 0.0;
#else
  return sqrt(x);
#endif
}

// cube root of x > 0: float estimate 2^(log2(x)/3), one Halley step
// y <- y (y^3 + 2x) / (2y^3 + x) (cubic convergence)
HD double cbrt_nr(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  const float xf = (float)x;
  double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf(xf) * (1.0f / 3.0f));
  const double y3 = y * y * y;
  y = y * (y3 + 2.0 * x) * rcp_nr(2.0 * y3 + x);
  return y;
#else
  return cbrt(x);
#endif
}

// dt of the current step: fixed, or cfl x the CFL minimum of w^n (capped).
// Returns false when no wet element defines it and there is no cap.
HD bool step_dt(const Ctrl *c, const Params &p, int slot, double &dt) {
  if (p.dt_fixed > 0.0) { dt = p.dt_fixed; return true; }
  double raw = bits_to_double(c->dtmin[slot]);
  if (raw == INFINITY) {
    if (p.dt_max > 0.0) { dt = p.dt_max; return true; }
    return false;
  }
  double d = p.cfl * raw;
  if (p.dt_max > 0.0 && d > p.dt_max) d = p.dt_max;
  dt = d;
  return true;
}

HD double tide_level(const Params &p, double t) {
  double z = p.tide_offset;
  for (int i = 0; i < p.n_tide; ++i) z += p.tide_amp[i] * cos(p.tide_omega[i] * t + p.tide_phase[i]);
  return z;
}

// hydrostatic flux g/2 (H^2 - h_b^2) written as g/2 zeta (zeta + 2 h_b)
HD double p_hydro(double g, double ze, double hb) { return 0.5 * g * ze * (ze + 2.0 * hb); }

// normal physical flux F(w).n of one side; u = 0 on a dry side
HD void flux_n(double g, double ze, double qx, double qy, double hb, bool wet, double nx, double ny,
               double &un, double f[3]) {
  const double H = ze + hb;
  const double qn = qx * nx + qy * ny;
  un = wet ? qn * rcp_nr(H) : 0.0;
  const double p = p_hydro(g, ze, hb);
  f[0] = qn;
  f[1] = qx * un + p * nx;
  f[2] = qy * un + p * ny;
}

// local Lax-Friedrichs flux from side L (normal n points from L to R)
HD void llf(double g, const double wl[3], const double wr[3], double hb, double nx, double ny,
            bool wetl, bool wetr, double out[3]) {
  double unl, unr, fl[3], fr[3];
  flux_n(g, wl[0], wl[1], wl[2], hb, wetl, nx, ny, unl, fl);
  flux_n(g, wr[0], wr[1], wr[2], hb, wetr, nx, ny, unr, fr);
  const double cl = sqrt_nr(g * fmax(wl[0] + hb, 0.0));
  const double cr = sqrt_nr(g * fmax(wr[0] + hb, 0.0));
  const double lam = fmax(fabs(unl) + cl, fabs(unr) + cr);
  for (int m = 0; m < 3; ++m) out[m] = 0.5 * (fl[m] + fr[m]) - 0.5 * lam * (wr[m] - wl[m]);
}

// land wall: LLF against the mirror state, closed form, zero mass flux
HD void wall(double g, const double w[3], double hb, double nx, double ny, bool wet, double out[3]) {
  const double p = p_hydro(g, w[0], hb);
  double f = p;
  if (wet) {
    const double H = w[0] + hb;
    const double iH = rcp_nr(H);
    const double qn = w[1] * nx + w[2] * ny;
    const double lam = fabs(qn) * iH + sqrt_nr(g * fmax(H, 0.0));
    f = qn * qn * iH + p + lam * qn;
  }
  out[0] = 0.0;
  out[1] = f * nx;
  out[2] = f * ny;
}

// p=1 vertex coefficients: value at vertex v = u0 + C1[v] u1 + C2[v] u2
HD double c1v(int v) { return v == 0 ? -1.0 : (v == 1 ? 1.0 : 0.0); }
HD double c2v(int v) { return v == 2 ? 2.0 : -1.0; }
// midpoint of local edge l (between vertices l+1 and l+2)
HD double c1m(int l) { return l == 0 ? 0.5 : (l == 1 ? -0.5 : 0.0); }
HD double c2m(int l) { return l == 2 ? -1.0 : 0.5; }

// gather weights: contribution to mode k of an element from the moments
// (P0, P1) of its local edge l is P0 (k=0), a1 P0 + b1 P1, a2 P0 + b2 P1
HD double ga1(int l) { return l == 0 ? 0.5 : (l == 1 ? -0.5 : 0.0); }
HD double gb1(int l) { return l == 2 ? 1.0 : -0.5; }
HD double ga2(int l) { return l == 2 ? -1.0 : 0.5; }
HD double gb2(int l) { return l == 0 ? 1.5 : (l == 1 ? -1.5 : 0.0); }

HD void holland(const Params &f, double x, double y, double t, double out[3]) {
  double cx = f.x0 + f.vx * t, cy = f.y0 + f.vy * t;
  double dx = x - cx, dy = y - cy;
  double r = sqrt(dx * dx + dy * dy);
  double pc = f.pn - f.dp;
  if (r <= 0.0) { out[0] = 0.0; out[1] = 0.0; out[2] = pc; return; }
  double a = pow(f.rmax / r, f.B);
  double e = exp(-a);
  double p = pc + f.dp * e;
  double rf2 = 0.5 * r * f.coriolis_f;
  double vg = sqrt(f.B * f.dp / f.rho_air * a * e + rf2 * rf2) - fabs(rf2);
  double ws = f.wind_factor * vg;
  double sgn = (f.coriolis_f < 0.0) ? -1.0 : 1.0;
  double wx = -sgn * ws * dy / r, wy = sgn * ws * dx / r;
  double cd = (0.75 + 0.067 * ws) * 1.0e-3;
  if (cd > 3.5e-3) cd = 3.5e-3;
  out[0] = f.rho_air * cd * ws * wx;
  out[1] = f.rho_air * cd * ws * wy;
  out[2] = p;
}

// ---------------------------------------------------------------- per-item math
// Post-processing of one element (slope limiter, then wet/dry).  u[9] is the
// unlimited state [var*3 + mode]; nbm[v][k] the unlimited mean of variable v
// of neighbour k (has[k] false: no neighbour); h[3] the vertex bathymetry.
HD void postprocess(double u[9], const double nbm[3][3], const bool has[3], const double h[3],
                    double hmean, const Params &p) {
  if (p.limiter) {
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

// One pass over the three Gauss-Lobatto points s = -1, 0, 1 (weights 1/3,
// 4/3, 1/3) of an edge in the e+ orientation, accumulating the flux moments
// m0 = sum_g w_g F_g and m1 = sum_g w_g s_g F_g (before the factor len/2)
// and the mass-flux integral.  kind 0: LLF between the two sides; 1: land
// wall seen from e+ (wet flag wetp); 2: wall seen from e- (normal -n).
struct EdgeGeo {
  double cp1[3], cp2[3], cm1[3], cm2[3];  // trace coefficients per point, e+ and e-
  double hq[3];                           // bathymetry at the points
  double nx, ny;
};

HD void edge_pass(int kind, const double up[9], const double um[9], bool ghost, double zb, bool wetp, bool wetm,
                  const EdgeGeo &G, const Params &p, double m0[3], double m1[3], double &mflux) {
  const double wq[3] = {1.0 / 3.0, 4.0 / 3.0, 1.0 / 3.0};
  for (int v = 0; v < 3; ++v) { m0[v] = 0.0; m1[v] = 0.0; }
  mflux = 0.0;
  for (int g = 0; g < 3; ++g) {
    double wp[3], wm[3], F[3];
    for (int v = 0; v < 3; ++v) wp[v] = up[3 * v] + G.cp1[g] * up[3 * v + 1] + G.cp2[g] * up[3 * v + 2];
    if (ghost) {
      wm[0] = zb; wm[1] = wp[1]; wm[2] = wp[2];
    } else {
      for (int v = 0; v < 3; ++v) wm[v] = um[3 * v] + G.cm1[g] * um[3 * v + 1] + G.cm2[g] * um[3 * v + 2];
    }
    if (kind == 0) llf(p.g, wp, wm, G.hq[g], G.nx, G.ny, wetp, wetm, F);
    else if (kind == 1) wall(p.g, wp, G.hq[g], G.nx, G.ny, wetp, F);
    else wall(p.g, wm, G.hq[g], -G.nx, -G.ny, true, F);
    const double sg = (double)(g - 1);
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
HD int edge_flux(const double up[9], const double um[9], int lp, int lm, int type, bool wetp, bool wetm_in,
                 double hA, double hB, double nx, double ny, double hl, double zb, const Params &p,
                 double mom[6]) {
  EdgeGeo G;
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
  double m0[3], m1[3], mflux;
  int mode;
  bool minus = false;
  if (type == DGSWE_BC_LAND) {
    edge_pass(1, up, um, true, zb, wetp, wetm, G, p, m0, m1, mflux);
    mode = 1;
  } else if (!wetp && !wetm) {
    for (int v = 0; v < 6; ++v) mom[v] = 0.0;
    return 3;
  } else {
    edge_pass(0, up, um, ghost, zb, wetp, wetm, G, p, m0, m1, mflux);
    mode = ghost ? 1 : 0;
    if (!(wetp && wetm)) {
      const bool flood = wetp ? (mflux > 0.0) : (mflux < 0.0);
      if (!flood) {
        if (wetp) {
          edge_pass(1, up, um, ghost, zb, true, wetm, G, p, m0, m1, mflux);
          mode = 1;
        } else if (ghost) {
          mode = 3;
        } else {
          edge_pass(2, up, um, false, zb, wetp, true, G, p, m0, m1, mflux);
          mode = 2;
          minus = true;
        }
      }
    }
  }
  // mode 2 holds the e- frame moments (P0, P1) with P1 along e-'s own
  // direction (-s); they are stored so that e- reads (-M0, M1) = (P0, P1)
  const double sgn = minus ? -1.0 : 1.0;
  for (int v = 0; v < 3; ++v) {
    mom[v] = sgn * hl * m0[v];
    mom[3 + v] = sgn * hl * m1[v];
  }
  return mode;
}

// Geometry and forcing of one element, as the area integrals need them.
struct ElemIn {
  double g1x, g1y, g2x, g2y, area;
  double h[3];
  double tx[3], ty[3], pa[3];
  double manning;
};

// Volume + source integrals of a post-processed state u; returns R_k / A
// (area part) in r[9]:  (1/3) [grad phi_k . sum_q F(w_q) + sum_q phi_k(q) s(w_q)].
HD void area_terms(const double u[9], bool wet, const ElemIn &E, const Params &p, double r[9]) {
  // gradient of a linear nodal field with vertex values f0, f1, f2: modes
  // (f1 - f0)/2 and (2 (f2 - f0) - (f1 - f0))/6 on grad phi_10, grad phi_01,
  // from vertex differences so a large common offset cancels exactly
  const double dh1 = E.h[1] - E.h[0], dh2 = E.h[2] - E.h[0];
  const double hm1 = 0.5 * dh1, hm2 = (2.0 * dh2 - dh1) * (1.0 / 6.0);
  const double dhx = hm1 * E.g1x + hm2 * E.g2x, dhy = hm1 * E.g1y + hm2 * E.g2y;
  const double dp1 = E.pa[1] - E.pa[0], dp2 = E.pa[2] - E.pa[0];
  const double pm1 = 0.5 * dp1, pm2 = (2.0 * dp2 - dp1) * (1.0 / 6.0);
  const double dpx = pm1 * E.g1x + pm2 * E.g2x, dpy = pm1 * E.g1y + pm2 * E.g2y;
  const double gn2 = p.g * E.manning * E.manning;
  const double irho = 1.0 / p.rho0;
  // area points: barycentric (2/3,1/6,1/6) and permutations; basis values
  // phi_10 = (-1/2, 1/2, 0), phi_01 = (-1/2, -1/2, 1)
  const double C1[3] = {-0.5, 0.5, 0.0}, C2[3] = {-0.5, -0.5, 1.0};
  const double L0[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
  const double L1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
  const double L2[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
  double sF[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  double S0[3] = {0, 0, 0}, S1[3] = {0, 0, 0}, S2[3] = {0, 0, 0};
  for (int q = 0; q < 3; ++q) {
    const double ze = u[0] + C1[q] * u[1] + C2[q] * u[2];
    const double qx = u[3] + C1[q] * u[4] + C2[q] * u[5];
    const double qy = u[6] + C1[q] * u[7] + C2[q] * u[8];
    const double hb = L0[q] * E.h[0] + L1[q] * E.h[1] + L2[q] * E.h[2];
    const double H = ze + hb;
    const double ph = p_hydro(p.g, ze, hb);
    double uu = 0.0, vv = 0.0;
    if (wet) {
      const double iH = rcp_nr(H);
      uu = qx * iH;
      vv = qy * iH;
    }
    sF[0][0] += qx;            sF[0][1] += qy;
    sF[1][0] += qx * uu + ph;  sF[1][1] += qx * vv;
    sF[2][0] += qy * uu;       sF[2][1] += qy * vv + ph;
    if (wet) {
      const double Hf = fmax(H, p.h0);
      const double qm = sqrt_nr(qx * qx + qy * qy);
      const double fr = gn2 * qm * rcp_nr(Hf * Hf * cbrt_nr(Hf));
      const double txq = L0[q] * E.tx[0] + L1[q] * E.tx[1] + L2[q] * E.tx[2];
      const double tyq = L0[q] * E.ty[0] + L1[q] * E.ty[1] + L2[q] * E.ty[2];
      const double sx = p.g * ze * dhx - fr * qx + txq * irho - H * irho * dpx;
      const double sy = p.g * ze * dhy - fr * qy + tyq * irho - H * irho * dpy;
      S0[1] += sx;          S0[2] += sy;
      S1[1] += C1[q] * sx;  S1[2] += C1[q] * sy;
      S2[1] += C2[q] * sx;  S2[2] += C2[q] * sy;
    }
  }
  for (int v = 0; v < 3; ++v) {
    r[3 * v + 0] = S0[v] * (1.0 / 3.0);
    r[3 * v + 1] = (E.g1x * sF[v][0] + E.g1y * sF[v][1] + S1[v]) * (1.0 / 3.0);
    r[3 * v + 2] = (E.g2x * sF[v][0] + E.g2y * sF[v][1] + S2[v]) * (1.0 / 3.0);
  }
}

// CFL candidate 2 r_e / (|Q_mean| / H_mean + sqrt(g H_mean)) of a state
// (INFINITY when dry); unchanged by the post-processing.
HD double cfl_candidate(const double u[9], double hmean, double inr2, const Params &p) {
  const double Hm = u[0] + hmean;
  const bool wet = p.wetdry ? (Hm > p.h0) : true;
  if (!wet) return INFINITY;
  const double lam = sqrt(u[3] * u[3] + u[6] * u[6]) / Hm + sqrt(p.g * Hm);
  return inr2 / lam;
}

HD double mean3(const double h[3]) { return (h[0] + h[1] + h[2]) / 3.0; }

// ---------------------------------------------------------------- global-memory views
// Element e of a [9][ne] state, post-processed with neighbour means read
// from the same array (used for the RK base and read-back).
HD void load_pp_global(const DevMesh &m, const Params &p, const double *w, int e, bool pp, double u[9],
                       double h[3]) {
  const size_t ne = (size_t)m.ne;
  for (int j = 0; j < 9; ++j) u[j] = w[j * ne + e];
  for (int k = 0; k < 3; ++k) h[k] = m.hbv[k * ne + e];
  if (!pp) return;
  double nbm[3][3];
  bool has[3];
  for (int k = 0; k < 3; ++k) {
    const int f = m.el_nb[k * ne + e];
    has[k] = f >= 0;
    for (int v = 0; v < 3; ++v) nbm[v][k] = has[k] ? w[(size_t)(3 * v) * ne + f] : 0.0;
  }
  postprocess(u, nbm, has, h, mean3(h), p);
}

HD void load_elem_in(const DevMesh &m, const DevState &s, const Params &p, int e, ElemIn &E) {
  const size_t ne = (size_t)m.ne, nn = (size_t)m.nn;
  E.g1x = m.gx1[e]; E.g1y = m.gy1[e]; E.g2x = m.gx2[e]; E.g2y = m.gy2[e];
  E.area = m.area[e];
  for (int k = 0; k < 3; ++k) {
    E.h[k] = m.hbv[k * ne + e];
    const int nd = m.el_node[k * ne + e];
    E.tx[k] = s.nodal[nd];
    E.ty[k] = s.nodal[nn + nd];
    E.pa[k] = s.nodal[2 * nn + nd];
  }
  E.manning = m.manning ? m.manning[e] : p.manning_n;
}

// ---------------------------------------------------------------- fused stage phases
// LDS layout of one chunk (sizes from the mesh maxima):
//   S[9][nl_max]  states of chunk + ring 1 (post-processed in phase P)
//   MQ[2][nm_max] unlimited Qx, Qy means of chunk + ring 1 + ring 2
//   MZ[n2_max]    unlimited zeta means of ring 2 (the zeta mean of chunk and
//                 ring 1 is S[0][i], which the post-processing never changes)
//   EM[6][ed_max] edge moments
//   GEO[5][C]     gradients of phi_10, phi_01 and area of the chunk elements
//   EMODE[ed_max], WET[nl_max]
struct Lds {
  double *S, *MQ, *MZ, *EM, *GEO;
  unsigned char *EMODE, *WET;
  int nls, nms, eds, cs;  // strides
};

HD Lds lds_view(const DevMesh &m, void *base) {
  Lds L;
  L.nls = m.nl_max; L.nms = m.nm_max; L.eds = m.ed_max; L.cs = m.C;
  L.S = (double *)base;
  L.MQ = L.S + 9 * (size_t)L.nls;
  L.MZ = L.MQ + 2 * (size_t)L.nms;
  L.EM = L.MZ + (size_t)m.n2_max;
  L.GEO = L.EM + 6 * (size_t)L.eds;
  L.EMODE = (unsigned char *)(L.GEO + 5 * (size_t)L.cs);
  L.WET = L.EMODE + L.eds;
  return L;
}

struct ChunkInfo {
  int c, c0, cc, h1o, n1, h2o, n2, leo, ne_loc, nbo;
  HD int nl() const { return cc + n1; }
};

HD ChunkInfo chunk_info(const DevMesh &m, int c) {
  ChunkInfo k;
  k.c = c;
  k.c0 = c * m.C;
  k.cc = m.ne - k.c0 < m.C ? m.ne - k.c0 : m.C;
  k.h1o = m.h1_off[c]; k.n1 = m.h1_off[c + 1] - k.h1o;
  k.h2o = m.h2_off[c]; k.n2 = m.h2_off[c + 1] - k.h2o;
  k.leo = m.le_off[c]; k.ne_loc = m.le_off[c + 1] - k.leo;
  k.nbo = m.nb_off[c];
  return k;
}

// one chunk-local edge record, loaded early and kept in registers
struct EdgeRec {
  uint32_t pm;
  int info;
  double nx, ny, hl, hA, hB;
};

HD void load_edge_rec(const DevMesh &m, const ChunkInfo &k, int j, EdgeRec &R) {
  const size_t r = (size_t)(k.leo + j);
  R.pm = m.le_pm[r]; R.info = m.le_info[r];
  R.nx = m.le_nx[r]; R.ny = m.le_ny[r]; R.hl = m.le_hl[r]; R.hA = m.le_hA[r]; R.hB = m.le_hB[r];
}

// vertex bathymetry of local element i (chunk: element arrays; ring 1:
// packed per chunk)
HD void load_local_hb(const DevMesh &m, const ChunkInfo &k, int i, double h[3]) {
  const size_t ne = (size_t)m.ne;
  if (i < k.cc) {
    for (int q = 0; q < 3; ++q) h[q] = m.hbv[q * ne + k.c0 + i];
  } else {
    const size_t nh1 = (size_t)m.h1_off[m.nch];
    const size_t r = (size_t)(k.h1o + i - k.cc);
    for (int q = 0; q < 3; ++q) h[q] = m.h1_hb[q * nh1 + r];
  }
}

// phase L for local element i of chunk + ring 1
HD void phase_load_nl(const DevMesh &m, const ChunkInfo &k, const Lds &L, const double *win, int i) {
  const size_t ne = (size_t)m.ne;
  const int g = i < k.cc ? k.c0 + i : m.h1[k.h1o + i - k.cc];
  double u[9];
  for (int j = 0; j < 9; ++j) u[j] = win[j * ne + g];
  for (int j = 0; j < 9; ++j) L.S[j * L.nls + i] = u[j];
  L.MQ[i] = u[3];
  L.MQ[L.nms + i] = u[6];
}

// phase L for ring-2 element j (means only)
HD void phase_load_h2(const DevMesh &m, const ChunkInfo &k, const Lds &L, const double *win, int j) {
  const size_t ne = (size_t)m.ne;
  const int g = m.h2[k.h2o + j];
  L.MZ[j] = win[g];
  L.MQ[k.nl() + j] = win[3 * ne + g];
  L.MQ[L.nms + k.nl() + j] = win[6 * ne + g];
}

// phase L: geometry of chunk element i into LDS
HD void phase_load_geo(const DevMesh &m, const ChunkInfo &k, const Lds &L, int i) {
  const int e = k.c0 + i;
  L.GEO[i] = m.gx1[e];
  L.GEO[L.cs + i] = m.gy1[e];
  L.GEO[2 * L.cs + i] = m.gx2[e];
  L.GEO[3 * L.cs + i] = m.gy2[e];
  L.GEO[4 * L.cs + i] = m.area[e];
}

// phase P for local element i of chunk + ring 1 (h: its vertex bathymetry);
// the post-processed state of a chunk element also goes to wpp if given
// local neighbour indices of local element i (chunk + ring 1)
HD void load_local_nb(const DevMesh &m, const ChunkInfo &k, int i, uint16_t nb[3]) {
  const int nl = k.nl();
  for (int q = 0; q < 3; ++q) nb[q] = m.nbl[k.nbo + q * nl + i];
}

HD void phase_post(const DevMesh &m, const Params &p, const ChunkInfo &k, const Lds &L, int pp_in, int i,
                   const double h[3], const uint16_t nb[3], double *wpp) {
  const int nl = k.nl();
  const double hmean = mean3(h);
  double u[9];
  for (int j = 0; j < 9; ++j) u[j] = L.S[j * L.nls + i];
  if (pp_in) {
    double nbm[3][3];
    bool has[3];
    for (int q = 0; q < 3; ++q) {
      const uint16_t f = nb[q];
      has[q] = f != kNone;
      const int fi = has[q] ? f : 0;
      nbm[0][q] = fi < nl ? L.S[fi] : L.MZ[fi - nl];
      nbm[1][q] = L.MQ[fi];
      nbm[2][q] = L.MQ[L.nms + fi];
    }
    postprocess(u, nbm, has, h, hmean, p);
    // the zeta mean S[0][i] is unchanged (neighbours read it concurrently)
    for (int j = 1; j < 9; ++j) L.S[j * L.nls + i] = u[j];
  }
  L.WET[i] = (p.wetdry ? (u[0] + hmean > p.h0) : true) ? 1 : 0;
  if (wpp && i < k.cc) {
    const size_t ne = (size_t)m.ne;
    for (int j = 0; j < 9; ++j) wpp[j * ne + k.c0 + i] = u[j];
  }
}

// phase E for chunk-local edge j with its record
HD void phase_edge(const Params &p, const Lds &L, double zb, int j, const EdgeRec &R) {
  const int lp = R.info & 3, lm = (R.info >> 2) & 3, type = R.info >> 4;
  const int ip = (int)(R.pm & 0xFFFFu), im = (int)(R.pm >> 16);
  double up[9], um[9];
  for (int q = 0; q < 9; ++q) up[q] = L.S[q * L.nls + ip];
  bool wetm = false;
  if (type == 0) {
    for (int q = 0; q < 9; ++q) um[q] = L.S[q * L.nls + im];
    wetm = L.WET[im] != 0;
  } else {
    for (int q = 0; q < 9; ++q) um[q] = 0.0;
  }
  double mom[6];
  const int mode = edge_flux(up, um, lp, lm, type, L.WET[ip] != 0, wetm, R.hA, R.hB, R.nx, R.ny, R.hl, zb, p, mom);
  for (int q = 0; q < 6; ++q) L.EM[q * L.eds + j] = mom[q];
  L.EMODE[j] = (unsigned char)mode;
}

// per-element inputs of phase A, loaded in phase L and kept in registers
// (nodal forcing at the vertices, RK base on the second stage)
struct ElemPre {
  double h[3];
  double tx[3], ty[3], pa[3];
  double wb[9];
  double inr2, manning;
  int ledge[3];
};

HD void load_elem_pre(const DevMesh &m, const DevState &s, const Params &p, const ChunkInfo &k, int i,
                      const double *wbase, ElemPre &P) {
  const size_t ne = (size_t)m.ne, nn = (size_t)m.nn;
  const int e = k.c0 + i;
  int node[3];
  for (int q = 0; q < 3; ++q) {
    P.h[q] = m.hbv[q * ne + e];
    node[q] = m.el_node[q * ne + e];
    P.ledge[q] = m.el_ledge[q * ne + e];
  }
  P.inr2 = m.inr2[e];
  P.manning = m.manning ? m.manning[e] : p.manning_n;
  for (int q = 0; q < 3; ++q) {
    P.tx[q] = s.nodal[node[q]];
    P.ty[q] = s.nodal[nn + node[q]];
    P.pa[q] = s.nodal[2 * nn + node[q]];
  }
  if (wbase)
    for (int j = 0; j < 9; ++j) P.wb[j] = wbase[j * ne + e];
}

// phase A for chunk element i; returns the CFL candidate of the output when
// want_dt, and sets bad on a non-finite output.  base: combine with the
// post-processed RK base P.wb (second stage).
HD double phase_area(const DevMesh &m, const Params &p, const ChunkInfo &k, const Lds &L, const ElemPre &P,
                     bool base, double *wout, double dt, int want_dt, int i, bool &bad) {
  const size_t ne = (size_t)m.ne;
  const int e = k.c0 + i;
  ElemIn E;
  for (int q = 0; q < 3; ++q) {
    E.h[q] = P.h[q];
    E.tx[q] = P.tx[q];
    E.ty[q] = P.ty[q];
    E.pa[q] = P.pa[q];
  }
  E.manning = P.manning;
  E.g1x = L.GEO[i]; E.g1y = L.GEO[L.cs + i]; E.g2x = L.GEO[2 * L.cs + i]; E.g2y = L.GEO[3 * L.cs + i];
  E.area = L.GEO[4 * L.cs + i];
  double u[9];
  for (int j = 0; j < 9; ++j) u[j] = L.S[j * L.nls + i];
  const bool wet = L.WET[i] != 0;
  double r[9];
  area_terms(u, wet, E, p, r);
  // fixed-order gather of the three edges: R_k / A -= edge_k / A
  const double iA = rcp_nr(E.area);
  for (int l = 0; l < 3; ++l) {
    const int code = P.ledge[l];
    const int j = code >> 1, side = code & 1;
    const int md = L.EMODE[j];
    if (md == 3 || md == 2 - side) continue;  // this side receives nothing
    const double sg = side ? -iA : iA;
    const double a1 = ga1(l), b1 = gb1(l), a2 = ga2(l), b2 = gb2(l);
    for (int v = 0; v < 3; ++v) {
      const double P0 = sg * L.EM[v * L.eds + j];
      const double P1 = iA * L.EM[(3 + v) * L.eds + j];
      r[3 * v + 0] -= P0;
      r[3 * v + 1] -= a1 * P0 + b1 * P1;
      r[3 * v + 2] -= a2 * P0 + b2 * P1;
    }
  }
  const double imu[3] = {1.0, 6.0, 2.0};
  bool fin = true;
  double out[9];
  for (int j = 0; j < 9; ++j) {
    double dw = r[j] * imu[j % 3];
    if (!wet && j >= 3) dw = 0.0;
    out[j] = base ? 0.5 * P.wb[j] + 0.5 * (u[j] + dt * dw) : u[j] + dt * dw;
    wout[j * ne + e] = out[j];
    fin = fin && __builtin_isfinite(out[j]);
  }
  bad = !fin;
  return want_dt ? cfl_candidate(out, mean3(E.h), P.inr2, p) : INFINITY;
}

#undef HD

// ---------------------------------------------------------------- kernels
template <int NT>
__device__ __forceinline__ double block_min(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = 1; i < NT / 64; ++i) v = fmin(v, red[i]);
  return v;  // valid in thread 0
}

// XCD-aware chunk order: consecutive workgroups land on different XCDs
// (round robin over 8), so XCD x processes the contiguous chunk range
// [x * nch / 8, (x + 1) * nch / 8) and neighbouring chunks share its L2.
__device__ __forceinline__ int chunk_of_block(int b, int nch) {
  const int nx = 8;
  const int per = nch / nx, rem = nch % nx;
  const int x = b % nx, r = b / nx;
  const int start = x * per + (x < rem ? x : rem);
  const int len = per + (x < rem ? 1 : 0);
  if (r < len) return start + r;
  return -1;
}

__global__ __launch_bounds__(kBlock) void k_forcing(DevMesh m, DevState s, Params p, int slot, int stage) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (s.ctrl->status) return;
  double dt;
  if (!step_dt(s.ctrl, p, slot, dt)) return;
  if (i >= m.nn) return;
  double out[3];
  holland(p, m.node_x[i], m.node_y[i], s.ctrl->t[slot] + (stage ? dt : 0.0), out);
  s.nodal[i] = out[0];
  s.nodal[(size_t)m.nn + i] = out[1];
  s.nodal[2 * (size_t)m.nn + i] = out[2];
}

// One RK stage over one chunk per workgroup of NT lanes (chunk size
// C <= NT, chunk + ring 1 <= 2 NT, chunk-local edges <= 2 NT).  Stage 1
// (stage == 0) also writes the post-processed w^n of its chunk to wpp, the
// RK base that stage 2 reads.
template <int NT, int WPE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void k_stage(
    DevMesh m, DevState s, Params p, const double *__restrict__ win, const double *__restrict__ wbase,
    double *__restrict__ wout, double *__restrict__ wpp, int slot, int stage, int pp_in, int want_dt) {
  extern __shared__ double lds_raw[];
  __shared__ double red[NT / 64];
  __shared__ int s_active;
  Ctrl *ctl = s.ctrl;
  const int tid = threadIdx.x;
  double dt = 0.0;
  // the go/no-go decision is taken once per block, so every lane reaches the
  // same barriers
  if (tid == 0) {
    int act = ctl->status == 0 ? 1 : 0;
    if (act && !step_dt(ctl, p, slot, dt)) {
      atomicCAS(&ctl->status, 0, (int)DGSWE_E_ALLDRY);
      act = 0;
    }
    s_active = act;
  }
  __syncthreads();
  if (!s_active) return;
  step_dt(ctl, p, slot, dt);
  const int c = chunk_of_block(blockIdx.x, m.nch);
  if (c < 0) return;
  const ChunkInfo k = chunk_info(m, c);
  const Lds L = lds_view(m, lds_raw);
  const int nl = k.nl();
  if (stage == 0 && blockIdx.x == 0 && tid == 0) ctl->dtmin[slot ^ 1] = double_to_bits(INFINITY);

  // phase L, with the loads of the later phases issued early
  const int i0 = tid, i1 = tid + NT;
  double h0[3], h1[3];
  uint16_t nb0[3], nb1[3];
  if (i0 < nl) { load_local_hb(m, k, i0, h0); load_local_nb(m, k, i0, nb0); }
  if (i1 < nl) { load_local_hb(m, k, i1, h1); load_local_nb(m, k, i1, nb1); }
  EdgeRec r0, r1;
  if (tid < k.ne_loc) load_edge_rec(m, k, tid, r0);
  if (tid + NT < k.ne_loc) load_edge_rec(m, k, tid + NT, r1);
  ElemPre pre;
  if (tid < k.cc) {
    load_elem_pre(m, s, p, k, tid, stage ? wbase : nullptr, pre);
    phase_load_geo(m, k, L, tid);
  }
  if (i0 < nl) phase_load_nl(m, k, L, win, i0);
  if (i1 < nl) phase_load_nl(m, k, L, win, i1);
  for (int j = tid; j < k.n2; j += NT) phase_load_h2(m, k, L, win, j);
  __syncthreads();
  double *wpp_out = stage == 0 ? wpp : nullptr;
  if (i0 < nl) phase_post(m, p, k, L, pp_in, i0, h0, nb0, wpp_out);
  if (i1 < nl) phase_post(m, p, k, L, pp_in, i1, h1, nb1, wpp_out);
  __syncthreads();
  const double ts = ctl->t[slot] + (stage ? dt : 0.0);
  const double zb = (p.n_tide > 0 || p.tide_offset != 0.0) ? tide_level(p, ts) : 0.0;
  if (tid < k.ne_loc) phase_edge(p, L, zb, tid, r0);
  if (tid + NT < k.ne_loc) phase_edge(p, L, zb, tid + NT, r1);
  __syncthreads();
  double cand = INFINITY;
  bool bad = false;
  if (tid < k.cc) cand = phase_area(m, p, k, L, pre, stage != 0, wout, dt, want_dt, tid, bad);
  if (bad) atomicCAS(&ctl->status, 0, (int)DGSWE_E_NONFINITE);
  if (want_dt) {
    const double bm = block_min<NT>(cand, red);
    if (tid == 0 && bm < INFINITY) atomicMin(&ctl->dtmin[slot ^ 1], double_to_bits(bm));
  }
  if (stage == 1 && blockIdx.x == 0 && tid == 0) {
    ctl->t[slot ^ 1] = ctl->t[slot] + dt;
    ctl->dt_last = dt;
    ctl->steps = ctl->steps + 1;
  }
}

// post-processing of a whole state (win -> wout)
__global__ __launch_bounds__(kBlock) void k_post_only(DevMesh m, Params p, const double *__restrict__ win,
                                                      double *__restrict__ wout) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= m.ne) return;
  double u[9], h[3];
  load_pp_global(m, p, win, e, true, u, h);
  for (int j = 0; j < 9; ++j) wout[(size_t)j * m.ne + e] = u[j];
}

__global__ void k_ctrl_reset(Ctrl *c, double t) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->t[0] = t;
    c->t[1] = t;
    c->dt_last = 0.0;
    c->dtmin[0] = double_to_bits(INFINITY);
    c->dtmin[1] = double_to_bits(INFINITY);
    c->steps = 0;
    c->status = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_init(DevMesh m, DevState s, Params p, const double *__restrict__ w) {
  __shared__ double red[kBlock / 64];
  const int e = blockIdx.x * kBlock + threadIdx.x;
  double cand = INFINITY;
  if (e < m.ne) {
    const size_t ne = (size_t)m.ne;
    double u[9];
    for (int j = 0; j < 9; ++j) u[j] = w[j * ne + e];
    const double h[3] = {m.hbv[e], m.hbv[ne + e], m.hbv[2 * ne + e]};
    cand = cfl_candidate(u, mean3(h), m.inr2[e], p);
  }
  const double bm = block_min<kBlock>(cand, red);
  if (threadIdx.x == 0 && bm < INFINITY) atomicMin(&s.ctrl->dtmin[0], double_to_bits(bm));
}

// Diagnostics: per-block partial sums (mass, volume, wet count), then one
// block adds the partials in a fixed order: deterministic.  Mean depth and
// zeta mean are unchanged by the post-processing, so the unlimited state
// gives the same values.
__global__ __launch_bounds__(kBlock) void k_diag1(DevMesh m, DevState s, Params p, const double *__restrict__ w) {
  __shared__ double sm[3][kBlock];
  const int e = blockIdx.x * kBlock + threadIdx.x;
  const size_t ne = (size_t)m.ne;
  double a = 0.0, b = 0.0, c = 0.0;
  if (e < m.ne) {
    const double h[3] = {m.hbv[e], m.hbv[ne + e], m.hbv[2 * ne + e]};
    const double hmean = mean3(h);
    const double z = w[e];
    a = m.area[e] * z;
    b = m.area[e] * (z + hmean);
    c = (p.wetdry ? (z + hmean > p.h0) : true) ? 1.0 : 0.0;
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
    s.partial[blockIdx.x] = sm[0][0];
    s.partial[nb + blockIdx.x] = sm[1][0];
    s.partial[2 * nb + blockIdx.x] = sm[2][0];
  }
}

__global__ __launch_bounds__(kBlock) void k_diag2(DevState s, int nb, double *out) {
  __shared__ double sm[3][kBlock];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nb; i += kBlock)
    for (int q = 0; q < 3; ++q) acc[q] += s.partial[(size_t)q * nb + i];
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
    out[3] = 0.0;
  }
}

// ---------------------------------------------------------------- launchers
static inline unsigned nblk(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

int diag_blocks(int ne) { return (int)nblk(ne); }

size_t stage_lds_bytes(const DevMesh &m) {
  return 8 * (9 * (size_t)m.nl_max + 2 * (size_t)m.nm_max + (size_t)m.n2_max + 6 * (size_t)m.ed_max +
              5 * (size_t)m.C) +
         (size_t)m.ed_max + (size_t)m.nl_max;
}

bool stage_block_ok(int block) {
  for (int b : kStageBlocks)
    if (b == block) return true;
  return false;
}

hipError_t launch_forcing(const DevMesh &m, const DevState &s, const Params &p, int slot, int stage,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_forcing, dim3(nblk(m.nn)), dim3(kBlock), 0, st, m, s, p, slot, stage);
  return hipGetLastError();
}

hipError_t launch_stage(const DevMesh &m, const DevState &s, const Params &p, const double *win,
                        const double *wbase, double *wout, double *wpp, int slot, int stage, int pp_in,
                        int want_dt, int block, hipStream_t st) {
  const size_t lds = stage_lds_bytes(m);
#define DGSWE_STAGE(NT, W)                                                                                  \
  hipLaunchKernelGGL((k_stage<NT, W>), dim3(m.nch), dim3(NT), lds, st, m, s, p, win, wbase, wout, wpp, slot, \
                     stage, pp_in, want_dt)
  switch (block) {
    case 384: DGSWE_STAGE(384, 3); break;
    default: DGSWE_STAGE(256, 2); break;
  }
#undef DGSWE_STAGE
  return hipGetLastError();
}

hipError_t launch_post_only(const DevMesh &m, const DevState &s, const Params &p, const double *win, double *wout,
                            hipStream_t st) {
  (void)s;
  hipLaunchKernelGGL(k_post_only, dim3(nblk(m.ne)), dim3(kBlock), 0, st, m, p, win, wout);
  return hipGetLastError();
}

hipError_t launch_init_state(const DevMesh &m, const DevState &s, const Params &p, const double *w, double t,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, st, s.ctrl, t);
  hipLaunchKernelGGL(k_init, dim3(nblk(m.ne)), dim3(kBlock), 0, st, m, s, p, w);
  return hipGetLastError();
}

hipError_t launch_diag(const DevMesh &m, const DevState &s, const Params &p, const double *w, double *out4,
                       hipStream_t st) {
  const int nb = (int)nblk(m.ne);
  hipLaunchKernelGGL(k_diag1, dim3(nb), dim3(kBlock), 0, st, m, s, p, w);
  hipLaunchKernelGGL(k_diag2, dim3(1), dim3(kBlock), 0, st, s, nb, out4);
  return hipGetLastError();
}

}  // namespace dgswe
