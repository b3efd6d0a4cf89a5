// gfx950 kernels of one SSP-RK(2,2) discontinuous Galerkin shallow-water
// step (arXiv 2508.21208, Sec. 2.2 and Sec. 5.2), FP64.
//
// Per stage:
//   k_forcing  one lane per mesh node: Holland wind stress and pressure at
//              the stage time (the paper's WIND node loops, Sec. 5.2)
//   k_edge     one lane per edge: traces of both elements at the three
//              Gauss-Lobatto points, local Lax-Friedrichs flux with the
//              wet/dry rules, evaluated ONCE per edge; the two flux moments
//              (integral of F and of s F along the edge) go to an edge buffer
//              (Algorithm 2 writes per-element slots instead)
//   k_element  one lane per element: volume and source integrals at the three
//              area points (Algorithm 1), then the fixed-order gather of its
//              three edges (Algorithm 3), the inverse diagonal mass matrix and
//              the Shu-Osher RK combination
//   k_post     one lane per element: slope limiter and wet/dry (SLOPELIM,
//              WETDRY), the wet flags of the next stage, the CFL candidate
//              of the next step (block min + one 64-bit integer atomicMin:
//              exact, so independent of order) and the time advance
// Element-indexed arrays are structure-of-arrays in a Hilbert order, so a
// wavefront streams 64 consecutive elements per array and the neighbour
// gathers of the edge and limiter kernels stay in the L2.  No floating-point
// atomics: every result is deterministic.
#include "dgswe_internal.h"
#include "../../include/dgswe.h"

namespace dgswe {

#define HD __host__ __device__ __forceinline__

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
  double H = ze + hb;
  double qn = qx * nx + qy * ny;
  un = wet ? qn / H : 0.0;
  double p = p_hydro(g, ze, hb);
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
  double cl = sqrt(g * fmax(wl[0] + hb, 0.0));
  double cr = sqrt(g * fmax(wr[0] + hb, 0.0));
  double lam = fmax(fabs(unl) + cl, fabs(unr) + cr);
  for (int m = 0; m < 3; ++m) out[m] = 0.5 * (fl[m] + fr[m]) - 0.5 * lam * (wr[m] - wl[m]);
}

// land wall: LLF against the mirror state, closed form, zero mass flux
HD void wall(double g, const double w[3], double hb, double nx, double ny, bool wet, double out[3]) {
  double p = p_hydro(g, w[0], hb);
  double f = p;
  if (wet) {
    double H = w[0] + hb;
    double qn = w[1] * nx + w[2] * ny;
    double lam = fabs(qn) / H + sqrt(g * fmax(H, 0.0));
    f = qn * qn / H + p + lam * qn;
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

// ---------------------------------------------------------------- bodies
HD void forcing_body(int i, const DevMesh &m, const DevState &s, const Params &p, double t) {
  double out[3];
  holland(p, m.node_x[i], m.node_y[i], t, out);
  s.nodal[i] = out[0];
  s.nodal[(size_t)m.nn + i] = out[1];
  s.nodal[2 * (size_t)m.nn + i] = out[2];
}

// Edge flux moments.  For the three Gauss-Lobatto points s = -1, 0, 1
// (weights 1/3, 4/3, 1/3) along the e+ orientation:
//   M0 = len/2 sum_g w_g F_g,  M1 = len/2 sum_g w_g s_g F_g  (e+ frame).
// e+ receives (M0, M1), e- receives (-M0, M1) in its own frame; emode says
// which sides receive anything (0 both, 1 e+ only, 2 e- only, 3 none).
HD void edge_body(int d, const DevMesh &m, const DevState &s, const Params &p, const double *w,
                  double zb) {
  const size_t ne = (size_t)m.ne, ned = (size_t)m.ned;
  const int ep = m.ed_ep[d], em = m.ed_em[d], info = m.ed_info[d];
  const int lp = info & 3, lm = (info >> 2) & 3, type = info >> 4;
  const double nx = m.ed_nx[d], ny = m.ed_ny[d], hl = m.ed_hlen[d];
  const int va = lp == 2 ? 0 : lp + 1, vb = lp == 0 ? 2 : lp - 1;
  const double hA = m.hbv[va * ne + ep], hB = m.hbv[vb * ne + ep];
  const double hq[3] = {hA, hA * 0.5 + hB * 0.5, hB};
  double up[9];
  for (int j = 0; j < 9; ++j) up[j] = w[j * ne + ep];
  double wp[3][3], wm[3][3];
  for (int v = 0; v < 3; ++v) {
    wp[0][v] = up[3 * v] + c1v(va) * up[3 * v + 1] + c2v(va) * up[3 * v + 2];
    wp[1][v] = up[3 * v] + c1m(lp) * up[3 * v + 1] + c2m(lp) * up[3 * v + 2];
    wp[2][v] = up[3 * v] + c1v(vb) * up[3 * v + 1] + c2v(vb) * up[3 * v + 2];
  }
  const bool wetp = s.wet[ep] != 0;
  bool wetm = false;
  if (type == 0) {
    double um[9];
    for (int j = 0; j < 9; ++j) um[j] = w[j * ne + em];
    // e- runs the edge backwards: its vertex (lm+2) sits at s = -1
    const int ma = lm == 2 ? 0 : lm + 1, mb = lm == 0 ? 2 : lm - 1;
    for (int v = 0; v < 3; ++v) {
      wm[0][v] = um[3 * v] + c1v(mb) * um[3 * v + 1] + c2v(mb) * um[3 * v + 2];
      wm[1][v] = um[3 * v] + c1m(lm) * um[3 * v + 1] + c2m(lm) * um[3 * v + 2];
      wm[2][v] = um[3 * v] + c1v(ma) * um[3 * v + 1] + c2v(ma) * um[3 * v + 2];
    }
    wetm = s.wet[em] != 0;
  } else {
    for (int g = 0; g < 3; ++g) { wm[g][0] = zb; wm[g][1] = wp[g][1]; wm[g][2] = wp[g][2]; }
    wetm = p.wetdry ? (zb + 0.5 * (hA + hB) > p.h0) : true;
  }
  double F[3][3];
  int mode = 0;
  bool store_minus = false;  // F holds the e- frame flux (mode 2)
  if (type == DGSWE_BC_LAND) {
    for (int g = 0; g < 3; ++g) wall(p.g, wp[g], hq[g], nx, ny, wetp, F[g]);
    mode = 1;
  } else if (!wetp && !wetm) {
    for (int g = 0; g < 3; ++g) F[g][0] = F[g][1] = F[g][2] = 0.0;
    mode = 3;
  } else {
    for (int g = 0; g < 3; ++g) llf(p.g, wp[g], wm[g], hq[g], nx, ny, wetp, wetm, F[g]);
    bool flood = true;
    if (!(wetp && wetm)) {
      double mflux = 0.0;
      mflux += (1.0 / 3.0) * F[0][0];
      mflux += (4.0 / 3.0) * F[1][0];
      mflux += (1.0 / 3.0) * F[2][0];
      flood = wetp ? (mflux > 0.0) : (mflux < 0.0);
    }
    if (type == DGSWE_BC_OCEAN) {
      mode = 1;
      if (!flood && wetp)
        for (int g = 0; g < 3; ++g) wall(p.g, wp[g], hq[g], nx, ny, true, F[g]);
      else if (!flood)
        mode = 3;
    } else if (!flood) {
      if (wetp) {
        for (int g = 0; g < 3; ++g) wall(p.g, wp[g], hq[g], nx, ny, true, F[g]);
        mode = 1;
      } else {
        for (int g = 0; g < 3; ++g) wall(p.g, wm[g], hq[g], -nx, -ny, true, F[g]);
        mode = 2;
        store_minus = true;
      }
    }
  }
  for (int v = 0; v < 3; ++v) {
    double m0 = hl * ((1.0 / 3.0) * (F[0][v] + F[2][v]) + (4.0 / 3.0) * F[1][v]);
    double m1 = hl * ((1.0 / 3.0) * (F[2][v] - F[0][v]));
    if (store_minus) {
      // e- frame moments (P0, P1) with P1 taken along e-'s own direction
      // (-s); stored so that e- reads (-M0, M1) = (P0, P1)
      m0 = -m0;
      m1 = -m1;
    }
    s.edge[v * ned + d] = m0;
    s.edge[(3 + v) * ned + d] = m1;
  }
  s.emode[d] = (unsigned char)mode;
}

// Volume + source integrals, fixed-order gather, inverse mass, RK update.
HD void element_body(int e, const DevMesh &m, const DevState &s, const Params &p, const double *w,
                     const double *wb, double dt) {
  const size_t ne = (size_t)m.ne, ned = (size_t)m.ned, nn = (size_t)m.nn;
  double u[9];
  for (int j = 0; j < 9; ++j) u[j] = w[j * ne + e];
  const bool wet = s.wet[e] != 0;
  const double g1x = m.gx1[e], g1y = m.gy1[e], g2x = m.gx2[e], g2y = m.gy2[e];
  const double A = m.area[e];
  const double h0v = m.hbv[e], h1v = m.hbv[ne + e], h2v = m.hbv[2 * ne + e];
  // Gradient of a linear nodal field with vertex values f0, f1, f2: its
  // modes 1, 2 are (f1 - f0)/2 and (2 (f2 - f0) - (f1 - f0))/6, built from
  // the vertex differences (exact for close values), so a large common
  // offset (1e5 Pa of air pressure, 3000 m of depth) cancels exactly.
  const double dh1 = h1v - h0v, dh2 = h2v - h0v;
  const double hm1 = 0.5 * dh1, hm2 = (2.0 * dh2 - dh1) * (1.0 / 6.0);
  const double dhx = hm1 * g1x + hm2 * g2x, dhy = hm1 * g1y + hm2 * g2y;
  const int n0 = m.el_node[e], n1 = m.el_node[ne + e], n2 = m.el_node[2 * ne + e];
  const double tx[3] = {s.nodal[n0], s.nodal[n1], s.nodal[n2]};
  const double ty[3] = {s.nodal[nn + n0], s.nodal[nn + n1], s.nodal[nn + n2]};
  const double pa[3] = {s.nodal[2 * nn + n0], s.nodal[2 * nn + n1], s.nodal[2 * nn + n2]};
  const double dp1 = pa[1] - pa[0], dp2 = pa[2] - pa[0];
  const double pm1 = 0.5 * dp1, pm2 = (2.0 * dp2 - dp1) * (1.0 / 6.0);
  const double dpx = pm1 * g1x + pm2 * g2x, dpy = pm1 * g1y + pm2 * g2y;
  const double nman = m.manning ? m.manning[e] : p.manning_n;
  const double gn2 = p.g * nman * nman;
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
    const double hb = L0[q] * h0v + L1[q] * h1v + L2[q] * h2v;
    const double H = ze + hb;
    const double ph = p_hydro(p.g, ze, hb);
    double uu = 0.0, vv = 0.0;
    if (wet) {
      const double iH = 1.0 / H;
      uu = qx * iH;
      vv = qy * iH;
    }
    sF[0][0] += qx;            sF[0][1] += qy;
    sF[1][0] += qx * uu + ph;  sF[1][1] += qx * vv;
    sF[2][0] += qy * uu;       sF[2][1] += qy * vv + ph;
    if (wet) {
      const double Hf = fmax(H, p.h0);
      const double qm = sqrt(qx * qx + qy * qy);
      const double fr = gn2 * qm / (Hf * Hf * cbrt(Hf));
      const double txq = L0[q] * tx[0] + L1[q] * tx[1] + L2[q] * tx[2];
      const double tyq = L0[q] * ty[0] + L1[q] * ty[1] + L2[q] * ty[2];
      const double sx = p.g * ze * dhx - fr * qx + txq * irho - H * irho * dpx;
      const double sy = p.g * ze * dhy - fr * qy + tyq * irho - H * irho * dpy;
      S0[1] += sx;          S0[2] += sy;
      S1[1] += C1[q] * sx;  S1[2] += C1[q] * sy;
      S2[1] += C2[q] * sx;  S2[2] += C2[q] * sy;
    }
  }
  // R_k / A (area part): (1/3) [grad phi_k . sum_q F + sum_q phi_k(q) S]
  double r[9];
  for (int v = 0; v < 3; ++v) {
    r[3 * v + 0] = S0[v] * (1.0 / 3.0);
    r[3 * v + 1] = (g1x * sF[v][0] + g1y * sF[v][1] + S1[v]) * (1.0 / 3.0);
    r[3 * v + 2] = (g2x * sF[v][0] + g2y * sF[v][1] + S2[v]) * (1.0 / 3.0);
  }
  // gather the three edges in fixed order
  double E[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int l = 0; l < 3; ++l) {
    const int code = m.el_edge[l * ne + e];
    const int d = code >> 1, side = code & 1;
    const int md = s.emode[d];
    if (md == 3 || md == 2 - side) continue;  // this side receives nothing
    const double sg = side ? -1.0 : 1.0;
    const double a1 = ga1(l), b1 = gb1(l), a2 = ga2(l), b2 = gb2(l);
    for (int v = 0; v < 3; ++v) {
      const double P0 = sg * s.edge[v * ned + d];
      const double P1 = s.edge[(3 + v) * ned + d];
      E[3 * v + 0] += P0;
      E[3 * v + 1] += a1 * P0 + b1 * P1;
      E[3 * v + 2] += a2 * P0 + b2 * P1;
    }
  }
  const double iA = 1.0 / A;
  const double imu[3] = {1.0, 6.0, 2.0};
  for (int j = 0; j < 9; ++j) {
    double dw = (r[j] - E[j] * iA) * imu[j % 3];
    if (!wet && j >= 3) dw = 0.0;
    double out;
    if (wb == nullptr) out = u[j] + dt * dw;
    else out = 0.5 * wb[j * ne + e] + 0.5 * (u[j] + dt * dw);
    s.wt[j * ne + e] = out;
  }
}

// Slope limiter (face-neighbour Barth-Jespersen) then wet/dry.  Returns the
// CFL candidate 2 r_e / lambda_e of the output (INFINITY if dry) and sets
// `bad` on a non-finite value.
HD double post_body(int e, const DevMesh &m, const DevState &s, const Params &p, double *wout,
                    bool &bad) {
  const size_t ne = (size_t)m.ne;
  double u[9];
  for (int j = 0; j < 9; ++j) u[j] = s.wt[j * ne + e];
  if (p.limiter) {
    const int f0 = m.el_nb[e], f1 = m.el_nb[ne + e], f2 = m.el_nb[2 * ne + e];
    for (int v = 0; v < 3; ++v) {
      const double mean = u[3 * v];
      const double *col = s.wt + (size_t)(3 * v) * ne;
      double hi = mean, lo = mean;
      if (f0 >= 0) { double t = col[f0]; hi = fmax(hi, t); lo = fmin(lo, t); }
      if (f1 >= 0) { double t = col[f1]; hi = fmax(hi, t); lo = fmin(lo, t); }
      if (f2 >= 0) { double t = col[f2]; hi = fmax(hi, t); lo = fmin(lo, t); }
      const double a = u[3 * v + 1], b = u[3 * v + 2];
      const double d0 = (mean - a - b) - mean, d1 = (mean + a - b) - mean, d2 = (mean + 2.0 * b) - mean;
      // the smallest ratio belongs to the largest excursion on each side
      const double dmax = fmax(d0, fmax(d1, d2)), dmin = fmin(d0, fmin(d1, d2));
      double alpha = 1.0;
      if (dmax > 0.0 && hi - mean < dmax) alpha = fmin(alpha, (hi - mean) / dmax);
      if (dmin < 0.0 && lo - mean > dmin) alpha = fmin(alpha, (lo - mean) / dmin);
      u[3 * v + 1] = a * alpha;
      u[3 * v + 2] = b * alpha;
    }
  }
  const double h0v = m.hbv[e], h1v = m.hbv[ne + e], h2v = m.hbv[2 * ne + e];
  const double hmean = (h0v + h1v + h2v) / 3.0;
  if (p.wetdry) {
    const double z0 = u[0] - u[1] - u[2], z1 = u[0] + u[1] - u[2], z2 = u[0] + 2.0 * u[2];
    double H[3] = {z0 + h0v, z1 + h1v, z2 + h2v};
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
      const double y0 = H[0] - h0v, y1 = H[1] - h1v, y2 = H[2] - h2v;
      u[1] = 0.5 * (y1 - y0);
      u[2] = 0.5 * (y2 - u[0]);
    }
  }
  bool fin = true;
  for (int j = 0; j < 9; ++j) {
    wout[j * ne + e] = u[j];
    fin = fin && __builtin_isfinite(u[j]);
  }
  bad = !fin;
  const double Hm = u[0] + hmean;
  const bool wet = p.wetdry ? (Hm > p.h0) : true;
  s.wet[e] = wet ? 1 : 0;
  if (!wet) return INFINITY;
  const double lam = sqrt(u[3] * u[3] + u[6] * u[6]) / Hm + sqrt(p.g * Hm);
  return m.inr2[e] / lam;
}

// wet flag + CFL candidate of a given state (used after set_state)
HD double init_body(int e, const DevMesh &m, const DevState &s, const Params &p) {
  const size_t ne = (size_t)m.ne;
  const double hmean = (m.hbv[e] + m.hbv[ne + e] + m.hbv[2 * ne + e]) / 3.0;
  const double Hm = s.w0[e] + hmean;
  const bool wet = p.wetdry ? (Hm > p.h0) : true;
  s.wet[e] = wet ? 1 : 0;
  if (!wet) return INFINITY;
  const double qx = s.w0[3 * ne + e], qy = s.w0[6 * ne + e];
  const double lam = sqrt(qx * qx + qy * qy) / Hm + sqrt(p.g * Hm);
  return m.inr2[e] / lam;
}

#undef HD

// ---------------------------------------------------------------- kernels
#ifdef __HIP_DEVICE_COMPILE__
#define DEVICE_ONLY 1
#endif

__device__ __forceinline__ double block_min(double v) {
  __shared__ double red[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kBlock / 64; ++i) v = fmin(v, red[i]);
  }
  return v;  // valid in thread 0
}

__global__ __launch_bounds__(kBlock) void k_forcing(DevMesh m, DevState s, Params p, int slot, int stage) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (s.ctrl->status) return;
  double dt;
  if (!step_dt(s.ctrl, p, slot, dt)) return;
  if (i >= m.nn) return;
  forcing_body(i, m, s, p, s.ctrl->t + (stage ? dt : 0.0));
}

__global__ __launch_bounds__(kBlock) void k_edge(DevMesh m, DevState s, Params p, const double *__restrict__ w,
                                                 int slot, int stage) {
  const int d = blockIdx.x * kBlock + threadIdx.x;
  Ctrl *c = s.ctrl;
  if (c->status) return;
  double dt;
  if (!step_dt(c, p, slot, dt)) {
    if (d == 0) atomicCAS(&c->status, 0, (int)DGSWE_E_ALLDRY);
    return;
  }
  if (d == 0 && stage == 0) c->dtmin[slot ^ 1] = double_to_bits(INFINITY);
  if (d >= m.ned) return;
  const double zb = p.n_tide > 0 || p.tide_offset != 0.0 ? tide_level(p, c->t + (stage ? dt : 0.0)) : 0.0;
  edge_body(d, m, s, p, w, zb);
}

__global__ __launch_bounds__(kBlock) void k_element(DevMesh m, DevState s, Params p, const double *__restrict__ w,
                                                    const double *__restrict__ wb, int slot) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (s.ctrl->status) return;
  double dt;
  if (!step_dt(s.ctrl, p, slot, dt)) return;
  if (e >= m.ne) return;
  element_body(e, m, s, p, w, wb, dt);
}

__global__ __launch_bounds__(kBlock) void k_post(DevMesh m, DevState s, Params p, double *__restrict__ wout,
                                                 int slot, int stage, int want_dt) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  Ctrl *c = s.ctrl;
  // no early return: every lane of the block reaches the barrier in block_min
  double dt = 0.0;
  const bool active = c->status == 0 && step_dt(c, p, slot, dt);
  double cand = INFINITY;
  bool bad = false;
  if (active && e < m.ne) cand = post_body(e, m, s, p, wout, bad);
  if (bad) atomicCAS(&c->status, 0, (int)DGSWE_E_NONFINITE);
  if (want_dt) {
    double bm = block_min(cand);
    if (threadIdx.x == 0 && bm < INFINITY) atomicMin(&c->dtmin[slot ^ 1], double_to_bits(bm));
  }
  if (active && stage == 1 && e == 0) {
    c->t = c->t + dt;
    c->dt_last = dt;
    c->steps = c->steps + 1;
  }
}

// post-processing of a state supplied by the caller (s.wt -> wout)
__global__ __launch_bounds__(kBlock) void k_post_only(DevMesh m, DevState s, Params p, double *__restrict__ wout) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= m.ne) return;
  bool bad = false;
  (void)post_body(e, m, s, p, wout, bad);
}

__global__ void k_ctrl_reset(Ctrl *c, double t) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->t = t;
    c->dt_last = 0.0;
    c->dtmin[0] = double_to_bits(INFINITY);
    c->dtmin[1] = double_to_bits(INFINITY);
    c->steps = 0;
    c->status = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_init(DevMesh m, DevState s, Params p, int slot) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  double cand = INFINITY;
  if (e < m.ne) cand = init_body(e, m, s, p);
  double bm = block_min(cand);
  if (threadIdx.x == 0 && bm < INFINITY) atomicMin(&s.ctrl->dtmin[slot], double_to_bits(bm));
}

// Diagnostics: per-block partial sums (mass, volume, wet count), then one
// block adds the partials in a fixed order: deterministic.
__global__ __launch_bounds__(kBlock) void k_diag1(DevMesh m, DevState s, Params p) {
  __shared__ double sm[3][kBlock];
  const int e = blockIdx.x * kBlock + threadIdx.x;
  const size_t ne = (size_t)m.ne;
  double a = 0.0, b = 0.0, c = 0.0;
  if (e < m.ne) {
    const double hmean = (m.hbv[e] + m.hbv[ne + e] + m.hbv[2 * ne + e]) / 3.0;
    const double z = s.w0[e];
    a = m.area[e] * z;
    b = m.area[e] * (z + hmean);
    c = (p.wetdry ? (z + hmean > p.h0) : true) ? 1.0 : 0.0;
  }
  sm[0][threadIdx.x] = a; sm[1][threadIdx.x] = b; sm[2][threadIdx.x] = c;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < 3; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + st];
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
    for (int k = 0; k < 3; ++k) acc[k] += s.partial[(size_t)k * nb + i];
  for (int k = 0; k < 3; ++k) sm[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < 3; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + st];
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

hipError_t launch_forcing(const DevMesh &m, const DevState &s, const Params &p, int slot, int stage,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_forcing, dim3(nblk(m.nn)), dim3(kBlock), 0, st, m, s, p, slot, stage);
  return hipGetLastError();
}

hipError_t launch_edge(const DevMesh &m, const DevState &s, const Params &p, const double *w, int slot,
                       int stage, hipStream_t st) {
  hipLaunchKernelGGL(k_edge, dim3(nblk(m.ned)), dim3(kBlock), 0, st, m, s, p, w, slot, stage);
  return hipGetLastError();
}

hipError_t launch_element(const DevMesh &m, const DevState &s, const Params &p, const double *w,
                          const double *wbase, int slot, int stage, hipStream_t st) {
  (void)stage;
  hipLaunchKernelGGL(k_element, dim3(nblk(m.ne)), dim3(kBlock), 0, st, m, s, p, w, wbase, slot);
  return hipGetLastError();
}

hipError_t launch_post(const DevMesh &m, const DevState &s, const Params &p, double *wout, int slot,
                       int stage, int want_dt, hipStream_t st) {
  hipLaunchKernelGGL(k_post, dim3(nblk(m.ne)), dim3(kBlock), 0, st, m, s, p, wout, slot, stage, want_dt);
  return hipGetLastError();
}

hipError_t launch_post_only(const DevMesh &m, const DevState &s, const Params &p, double *wout,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_post_only, dim3(nblk(m.ne)), dim3(kBlock), 0, st, m, s, p, wout);
  return hipGetLastError();
}

hipError_t launch_init_state(const DevMesh &m, const DevState &s, const Params &p, int slot, double t,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, st, s.ctrl, t);
  hipLaunchKernelGGL(k_init, dim3(nblk(m.ne)), dim3(kBlock), 0, st, m, s, p, slot);
  return hipGetLastError();
}

hipError_t launch_diag(const DevMesh &m, const DevState &s, const Params &p, double *out4, hipStream_t st) {
  const int nb = (int)nblk(m.ne);
  hipLaunchKernelGGL(k_diag1, dim3(nb), dim3(kBlock), 0, st, m, s, p);
  hipLaunchKernelGGL(k_diag2, dim3(1), dim3(kBlock), 0, st, s, nb, out4);
  return hipGetLastError();
}

}  // namespace dgswe
