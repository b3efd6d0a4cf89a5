/*
 * Plain FP64 CPU oracle of one explicit SSP Runge-Kutta discontinuous
 * Galerkin step for the 2-D depth-averaged shallow water equations.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP library; the two meet only through the seeded input generators.
 *
 * What it computes, and where the paper defines it (arXiv 2508.21208):
 *   - the PDE in (zeta, Hu_x, Hu_y) form ........ Sec. 2.1, Eq. (SWE)
 *   - conservative form w_t + div F(w) = s ....... Sec. 2.2, Eq. (cons_form)
 *   - element weak form ......................... Sec. 2.2, Eq. (elem_weak_form)
 *     (the volume term enters with a plus sign: integration by parts of
 *      (div F, v) gives -(grad v, F) on the left, i.e. +(grad v, F) on the
 *      right; the AREA algorithm also adds it)
 *   - Dubiner modal basis, p = 1 and p = 2 ...... Sec. 2.2, Eq. (dubiner)
 *     (the paper implements p = 1 and states that higher orders are
 *      supported; p = 2 follows the same definitions with the readings
 *      marked P2 below)
 *   - semi-discrete ODE and SSP Runge-Kutta ..... Sec. 2.2, Eq. (RKSSP)
 *   - AREA / EDGE / GATHER structure ............ Sec. 5.2, Algorithms 1-3:
 *     every edge flux is evaluated once and written into per-element,
 *     per-local-edge slots, then each element sums its three slots in a
 *     fixed order (no atomics, deterministic).
 *   - slope limiter, wet/dry, wind/pressure ..... Sec. 2.2 and Sec. 5.2
 *     ("Other kernels"); the paper names these steps but gives no formulas,
 *     so the readings below are used (each marked READING).
 *
 * Conventions (all READINGS where the paper is silent):
 *   state w[(m*3 + k)*ne + e]: variable m in {zeta, Qx, Qy}, mode k, element e.
 *   Reference triangle (-1,-1), (1,-1), (-1,1); local edge l lies opposite
 *   vertex l and runs from vertex (l+1)%3 to (l+2)%3.
 *   Interior edge: e+ = smaller element id, normal points from e+ to e-.
 *   Area rule: 3-point degree-2 rule, barycentric (2/3,1/6,1/6) and
 *   permutations, weight A/3.  Edge rule: 3-point Gauss-Lobatto
 *   s = -1, 0, 1 with weights 1/3, 4/3, 1/3 (times len/2).
 *   Flux: local Lax-Friedrichs.  Time stepping: SSP-RK(2,2) in Shu-Osher
 *   form with limiter + wet/dry after each stage.
 *
 * Built with -O2 -ffp-contract=off; OpenMP only splits independent loops
 * (no reductions other than an exact min), so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_INVALID 1
#define OR_E_MESH 2
#define OR_E_NOMEM 3
#define OR_E_NONFINITE 5
#define OR_E_ALLDRY 6

#define BC_LAND 1
#define BC_OCEAN 2

typedef void (*or_source_fn)(double t, int32_t npts, const double *xy, double *out, void *ctx);

typedef struct {
  double g, rho0, h0, cfl, dt_fixed, dt_max;
  int32_t limiter;  /* 0: off, 1: face-neighbour, 2: vertex-based (p = 1) */
  int32_t wetdry;
  int32_t rk;       /* 22, 33, 32, 42, 52: SSPRK(s, q) */
  int32_t flux;     /* 0: local Lax-Friedrichs, 1: Roe on edges wet on both sides */
} or_params;

typedef struct {
  /* Manning coefficient: scalar, or per element when `manning_elem` set */
  double manning_n;
  double *manning_elem;
  /* tidal elevation on ocean edges: offset + sum amp cos(omega t + phase) */
  int32_t n_tide;
  double tide_amp[16], tide_omega[16], tide_phase[16], tide_offset;
  /* static nodal wind stress [nn][2] (N/m^2) and pressure [nn] (Pa) */
  double *wind_tau, *patm;
  /* Holland (1980) parametric vortex moving at constant velocity */
  int32_t holland;
  double x0, y0, vx, vy, dp, pn, rmax, B, rho_air, coriolis_f, wind_factor;
  /* Coriolis parameter of the momentum equations (1/s) and a uniform
   * rainfall rate (m/s): the remaining sources of Sec. 2.1 */
  double coriolis, rain;
} or_forcing;

typedef struct or_mesh {
  int32_t nn, ne, ned;
  double *xy, *hb;
  int32_t *tri;
  /* edges */
  int32_t *ed_el;   /* [ned][2] e+, e- (-1 on a boundary) */
  int32_t *ed_loc;  /* [ned][2] local edge number on each side */
  int32_t *ed_type; /* 0 interior, BC_LAND, BC_OCEAN */
  double *ed_n;     /* [ned][2] unit normal, from e+ outward */
  double *ed_len;
  /* elements */
  int32_t *el_edge; /* [ne][3] */
  int32_t *el_nb;   /* [ne][3] neighbour across local edge, -1 if none */
  double *area, *inr2;
  double *gphi;     /* [ne][2 modes (1,2)][2] physical gradients of phi_1, phi_2 */
  double *glam;     /* [ne][3][2] gradients of the barycentric coordinates */
  double *qxy;      /* [ne][3 points][2] physical area quadrature points */
  or_params prm;
  or_forcing frc;
  double t, dt_last;
  int64_t steps;
  int32_t nm;       /* modes per variable: 3 (p = 1) or 6 (p = 2) */
  int32_t nq;       /* area quadrature points per element */
  double *jit;      /* p = 2: [ne][4] J^{-T} = [[a, b], [c, d]] (grad = J^{-T} grad_ref) */
  double *w, *w1, *wt, *dw, *slot, *nodal, *extra;
  or_source_fn src_fn;
  void *src_ctx;
} or_mesh;

/* ------------------------------------------------------------------ */
/* basis and quadrature (Sec. 2.2, Eq. dubiner)                         */
/* ------------------------------------------------------------------ */

/* Dubiner p = 1 on the reference triangle.  With a = 2(1+xi)/(1-eta) - 1,
 * b = eta: phi_00 = 1; phi_10 = P_1(a) (1-b)/2 = (1 + 2 xi + eta)/2;
 * phi_01 = P_1^{(1,0)}(b) = (1 + 3 eta)/2.  Order [phi_00, phi_10, phi_01]. */
void or_basis(double xi, double eta, double phi[3], double dphi[3][2]) {
  phi[0] = 1.0;
  phi[1] = 0.5 * (1.0 + 2.0 * xi + eta);
  phi[2] = 0.5 * (1.0 + 3.0 * eta);
  if (dphi) {
    dphi[0][0] = 0.0; dphi[0][1] = 0.0;
    dphi[1][0] = 1.0; dphi[1][1] = 0.5;
    dphi[2][0] = 0.0; dphi[2][1] = 1.5;
  }
}

/* reference coordinates of a point with barycentric coordinates lam */
static void ref_point(const double lam[3], double *xi, double *eta) {
  /* vertices (-1,-1), (1,-1), (-1,1) */
  *xi = -lam[0] + lam[1] - lam[2];
  *eta = -lam[0] - lam[1] + lam[2];
}

/* Area rule: 3 interior points, degree 2, weight A/3 each (READING: the paper
 * states only "Gauss-Lobatto quadrature"). */
static const double AREA_BARY[3][3] = {
    {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0},
    {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0},
    {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0}};
static const double AREA_WFRAC[3] = {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0};

/* Edge rule: 3-point Gauss-Lobatto on [-1,1], exact to degree 3. */
static const double EDGE_S[3] = {-1.0, 0.0, 1.0};
static const double EDGE_W[3] = {1.0 / 3.0, 4.0 / 3.0, 1.0 / 3.0};

void or_area_rule(double bary[9], double wfrac[3]) {
  for (int q = 0; q < 3; ++q) {
    for (int v = 0; v < 3; ++v) bary[q * 3 + v] = AREA_BARY[q][v];
    wfrac[q] = AREA_WFRAC[q];
  }
}

void or_edge_rule(double s[3], double w[3]) {
  for (int g = 0; g < 3; ++g) { s[g] = EDGE_S[g]; w[g] = EDGE_W[g]; }
}

/* basis values on local edge l at parameter s in [-1,1] */
static void edge_basis(int l, double s, double phi[3]) {
  static const double V[3][2] = {{-1.0, -1.0}, {1.0, -1.0}, {-1.0, 1.0}};
  int a = (l + 1) % 3, b = (l + 2) % 3;
  double xi = V[a][0] * 0.5 * (1.0 - s) + V[b][0] * 0.5 * (1.0 + s);
  double eta = V[a][1] * 0.5 * (1.0 - s) + V[b][1] * 0.5 * (1.0 + s);
  or_basis(xi, eta, phi, NULL);
}

static void area_basis(int q, double phi[3]) {
  double xi, eta;
  ref_point(AREA_BARY[q], &xi, &eta);
  or_basis(xi, eta, phi, NULL);
}

/* diagonal of the physical mass matrix divided by the area */
static const double MU[3] = {1.0, 1.0 / 6.0, 1.0 / 2.0};

/* ------------------------------------------------------------------ */
/* pointwise physics (Sec. 2.1 Eq. SWE, Sec. 2.2 Eq. cons_form)        */
/* ------------------------------------------------------------------ */

/* Hydrostatic part of the momentum flux, g/2 (H^2 - h_b^2), evaluated as
 * g/2 zeta (zeta + 2 h_b) (the same quantity without cancellation).  READING:
 * the flux matrix printed in Sec. 2.2 omits the 1/2 that Eq. (SWE) and the
 * AREA kernel's flux list carry; the 1/2 is used. */
static double p_hydro(double g, double ze, double hb) { return 0.5 * g * ze * (ze + 2.0 * hb); }

/* physical flux F(w) = [[Qx, Qy], [Qx u + p, Qx v], [Qy u, Qy v + p]] */
static void phys_flux(double g, double ze, double qx, double qy, double hb, int wet, double F[3][2]) {
  double H = ze + hb;
  double u = 0.0, v = 0.0;
  if (wet) { u = qx / H; v = qy / H; }
  double p = p_hydro(g, ze, hb);
  F[0][0] = qx; F[0][1] = qy;
  F[1][0] = qx * u + p; F[1][1] = qx * v;
  F[2][0] = qy * u; F[2][1] = qy * v + p;
}

/* Local Lax-Friedrichs flux (Sec. 2.2 names LLF or Roe; READING: LLF).
 * Left state L with normal n pointing from L to R. A dry side contributes
 * u = 0. */
void or_llf(double g, const double wl[3], const double wr[3], double hb, double nx, double ny,
            int wetl, int wetr, double out[3]) {
  double Fl[3][2], Fr[3][2];
  phys_flux(g, wl[0], wl[1], wl[2], hb, wetl, Fl);
  phys_flux(g, wr[0], wr[1], wr[2], hb, wetr, Fr);
  double Hl = wl[0] + hb, Hr = wr[0] + hb;
  double unl = 0.0, unr = 0.0;
  if (wetl) unl = (wl[1] * nx + wl[2] * ny) / Hl;
  if (wetr) unr = (wr[1] * nx + wr[2] * ny) / Hr;
  double cl = sqrt(g * fmax(Hl, 0.0)), cr = sqrt(g * fmax(Hr, 0.0));
  double lam = fmax(fabs(unl) + cl, fabs(unr) + cr);
  for (int m = 0; m < 3; ++m) {
    double fl = Fl[m][0] * nx + Fl[m][1] * ny;
    double fr = Fr[m][0] * nx + Fr[m][1] * ny;
    out[m] = 0.5 * (fl + fr) - 0.5 * lam * (wr[m] - wl[m]);
  }
}

/* Roe's flux (the paper names it beside LLF, Sec. 2.2) for two wet sides,
 * normal n from L to R, in the normal / tangential frame t = (-ny, nx):
 * Roe averages u = (sqrt(H_L) u_L + sqrt(H_R) u_R) / (sqrt(H_L) + sqrt(H_R))
 * (both components) and c = sqrt(g (H_L + H_R) / 2); waves u_n - c, u_n,
 * u_n + c with eigenvectors (1, u_n - c, u_t), (0, 0, 1), (1, u_n + c, u_t)
 * on (H, q_n, q_t) and strengths a1 = ((u_n + c) dH - dq_n) / (2c),
 * a2 = dq_t - u_t dH, a3 = (dq_n - (u_n - c) dH) / (2c), dH = zeta_R -
 * zeta_L (the bathymetry is shared);
 * F = (F_L + F_R).n / 2 - sum_k |lam_k| a_k r_k / 2.
 * READING: Harten-Hyman entropy fix on the two acoustic waves, |lam| ->
 * (lam^2 + d^2) / (2 d) when |lam| < d = max(0, lam - lam(L), lam(R) - lam);
 * a side with zero or negative depth at the point falls back to LLF. */
void or_roe(double g, const double wl[3], const double wr[3], double hb, double nx, double ny, double out[3]) {
  double Hl = wl[0] + hb, Hr = wr[0] + hb;
  if (!(Hl > 0.0 && Hr > 0.0)) {
    or_llf(g, wl, wr, hb, nx, ny, 1, 1, out);
    return;
  }
  double Fl[3][2], Fr[3][2];
  phys_flux(g, wl[0], wl[1], wl[2], hb, 1, Fl);
  phys_flux(g, wr[0], wr[1], wr[2], hb, 1, Fr);
  double unl = (wl[1] * nx + wl[2] * ny) / Hl, unr = (wr[1] * nx + wr[2] * ny) / Hr;
  double utl = (-wl[1] * ny + wl[2] * nx) / Hl, utr = (-wr[1] * ny + wr[2] * nx) / Hr;
  double sl = sqrt(Hl), sr = sqrt(Hr);
  double un = (sl * unl + sr * unr) / (sl + sr);
  double ut = (sl * utl + sr * utr) / (sl + sr);
  double c = sqrt(g * 0.5 * (Hl + Hr));
  double dH = wr[0] - wl[0];
  double dqn = (wr[1] - wl[1]) * nx + (wr[2] - wl[2]) * ny;
  double dqt = -(wr[1] - wl[1]) * ny + (wr[2] - wl[2]) * nx;
  double a1 = ((un + c) * dH - dqn) / (2.0 * c);
  double a2 = dqt - ut * dH;
  double a3 = (dqn - (un - c) * dH) / (2.0 * c);
  double l1 = un - c, l2 = un, l3 = un + c;
  double cl = sqrt(g * Hl), cr = sqrt(g * Hr);
  double d1 = fmax(0.0, fmax(l1 - (unl - cl), (unr - cr) - l1));
  double d3 = fmax(0.0, fmax(l3 - (unl + cl), (unr + cr) - l3));
  double m1 = fabs(l1), m2 = fabs(l2), m3 = fabs(l3);
  if (m1 < d1) m1 = (l1 * l1 + d1 * d1) / (2.0 * d1);
  if (m3 < d3) m3 = (l3 * l3 + d3 * d3) / (2.0 * d3);
  /* dissipation on (H, q_n, q_t), then back to (q_x, q_y) */
  double DH = m1 * a1 + m3 * a3;
  double Dn = m1 * a1 * (un - c) + m3 * a3 * (un + c);
  double Dt = m1 * a1 * ut + m2 * a2 + m3 * a3 * ut;
  double D[3] = {DH, Dn * nx - Dt * ny, Dn * ny + Dt * nx};
  for (int m = 0; m < 3; ++m) {
    double fl = Fl[m][0] * nx + Fl[m][1] * ny;
    double fr = Fr[m][0] * nx + Fr[m][1] * ny;
    out[m] = 0.5 * (fl + fr) - 0.5 * D[m];
  }
}

/* No-normal-flow (land) flux: LLF against the mirror state
 * (zeta, Q - 2 (Q.n) n), written out in closed form; the mass flux is 0. */
void or_wall(double g, const double w[3], double hb, double nx, double ny, int wet, double out[3]) {
  double H = w[0] + hb;
  double p = p_hydro(g, w[0], hb);
  double f = p;
  if (wet) {
    double qn = w[1] * nx + w[2] * ny;
    double lam = fabs(qn) / H + sqrt(g * fmax(H, 0.0));
    f = qn * qn / H + p + lam * qn;
  }
  out[0] = 0.0;
  out[1] = f * nx;
  out[2] = f * ny;
}

/* Holland (1980) vortex: pressure p = pc + dp exp(-(Rmax/r)^B), gradient wind
 * Vg = sqrt(B dp/rho_air (Rmax/r)^B exp(-(Rmax/r)^B) + (r f/2)^2) - r f/2,
 * surface wind = wind_factor * Vg, tangential (counter-clockwise for f > 0),
 * stress rho_air Cd |W| W with Cd = min(3.5e-3, (0.75 + 0.067|W|) 1e-3)
 * (Garratt).  READING: the paper lists wind stress and atmospheric pressure as
 * forcing terms (Sec. 2.1) and computes them per mesh node (Sec. 5.2) without
 * giving a model. */
void or_holland(const or_forcing *f, double x, double y, double t, double out[3]) {
  double cx = f->x0 + f->vx * t, cy = f->y0 + f->vy * t;
  double dx = x - cx, dy = y - cy;
  double r = sqrt(dx * dx + dy * dy);
  double pc = f->pn - f->dp;
  if (r <= 0.0) { out[0] = 0.0; out[1] = 0.0; out[2] = pc; return; }
  double a = pow(f->rmax / r, f->B);
  double e = exp(-a);
  double p = pc + f->dp * e;
  double rf2 = 0.5 * r * f->coriolis_f;
  double vg = sqrt(f->B * f->dp / f->rho_air * a * e + rf2 * rf2) - fabs(rf2);
  double ws = f->wind_factor * vg;
  double sgn = (f->coriolis_f < 0.0) ? -1.0 : 1.0;
  double wx = -sgn * ws * dy / r, wy = sgn * ws * dx / r;
  double cd = (0.75 + 0.067 * ws) * 1.0e-3;
  if (cd > 3.5e-3) cd = 3.5e-3;
  out[0] = f->rho_air * cd * ws * wx;
  out[1] = f->rho_air * cd * ws * wy;
  out[2] = p;
}

static double tide_level(const or_forcing *f, double t) {
  double z = f->tide_offset;
  for (int i = 0; i < f->n_tide; ++i) z += f->tide_amp[i] * cos(f->tide_omega[i] * t + f->tide_phase[i]);
  return z;
}

/* ------------------------------------------------------------------ */
/* mesh preprocessing                                                   */
/* ------------------------------------------------------------------ */
typedef struct { int64_t key; int32_t e, l; } edge_rec;

static int cmp_edge(const void *a, const void *b) {
  const edge_rec *x = (const edge_rec *)a, *y = (const edge_rec *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->e != y->e) return x->e < y->e ? -1 : 1;
  return 0;
}

typedef struct { int64_t key; int32_t type; } bnd_rec;
static int cmp_bnd(const void *a, const void *b) {
  const bnd_rec *x = (const bnd_rec *)a, *y = (const bnd_rec *)b;
  return x->key < y->key ? -1 : (x->key > y->key ? 1 : 0);
}

void or_destroy(or_mesh *M) {
  if (!M) return;
  free(M->xy); free(M->hb); free(M->tri);
  free(M->ed_el); free(M->ed_loc); free(M->ed_type); free(M->ed_n); free(M->ed_len);
  free(M->el_edge); free(M->el_nb); free(M->area); free(M->inr2); free(M->gphi); free(M->glam);
  free(M->qxy); free(M->jit);
  free(M->w); free(M->w1); free(M->wt); free(M->dw); free(M->slot); free(M->nodal); free(M->extra);
  free(M->frc.manning_elem); free(M->frc.wind_tau); free(M->frc.patm);
  free(M);
}

or_mesh *or_create(int32_t nn, const double *xy, const double *hb, int32_t ne, const int32_t *tri,
                   int32_t nb, const int32_t *bnd, const int32_t *btype, int32_t *status) {
  *status = OR_E_INVALID;
  if (nn <= 0 || ne <= 0 || nb < 0 || !xy || !hb || !tri || (nb > 0 && (!bnd || !btype))) return NULL;
  or_mesh *M = (or_mesh *)calloc(1, sizeof(or_mesh));
  if (!M) { *status = OR_E_NOMEM; return NULL; }
  M->nn = nn; M->ne = ne;
  M->xy = malloc(sizeof(double) * 2 * nn); M->hb = malloc(sizeof(double) * nn);
  M->tri = malloc(sizeof(int32_t) * 3 * ne);
  memcpy(M->xy, xy, sizeof(double) * 2 * nn); memcpy(M->hb, hb, sizeof(double) * nn);
  memcpy(M->tri, tri, sizeof(int32_t) * 3 * ne);
  *status = OR_E_MESH;
  for (int64_t i = 0; i < 3 * (int64_t)ne; ++i)
    if (tri[i] < 0 || tri[i] >= nn) { or_destroy(M); return NULL; }
  /* geometry */
  M->area = malloc(sizeof(double) * ne); M->inr2 = malloc(sizeof(double) * ne);
  M->gphi = malloc(sizeof(double) * 4 * ne); M->glam = malloc(sizeof(double) * 6 * ne);
  M->qxy = malloc(sizeof(double) * 6 * ne);
  for (int32_t e = 0; e < ne; ++e) {
    const int32_t *v = tri + 3 * e;
    double x1 = xy[2 * v[0]], y1 = xy[2 * v[0] + 1];
    double x2 = xy[2 * v[1]], y2 = xy[2 * v[1] + 1];
    double x3 = xy[2 * v[2]], y3 = xy[2 * v[2] + 1];
    double A = 0.5 * ((x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1));
    if (!(A > 0.0)) { or_destroy(M); return NULL; }
    M->area[e] = A;
    double l0 = hypot(x3 - x2, y3 - y2), l1 = hypot(x1 - x3, y1 - y3), l2 = hypot(x2 - x1, y2 - y1);
    M->inr2[e] = 2.0 * (2.0 * A / (l0 + l1 + l2));
    /* Jacobian of the map from the reference triangle: J = 1/2 [[x2-x1, x3-x1],[y2-y1, y3-y1]] */
    double J11 = 0.5 * (x2 - x1), J12 = 0.5 * (x3 - x1), J21 = 0.5 * (y2 - y1), J22 = 0.5 * (y3 - y1);
    double det = J11 * J22 - J12 * J21;
    /* grad phi = J^{-T} grad_ref phi;  J^{-T} = 1/det [[J22, -J21], [-J12, J11]] */
    double ref[3][2], phi[3];
    or_basis(0.0, 0.0, phi, ref);
    for (int k = 1; k < 3; ++k) {
      double gx = (J22 * ref[k][0] - J21 * ref[k][1]) / det;
      double gy = (-J12 * ref[k][0] + J11 * ref[k][1]) / det;
      M->gphi[4 * e + 2 * (k - 1)] = gx;
      M->gphi[4 * e + 2 * (k - 1) + 1] = gy;
    }
    /* barycentric gradients: grad lam_i = (y_j - y_k, x_k - x_j) / (2A) */
    double X[3] = {x1, x2, x3}, Y[3] = {y1, y2, y3};
    for (int i = 0; i < 3; ++i) {
      int j = (i + 1) % 3, k = (i + 2) % 3;
      M->glam[6 * e + 2 * i] = (Y[j] - Y[k]) / (2.0 * A);
      M->glam[6 * e + 2 * i + 1] = (X[k] - X[j]) / (2.0 * A);
    }
    for (int q = 0; q < 3; ++q) {
      M->qxy[6 * e + 2 * q] = AREA_BARY[q][0] * x1 + AREA_BARY[q][1] * x2 + AREA_BARY[q][2] * x3;
      M->qxy[6 * e + 2 * q + 1] = AREA_BARY[q][0] * y1 + AREA_BARY[q][1] * y2 + AREA_BARY[q][2] * y3;
    }
  }
  /* edges: sort (node pair, element) records */
  edge_rec *R = malloc(sizeof(edge_rec) * 3 * (size_t)ne);
  for (int32_t e = 0; e < ne; ++e)
    for (int l = 0; l < 3; ++l) {
      int32_t a = tri[3 * e + (l + 1) % 3], b = tri[3 * e + (l + 2) % 3];
      int64_t lo = a < b ? a : b, hi = a < b ? b : a;
      R[3 * e + l].key = lo * (int64_t)nn + hi; R[3 * e + l].e = e; R[3 * e + l].l = l;
    }
  qsort(R, 3 * (size_t)ne, sizeof(edge_rec), cmp_edge);
  bnd_rec *B = malloc(sizeof(bnd_rec) * (nb > 0 ? nb : 1));
  for (int32_t i = 0; i < nb; ++i) {
    int32_t a = bnd[2 * i], b = bnd[2 * i + 1];
    if (a < 0 || a >= nn || b < 0 || b >= nn || a == b || (btype[i] != BC_LAND && btype[i] != BC_OCEAN)) {
      free(R); free(B); *status = (btype[i] == 3) ? OR_E_INVALID : OR_E_MESH; or_destroy(M); return NULL;
    }
    int64_t lo = a < b ? a : b, hi = a < b ? b : a;
    B[i].key = lo * (int64_t)nn + hi; B[i].type = btype[i];
  }
  qsort(B, nb, sizeof(bnd_rec), cmp_bnd);
  for (int32_t i = 1; i < nb; ++i)
    if (B[i].key == B[i - 1].key) { free(R); free(B); or_destroy(M); return NULL; }
  int32_t ned = 0;
  for (int64_t i = 0; i < 3 * (int64_t)ne;) {
    int64_t j = i + 1;
    while (j < 3 * (int64_t)ne && R[j].key == R[i].key) ++j;
    if (j - i > 2) { free(R); free(B); or_destroy(M); return NULL; }
    ++ned; i = j;
  }
  M->ned = ned;
  M->ed_el = malloc(sizeof(int32_t) * 2 * ned); M->ed_loc = malloc(sizeof(int32_t) * 2 * ned);
  M->ed_type = malloc(sizeof(int32_t) * ned); M->ed_n = malloc(sizeof(double) * 2 * ned);
  M->ed_len = malloc(sizeof(double) * ned);
  M->el_edge = malloc(sizeof(int32_t) * 3 * ne); M->el_nb = malloc(sizeof(int32_t) * 3 * ne);
  int32_t d = 0, nbused = 0;
  for (int64_t i = 0; i < 3 * (int64_t)ne;) {
    int64_t j = i + 1;
    while (j < 3 * (int64_t)ne && R[j].key == R[i].key) ++j;
    int32_t ep = R[i].e, lp = R[i].l;  /* sorted by element: R[i] has the smaller id */
    M->ed_el[2 * d] = ep; M->ed_loc[2 * d] = lp;
    M->el_edge[3 * ep + lp] = d;
    if (j - i == 2) {
      int32_t em = R[i + 1].e, lm = R[i + 1].l;
      M->ed_el[2 * d + 1] = em; M->ed_loc[2 * d + 1] = lm; M->ed_type[d] = 0;
      M->el_edge[3 * em + lm] = d;
      M->el_nb[3 * ep + lp] = em; M->el_nb[3 * em + lm] = ep;
    } else {
      M->ed_el[2 * d + 1] = -1; M->ed_loc[2 * d + 1] = -1;
      M->el_nb[3 * ep + lp] = -1;
      bnd_rec key = {R[i].key, 0};
      bnd_rec *hit = nb > 0 ? bsearch(&key, B, nb, sizeof(bnd_rec), cmp_bnd) : NULL;
      if (!hit) { free(R); free(B); or_destroy(M); return NULL; }
      M->ed_type[d] = hit->type; ++nbused;
    }
    /* normal and length from the e+ side: A -> B counter-clockwise */
    int32_t na = tri[3 * ep + (lp + 1) % 3], nb2 = tri[3 * ep + (lp + 2) % 3];
    double dx = xy[2 * nb2] - xy[2 * na], dy = xy[2 * nb2 + 1] - xy[2 * na + 1];
    double len = hypot(dx, dy);
    M->ed_len[d] = len; M->ed_n[2 * d] = dy / len; M->ed_n[2 * d + 1] = -dx / len;
    ++d; i = j;
  }
  free(R); free(B);
  if (nbused != nb) { or_destroy(M); return NULL; } /* a listed boundary edge is not on the boundary */
  size_t s9 = sizeof(double) * 9 * (size_t)ne;
  M->w = calloc(1, s9); M->w1 = calloc(1, s9); M->wt = calloc(1, s9); M->dw = calloc(1, s9);
  M->slot = calloc(1, sizeof(double) * 27 * (size_t)ne);
  M->nodal = calloc(1, sizeof(double) * 3 * (size_t)nn);
  M->extra = NULL;
  if (!M->w || !M->w1 || !M->wt || !M->dw || !M->slot || !M->nodal) { or_destroy(M); *status = OR_E_NOMEM; return NULL; }
  M->nm = 3; M->nq = 3;
  M->prm.rk = 22;
  M->prm.flux = 0;
  M->prm.g = 9.81; M->prm.rho0 = 1000.0; M->prm.h0 = 0.01; M->prm.cfl = 0.2;
  M->prm.dt_fixed = 0.0; M->prm.dt_max = 0.0; M->prm.limiter = 1; M->prm.wetdry = 1;
  M->frc.pn = 101300.0;
  *status = OR_OK;
  return M;
}

/* ------------------------------------------------------------------ */
/* configuration                                                        */
/* ------------------------------------------------------------------ */
int32_t or_set_params(or_mesh *M, double g, double rho0, double h0, double cfl, double dt_fixed,
                      double dt_max, int32_t limiter, int32_t wetdry) {
  if (!(g > 0.0) || !(rho0 > 0.0) || !(h0 > 0.0) || (dt_fixed <= 0.0 && !(cfl > 0.0))) return OR_E_INVALID;
  if (limiter < 0 || limiter > 2) return OR_E_INVALID;
  M->prm.g = g; M->prm.rho0 = rho0; M->prm.h0 = h0; M->prm.cfl = cfl; M->prm.dt_fixed = dt_fixed;
  M->prm.dt_max = dt_max; M->prm.limiter = limiter; M->prm.wetdry = wetdry;
  return OR_OK;
}

int32_t or_set_forcing(or_mesh *M, double manning_n, const double *manning_elem, int32_t n_tide,
                       const double *amp, const double *omega, const double *phase, double offset,
                       const double *wind_tau, const double *patm, int32_t holland, const double *hp) {
  if (n_tide < 0 || n_tide > 16) return OR_E_INVALID;
  or_forcing *f = &M->frc;
  free(f->manning_elem); f->manning_elem = NULL;
  free(f->wind_tau); f->wind_tau = NULL;
  free(f->patm); f->patm = NULL;
  f->manning_n = manning_n;
  if (manning_elem) {
    f->manning_elem = malloc(sizeof(double) * M->ne);
    memcpy(f->manning_elem, manning_elem, sizeof(double) * M->ne);
  }
  f->n_tide = n_tide;
  for (int i = 0; i < n_tide; ++i) { f->tide_amp[i] = amp[i]; f->tide_omega[i] = omega[i]; f->tide_phase[i] = phase[i]; }
  f->tide_offset = offset;
  if (wind_tau) { f->wind_tau = malloc(sizeof(double) * 2 * M->nn); memcpy(f->wind_tau, wind_tau, sizeof(double) * 2 * M->nn); }
  if (patm) { f->patm = malloc(sizeof(double) * M->nn); memcpy(f->patm, patm, sizeof(double) * M->nn); }
  f->holland = holland;
  if (holland) {
    /* hp: x0, y0, vx, vy, dp, pn, rmax, B, rho_air, coriolis_f, wind_factor */
    f->x0 = hp[0]; f->y0 = hp[1]; f->vx = hp[2]; f->vy = hp[3]; f->dp = hp[4]; f->pn = hp[5];
    f->rmax = hp[6]; f->B = hp[7]; f->rho_air = hp[8]; f->coriolis_f = hp[9]; f->wind_factor = hp[10];
  }
  return OR_OK;
}

/* READING (Sec. 2.1 lists Coriolis and rain among the sources): Coriolis
 * S_Qx += f Qy, S_Qy -= f Qx in wet elements; rain S_zeta += R everywhere
 * (a dry element fills and wets). */
int32_t or_set_sources(or_mesh *M, double coriolis, double rain) {
  M->frc.coriolis = coriolis;
  M->frc.rain = rain;
  return OR_OK;
}

void or_set_extra_source(or_mesh *M, or_source_fn fn, void *ctx) {
  M->src_fn = fn; M->src_ctx = ctx;
  free(M->extra); M->extra = NULL;
  if (fn) M->extra = calloc(1, sizeof(double) * 3 * M->nq * (size_t)M->ne);
}

int32_t or_set_state(or_mesh *M, double t, const double *w) {
  memcpy(M->w, w, sizeof(double) * 3 * M->nm * (size_t)M->ne);
  M->t = t; M->steps = 0; M->dt_last = 0.0;
  return OR_OK;
}

void or_get_state(const or_mesh *M, double *w, double *t, double *dt_last, int64_t *steps) {
  if (w) memcpy(w, M->w, sizeof(double) * 3 * M->nm * (size_t)M->ne);
  if (t) *t = M->t;
  if (dt_last) *dt_last = M->dt_last;
  if (steps) *steps = M->steps;
}

void or_info(const or_mesh *M, int32_t out[4]) { out[0] = M->nn; out[1] = M->ne; out[2] = M->ned; out[3] = 0; }

void or_geometry(const or_mesh *M, double *area, double *inr2, int32_t *el_nb, int32_t *ed_el,
                 int32_t *ed_type, double *ed_len, double *ed_n, double *qxy) {
  if (area) memcpy(area, M->area, sizeof(double) * M->ne);
  if (inr2) memcpy(inr2, M->inr2, sizeof(double) * M->ne);
  if (el_nb) memcpy(el_nb, M->el_nb, sizeof(int32_t) * 3 * M->ne);
  if (ed_el) memcpy(ed_el, M->ed_el, sizeof(int32_t) * 2 * M->ned);
  if (ed_type) memcpy(ed_type, M->ed_type, sizeof(int32_t) * M->ned);
  if (ed_len) memcpy(ed_len, M->ed_len, sizeof(double) * M->ned);
  if (ed_n) memcpy(ed_n, M->ed_n, sizeof(double) * 2 * M->ned);
  if (qxy) memcpy(qxy, M->qxy, sizeof(double) * 2 * M->nq * M->ne);
}

/* ------------------------------------------------------------------ */
/* the step                                                             */
/* ------------------------------------------------------------------ */
#define W(w, m, k, e, ne) (w)[((size_t)((m) * 3 + (k))) * (ne) + (e)]

static double hb_mean(const or_mesh *M, int32_t e) {
  const int32_t *v = M->tri + 3 * e;
  return (M->hb[v[0]] + M->hb[v[1]] + M->hb[v[2]]) / 3.0;
}

/* wet/dry status of an element: wet when its mean depth exceeds H0 */
static int is_wet(const or_mesh *M, const double *w, int32_t e) {
  if (!M->prm.wetdry) return 1;
  return (W(w, 0, 0, e, M->ne) + hb_mean(M, e)) > M->prm.h0;
}

/* state at reference point with basis values phi */
static void eval_state(const double *w, int32_t e, int32_t ne, const double phi[3], double out[3]) {
  for (int m = 0; m < 3; ++m) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) s += W(w, m, k, e, ne) * phi[k];
    out[m] = s;
  }
}

/* WIND (Sec. 5.2, "Other kernels"): nodal wind stress and pressure at time t */
static void forcing_at_nodes(or_mesh *M, double t) {
  const or_forcing *f = &M->frc;
  int32_t nn = M->nn;
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < nn; ++i) {
    double out[3] = {0.0, 0.0, 0.0};
    if (f->holland) {
      or_holland(f, M->xy[2 * i], M->xy[2 * i + 1], t, out);
    } else {
      if (f->wind_tau) { out[0] = f->wind_tau[2 * i]; out[1] = f->wind_tau[2 * i + 1]; }
      if (f->patm) out[2] = f->patm[i];
    }
    M->nodal[3 * i] = out[0]; M->nodal[3 * i + 1] = out[1]; M->nodal[3 * i + 2] = out[2];
  }
}

/* EDGE (Alg. 2) plus boundary edges: evaluate the numerical flux once per
 * edge at the three Gauss-Lobatto points and write the weighted projections
 * onto each side's basis into that side's slot [e][l][k][m].
 *
 * Wet/dry edge rules (READING; the paper omits its wet/dry branching):
 *   both sides dry        -> no flux;
 *   one side dry          -> LLF with u = 0 on the dry side; if the
 *                            integrated mass flux runs from the wet side into
 *                            the dry side it is used for both sides,
 *                            otherwise the wet side sees a wall and the dry
 *                            side gets nothing.
 * Ocean edges use the ghost state (zeta_b(t), Q+), wet iff zeta_b plus the
 * edge's mean bathymetry exceeds H0; land edges use the wall flux. */
static void edge_integrals(or_mesh *M, const double *w, double t) {
  const double g = M->prm.g, h0 = M->prm.h0;
  const int32_t ne = M->ne, ned = M->ned;
  const double zb = tide_level(&M->frc, t);
#pragma omp parallel for schedule(static)
  for (int32_t d = 0; d < ned; ++d) {
    int32_t ep = M->ed_el[2 * d], em = M->ed_el[2 * d + 1];
    int lp = M->ed_loc[2 * d], lm = M->ed_loc[2 * d + 1];
    int type = M->ed_type[d];
    double nx = M->ed_n[2 * d], ny = M->ed_n[2 * d + 1], len = M->ed_len[d];
    int32_t na = M->tri[3 * ep + (lp + 1) % 3], nb = M->tri[3 * ep + (lp + 2) % 3];
    double Fp[3][3], Fm[3][3], php[3][3], phm[3][3], wp[3][3], wm[3][3], hbq[3];
    int wetp = is_wet(M, w, ep), wetm = 0;
    for (int gq = 0; gq < 3; ++gq) {
      double s = EDGE_S[gq];
      edge_basis(lp, s, php[gq]);
      eval_state(w, ep, ne, php[gq], wp[gq]);
      hbq[gq] = M->hb[na] * 0.5 * (1.0 - s) + M->hb[nb] * 0.5 * (1.0 + s);
      if (type == 0) {
        edge_basis(lm, -s, phm[gq]); /* the e- side runs the edge backwards */
        eval_state(w, em, ne, phm[gq], wm[gq]);
      } else {
        wm[gq][0] = zb; wm[gq][1] = wp[gq][1]; wm[gq][2] = wp[gq][2];
      }
    }
    if (type == 0) wetm = is_wet(M, w, em);
    else if (type == BC_OCEAN) wetm = M->prm.wetdry ? (zb + 0.5 * (M->hb[na] + M->hb[nb]) > h0) : 1;
    if (type == BC_LAND) {
      for (int gq = 0; gq < 3; ++gq) {
        or_wall(g, wp[gq], hbq[gq], nx, ny, wetp, Fp[gq]);
        for (int m = 0; m < 3; ++m) Fm[gq][m] = 0.0;
      }
    } else if (!wetp && !wetm) {
      for (int gq = 0; gq < 3; ++gq)
        for (int m = 0; m < 3; ++m) { Fp[gq][m] = 0.0; Fm[gq][m] = 0.0; }
    } else {
      double F[3][3];
      for (int gq = 0; gq < 3; ++gq) {
        if (M->prm.flux == 1 && wetp && wetm) or_roe(g, wp[gq], wm[gq], hbq[gq], nx, ny, F[gq]);
        else or_llf(g, wp[gq], wm[gq], hbq[gq], nx, ny, wetp, wetm, F[gq]);
      }
      int flood = 1;
      if (!(wetp && wetm)) {
        double mflux = 0.0;
        for (int gq = 0; gq < 3; ++gq) mflux += EDGE_W[gq] * F[gq][0];
        flood = wetp ? (mflux > 0.0) : (mflux < 0.0);
      }
      if (flood) {
        for (int gq = 0; gq < 3; ++gq)
          for (int m = 0; m < 3; ++m) { Fp[gq][m] = F[gq][m]; Fm[gq][m] = -F[gq][m]; }
      } else if (wetp) {
        for (int gq = 0; gq < 3; ++gq) {
          or_wall(g, wp[gq], hbq[gq], nx, ny, 1, Fp[gq]);
          for (int m = 0; m < 3; ++m) Fm[gq][m] = 0.0;
        }
      } else {
        for (int gq = 0; gq < 3; ++gq) {
          or_wall(g, wm[gq], hbq[gq], -nx, -ny, 1, Fm[gq]);
          for (int m = 0; m < 3; ++m) Fp[gq][m] = 0.0;
        }
      }
    }
    /* slot[e][l][k][m] = sum_g (len/2) w_g phi_k(x_g) F_m(x_g) */
    double *sp = M->slot + 27 * (size_t)ep + 9 * lp;
    for (int k = 0; k < 3; ++k)
      for (int m = 0; m < 3; ++m) {
        double s = 0.0;
        for (int gq = 0; gq < 3; ++gq) s += 0.5 * len * EDGE_W[gq] * php[gq][k] * Fp[gq][m];
        sp[3 * k + m] = s;
      }
    if (type == 0) {
      double *sm = M->slot + 27 * (size_t)em + 9 * lm;
      for (int k = 0; k < 3; ++k)
        for (int m = 0; m < 3; ++m) {
          double s = 0.0;
          for (int gq = 0; gq < 3; ++gq) s += 0.5 * len * EDGE_W[gq] * phm[gq][k] * Fm[gq][m];
          sm[3 * k + m] = s;
        }
    }
  }
}

/* AREA (Alg. 1) + GATHER (Alg. 3) + inverse of the diagonal mass matrix:
 *   R_k = sum_q (A/3) grad phi_k . F(w_q) + sum_q (A/3) phi_k(q) s(w_q)
 *         - sum_l slot[e][l][k]
 *   dw_k/dt = R_k / (A mu_k),   mu = (1, 1/6, 1/2)
 * Sources (Eq. SWE, READING for the unspecified laws):
 *   s_zeta = R = 0 (no rain),
 *   s_Q = g zeta grad h_b - g n^2 |Q| Q / max(H,H0)^{7/3}   (Manning)
 *         + tau_s / rho0 - (H / rho0) grad p_a,
 * with tau_s and p_a the linear interpolants of the nodal values.  In a dry
 * element the momentum right-hand side is zero. */
static void element_rhs(or_mesh *M, const double *w, double t, double *dw) {
  const double g = M->prm.g, h0 = M->prm.h0, rho0 = M->prm.rho0;
  const int32_t ne = M->ne;
  if (M->src_fn) M->src_fn(t, 3 * ne, M->qxy, M->extra, M->src_ctx);
#pragma omp parallel for schedule(static)
  for (int32_t e = 0; e < ne; ++e) {
    const int32_t *v = M->tri + 3 * e;
    double A = M->area[e];
    double gp[3][2] = {{0.0, 0.0}, {M->gphi[4 * e], M->gphi[4 * e + 1]}, {M->gphi[4 * e + 2], M->gphi[4 * e + 3]}};
    const double *gl = M->glam + 6 * e;
    double hbv[3], tx[3], ty[3], pa[3];
    for (int i = 0; i < 3; ++i) {
      hbv[i] = M->hb[v[i]];
      tx[i] = M->nodal[3 * v[i]]; ty[i] = M->nodal[3 * v[i] + 1]; pa[i] = M->nodal[3 * v[i] + 2];
    }
    /* gradient of a linear nodal field f: sum_v f_v grad lam_v, written as
     * sum_{v=1,2} (f_v - f_0) grad lam_v (the barycentric gradients sum to
     * zero), so an ambient offset such as 1e5 Pa of air pressure cancels
     * exactly instead of swamping the gradient */
    double dhx = 0.0, dhy = 0.0, dpx = 0.0, dpy = 0.0;
    for (int i = 1; i < 3; ++i) {
      dhx += (hbv[i] - hbv[0]) * gl[2 * i]; dhy += (hbv[i] - hbv[0]) * gl[2 * i + 1];
      dpx += (pa[i] - pa[0]) * gl[2 * i]; dpy += (pa[i] - pa[0]) * gl[2 * i + 1];
    }
    double n = M->frc.manning_elem ? M->frc.manning_elem[e] : M->frc.manning_n;
    int wet = is_wet(M, w, e);
    double R[3][3] = {{0.0}};
    double wq[3][3], hq[3], phq[3][3];
    for (int q = 0; q < 3; ++q) {
      area_basis(q, phq[q]);
      eval_state(w, e, ne, phq[q], wq[q]);
      hq[q] = AREA_BARY[q][0] * hbv[0] + AREA_BARY[q][1] * hbv[1] + AREA_BARY[q][2] * hbv[2];
    }
    /* volume term */
    for (int q = 0; q < 3; ++q) {
      double F[3][2];
      phys_flux(g, wq[q][0], wq[q][1], wq[q][2], hq[q], wet, F);
      double wA = AREA_WFRAC[q] * A;
      for (int m = 0; m < 3; ++m)
        for (int k = 1; k < 3; ++k) R[m][k] += wA * (gp[k][0] * F[m][0] + gp[k][1] * F[m][1]);
    }
    /* source term */
    for (int q = 0; q < 3; ++q) {
      double ze = wq[q][0], qx = wq[q][1], qy = wq[q][2];
      double H = ze + hq[q];
      double S[3] = {0.0, 0.0, 0.0};
      if (wet) {
        double Hf = fmax(H, h0);
        double qm = sqrt(qx * qx + qy * qy);
        double fr = g * n * n * qm / pow(Hf, 7.0 / 3.0);
        double txq = AREA_BARY[q][0] * tx[0] + AREA_BARY[q][1] * tx[1] + AREA_BARY[q][2] * tx[2];
        double tyq = AREA_BARY[q][0] * ty[0] + AREA_BARY[q][1] * ty[1] + AREA_BARY[q][2] * ty[2];
        S[1] = g * ze * dhx - fr * qx + txq / rho0 - H / rho0 * dpx + M->frc.coriolis * qy;
        S[2] = g * ze * dhy - fr * qy + tyq / rho0 - H / rho0 * dpy - M->frc.coriolis * qx;
      }
      S[0] += M->frc.rain;
      if (M->extra)
        for (int m = 0; m < 3; ++m) S[m] += M->extra[(size_t)m * 3 * ne + 3 * (size_t)e + q];
      double wA = AREA_WFRAC[q] * A;
      for (int m = 0; m < 3; ++m)
        for (int k = 0; k < 3; ++k) R[m][k] += wA * phq[q][k] * S[m];
    }
    /* gather: fixed order l = 0, 1, 2 */
    const double *sl = M->slot + 27 * (size_t)e;
    for (int l = 0; l < 3; ++l)
      for (int k = 0; k < 3; ++k)
        for (int m = 0; m < 3; ++m) R[m][k] -= sl[9 * l + 3 * k + m];
    if (!wet)
      for (int k = 0; k < 3; ++k) { R[1][k] = 0.0; R[2][k] = 0.0; }
    for (int m = 0; m < 3; ++m)
      for (int k = 0; k < 3; ++k) W(dw, m, k, e, ne) = R[m][k] / (A * MU[k]);
  }
}

static void edge_integrals2(or_mesh *M, const double *w, double t);
static void element_rhs2(or_mesh *M, const double *w, double t, double *dw);
static int32_t postprocess2(or_mesh *M, const double *wt, double *out);

/* L_h(w) of Eq. (RKSSP) at time t */
int32_t or_rhs(or_mesh *M, const double *w, double t, double *dw) {
  forcing_at_nodes(M, t);
  if (M->nm == 6) {
    edge_integrals2(M, w, t);
    element_rhs2(M, w, t, dw);
  } else {
    edge_integrals(M, w, t);
    element_rhs(M, w, t, dw);
  }
  return OR_OK;
}

/* vertex values of a p=1 field: v1 = u0-u1-u2, v2 = u0+u1-u2, v3 = u0+2u2 */
static void to_vertices(double u0, double u1, double u2, double v[3]) {
  v[0] = u0 - u1 - u2; v[1] = u0 + u1 - u2; v[2] = u0 + 2.0 * u2;
}

/* Post-processing after each stage: slope limiter, then wet/dry (READINGS;
 * Sec. 2.2 names an optional slope limiter, Sec. 5.2 the SLOPELIM and
 * WETDRY kernels, neither with formulas).  Both leave the zeta mean (mode 0)
 * untouched.
 *
 * Limiter (face-neighbour Barth-Jespersen on zeta, Qx, Qy): with u0 the
 * element mean and [m, M] the range of the means over the element and its
 * face neighbours, alpha = min over vertices of
 *   min(1, (M - u0)/(u_v - u0)) if u_v > u0,  min(1, (m - u0)/(u_v - u0)) if u_v < u0,
 * and modes 1, 2 are scaled by alpha.
 *
 * Wet/dry with threshold H0 (vertex depths H_v = zeta_v + h_b,v, mean depth
 * Hm = zeta_0 + mean(h_b,v)):
 *   Hm <= H0       -> dry: flat depth H_v = Hm, all momentum set to 0;
 *   min H_v < H0   -> vertices below H0 raised to H0, the added volume taken
 *                     from the other vertices in proportion to H_v - H0
 *                     (flat at Hm if rounding leaves nothing to take from);
 *   otherwise      -> unchanged. */
int32_t or_postprocess(or_mesh *M, const double *wt, double *out) {
  if (M->nm == 6) return postprocess2(M, wt, out);
  const int32_t ne = M->ne;
  const double h0 = M->prm.h0;
  /* vertex-based limiter (READING of the optional limiter, after Kuzmin's
   * vertex-based limiter): the bounds at a mesh node are the smallest and
   * largest unlimited mean of the elements that have the node as a vertex;
   * each element then takes the largest alpha in [0, 1] that keeps all three
   * of its vertex values, mean + alpha (u_v - mean), inside the bounds of
   * the node at that vertex. */
  double *nlo = NULL, *nhi = NULL;
  if (M->prm.limiter == 2) {
    const int32_t nn = M->nn;
    nlo = malloc(sizeof(double) * 3 * (size_t)nn);
    nhi = malloc(sizeof(double) * 3 * (size_t)nn);
    if (!nlo || !nhi) { free(nlo); free(nhi); return OR_E_NOMEM; }
    for (size_t i = 0; i < 3 * (size_t)nn; ++i) { nlo[i] = INFINITY; nhi[i] = -INFINITY; }
    for (int32_t e = 0; e < ne; ++e)
      for (int i = 0; i < 3; ++i) {
        const int32_t n = M->tri[3 * e + i];
        for (int m = 0; m < 3; ++m) {
          const double mean = W(wt, m, 0, e, ne);
          if (mean < nlo[3 * n + m]) nlo[3 * n + m] = mean;
          if (mean > nhi[3 * n + m]) nhi[3 * n + m] = mean;
        }
      }
  }
#pragma omp parallel for schedule(static)
  for (int32_t e = 0; e < ne; ++e) {
    double u[3][3];
    for (int m = 0; m < 3; ++m)
      for (int k = 0; k < 3; ++k) u[m][k] = W(wt, m, k, e, ne);
    if (M->prm.limiter == 2) {
      for (int m = 0; m < 3; ++m) {
        const double mean = u[m][0];
        double vv[3];
        to_vertices(u[m][0], u[m][1], u[m][2], vv);
        double alpha = 1.0;
        for (int i = 0; i < 3; ++i) {
          const int32_t n = M->tri[3 * e + i];
          double a = 1.0;
          if (vv[i] > mean) a = fmin(1.0, (nhi[3 * n + m] - mean) / (vv[i] - mean));
          else if (vv[i] < mean) a = fmin(1.0, (nlo[3 * n + m] - mean) / (vv[i] - mean));
          if (a < alpha) alpha = a;
        }
        u[m][1] *= alpha; u[m][2] *= alpha;
      }
    } else if (M->prm.limiter) {
      for (int m = 0; m < 3; ++m) {
        double mean = u[m][0], hi = mean, lo = mean;
        for (int l = 0; l < 3; ++l) {
          int32_t f = M->el_nb[3 * e + l];
          if (f < 0) continue;
          double nbm = W(wt, m, 0, f, ne);
          if (nbm > hi) hi = nbm;
          if (nbm < lo) lo = nbm;
        }
        double vv[3];
        to_vertices(u[m][0], u[m][1], u[m][2], vv);
        double alpha = 1.0;
        for (int i = 0; i < 3; ++i) {
          double a = 1.0;
          if (vv[i] > mean) a = fmin(1.0, (hi - mean) / (vv[i] - mean));
          else if (vv[i] < mean) a = fmin(1.0, (lo - mean) / (vv[i] - mean));
          if (a < alpha) alpha = a;
        }
        u[m][1] *= alpha; u[m][2] *= alpha;
      }
    }
    if (M->prm.wetdry) {
      const int32_t *vt = M->tri + 3 * e;
      double hbv[3] = {M->hb[vt[0]], M->hb[vt[1]], M->hb[vt[2]]};
      double zv[3], Hv[3];
      to_vertices(u[0][0], u[0][1], u[0][2], zv);
      for (int i = 0; i < 3; ++i) Hv[i] = zv[i] + hbv[i];
      double Hm = u[0][0] + hb_mean(M, e);
      int changed = 0;
      if (Hm <= h0) {
        for (int i = 0; i < 3; ++i) Hv[i] = Hm;
        for (int k = 0; k < 3; ++k) { u[1][k] = 0.0; u[2][k] = 0.0; }
        changed = 1;
      } else {
        double hmin = fmin(Hv[0], fmin(Hv[1], Hv[2]));
        if (hmin < h0) {
          double D = 0.0, S = 0.0;
          for (int i = 0; i < 3; ++i) {
            if (Hv[i] < h0) D += h0 - Hv[i];
            else S += Hv[i] - h0;
          }
          if (S > D) {
            for (int i = 0; i < 3; ++i) {
              if (Hv[i] < h0) Hv[i] = h0;
              else Hv[i] = Hv[i] - D * (Hv[i] - h0) / S;
            }
          } else {
            /* S - D = 3 (Hm - H0) > 0 in exact arithmetic; when rounding
             * makes it vanish the element is made flat at its mean depth */
            for (int i = 0; i < 3; ++i) Hv[i] = Hm;
          }
          changed = 1;
        }
      }
      if (changed) {
        for (int i = 0; i < 3; ++i) zv[i] = Hv[i] - hbv[i];
        /* rebuild modes 1, 2 from vertex values; mode 0 is kept */
        u[0][1] = 0.5 * (zv[1] - zv[0]);
        u[0][2] = 0.5 * (zv[2] - u[0][0]);
      }
    }
    for (int m = 0; m < 3; ++m)
      for (int k = 0; k < 3; ++k) W(out, m, k, e, ne) = u[m][k];
  }
  free(nlo);
  free(nhi);
  return OR_OK;
}

/* CFL step size: dt = cfl * min over wet elements of 2 r_e / (|Q_mean|/H_mean
 * + sqrt(g H_mean)) (READING: the paper runs a fixed dt); `dt_fixed` > 0
 * overrides it, `dt_max` > 0 caps it.  Returns the raw minimum. */
double or_dt_raw(const or_mesh *M, const double *w) {
  const int32_t ne = M->ne;
  const double g = M->prm.g;
  double mn = INFINITY;
#pragma omp parallel for reduction(min : mn) schedule(static)
  for (int32_t e = 0; e < ne; ++e) {
    if (!is_wet(M, w, e)) continue;
    double H = w[e] + hb_mean(M, e);
    double qx = w[(size_t)M->nm * ne + e], qy = w[2 * (size_t)M->nm * ne + e];
    double lam = sqrt(qx * qx + qy * qy) / H + sqrt(g * H);
    double c = M->inr2[e] / lam;
    if (c < mn) mn = c;
  }
  return mn;
}

static int32_t pick_dt(const or_mesh *M, const double *w, double *dt) {
  if (M->prm.dt_fixed > 0.0) { *dt = M->prm.dt_fixed; return OR_OK; }
  double raw = or_dt_raw(M, w);
  if (isinf(raw)) {
    if (M->prm.dt_max > 0.0) { *dt = M->prm.dt_max; return OR_OK; }
    return OR_E_ALLDRY;
  }
  if (!isfinite(raw)) return OR_E_NONFINITE;
  double d = M->prm.cfl * raw;
  if (M->prm.dt_max > 0.0 && d > M->prm.dt_max) d = M->prm.dt_max;
  *dt = d;
  return OR_OK;
}

/* SSP-RK(2,2) in Shu-Osher form (Sec. 2.2, Eq. RKSSP; READING for the
 * paper's optimized scheme whose coefficients are not given):
 *   w1      = PP(w^n + dt L(w^n, t^n))
 *   w^{n+1} = PP(1/2 w^n + 1/2 (w1 + dt L(w1, t^n + dt))) */
/* The time steppers in Shu-Osher form (Eq. RKSSP; the paper names
 * optimized SSP schemes without coefficients, reading Z7):
 *   SSPRK(2,2): w1 = w + dt L(w), w+ = 1/2 w + 1/2 (w1 + dt L(w1));
 *   SSPRK(3,3): w1 = w + dt L(w), w2 = 3/4 w + 1/4 (w1 + dt L(w1)),
 *               w+ = 1/3 w + 2/3 (w2 + dt L(w2)), stage times t, t+dt, t+dt/2;
 *   SSPRK(s,2): w_k = w_{k-1} + dt/(s-1) L(w_{k-1}) for k < s,
 *               w+ = 1/s w + (s-1)/s (w_{s-1} + dt/(s-1) L(w_{s-1})),
 *               stage k at t + k dt/(s-1).
 * Each stage is post-processed. */
/* interior numerical flux: 0 LLF (default), 1 Roe where both sides are wet
 * (an edge with a dry side keeps the LLF wet/dry rules) */
int32_t or_set_flux(or_mesh *M, int32_t flux) {
  if (flux != 0 && flux != 1) return OR_E_INVALID;
  M->prm.flux = flux;
  return OR_OK;
}

int32_t or_set_scheme(or_mesh *M, int32_t rk) {
  if (rk != 22 && rk != 33 && rk != 32 && rk != 42 && rk != 52) return OR_E_INVALID;
  M->prm.rk = rk;
  return OR_OK;
}

/* stage k of scheme rk: out = a w + b (in + h dt L(in)) at time t + c dt */
static int scheme_stage(int32_t rk, int k, double *a, double *b, double *h, double *c) {
  if (rk == 33) {
    static const double A[3] = {0.0, 0.75, 1.0 / 3.0}, B[3] = {1.0, 0.25, 2.0 / 3.0}, Cc[3] = {0.0, 1.0, 0.5};
    *a = A[k]; *b = B[k]; *h = 1.0; *c = Cc[k];
    return 3;
  }
  int s = rk / 10;  /* 22 -> 2 */
  *h = 1.0 / (s - 1);
  *c = k * (*h);
  if (k == s - 1) { *a = 1.0 / s; *b = (double)(s - 1) / s; *c = 1.0; }
  else { *a = 0.0; *b = 1.0; }
  return s;
}

int32_t or_step(or_mesh *M, int32_t nsteps) {
  const int32_t ne = M->ne;
  const size_t n9 = 3 * (size_t)M->nm * ne;
  if (M->nm == 6 && M->prm.limiter == 2) return OR_E_INVALID;
  for (int32_t s = 0; s < nsteps; ++s) {
    double dt;
    int32_t st = pick_dt(M, M->w, &dt);
    if (st != OR_OK) return st;
    double a, b, h, c;
    const int ns = scheme_stage(M->prm.rk, 0, &a, &b, &h, &c);
    for (int k = 0; k < ns; ++k) {
      scheme_stage(M->prm.rk, k, &a, &b, &h, &c);
      const double *in = k == 0 ? M->w : M->w1;
      const double hdt = h * dt;
      or_rhs(M, in, M->t + c * dt, M->dw);
      if (a == 0.0) {
#pragma omp parallel for schedule(static)
        for (size_t i = 0; i < n9; ++i) M->wt[i] = in[i] + hdt * M->dw[i];
      } else {
#pragma omp parallel for schedule(static)
        for (size_t i = 0; i < n9; ++i) M->wt[i] = a * M->w[i] + b * (in[i] + hdt * M->dw[i]);
      }
      /* the last stage's result becomes w; earlier ones go to w1 */
      or_postprocess(M, M->wt, k == ns - 1 ? M->w : M->w1);
    }
    M->t += dt;
    M->dt_last = dt;
    M->steps += 1;
    for (size_t i = 0; i < n9; i += 1)
      if (!isfinite(M->w[i])) return OR_E_NONFINITE;
  }
  return OR_OK;
}

/* Diagnostics: mass M = sum A zeta_0, volume V = sum A Hmean, wet/dry counts
 * (sequential sum in element order). */
void or_diagnostics(const or_mesh *M, const double *w, double out[4]) {
  const int32_t ne = M->ne;
  double mass = 0.0, vol = 0.0;
  int64_t nwet = 0;
  for (int32_t e = 0; e < ne; ++e) {
    mass += M->area[e] * w[e];
    vol += M->area[e] * (w[e] + hb_mean(M, e));
    nwet += is_wet(M, w, e);
  }
  out[0] = mass; out[1] = vol; out[2] = (double)nwet; out[3] = (double)(ne - nwet);
}

double or_time(const or_mesh *M) { return M->t; }

/* Holland vortex at one point, parameters as in or_set_forcing's `hp` */
void or_holland_at(const double hp[11], double x, double y, double t, double out[3]) {
  or_forcing f;
  memset(&f, 0, sizeof f);
  f.x0 = hp[0]; f.y0 = hp[1]; f.vx = hp[2]; f.vy = hp[3]; f.dp = hp[4]; f.pn = hp[5];
  f.rmax = hp[6]; f.B = hp[7]; f.rho_air = hp[8]; f.coriolis_f = hp[9]; f.wind_factor = hp[10];
  or_holland(&f, x, y, t, out);
}

/* ------------------------------------------------------------------ */
/* p = 2 (six modes per variable)                                       */
/* ------------------------------------------------------------------ */

/* Dubiner p = 2, order [phi_00, phi_10, phi_01, phi_20, phi_11, phi_02]:
 * phi_ij = P_i(a) ((1-b)/2)^i P_j^{(2i+1,0)}(b), a = 2(1+xi)/(1-eta) - 1,
 * b = eta.  With A = a (1-b)/2 = (1 + 2 xi + eta)/2 and B = (1-b)/2:
 *   phi_20 = P_2(a) B^2 = (3 A^2 - B^2)/2,
 *   phi_11 = A P_1^{(3,0)}(eta) = A (3 + 5 eta)/2,
 *   phi_02 = P_2^{(1,0)}(eta) = (5 eta^2 + 2 eta - 1)/2. */
void or_basis2(double xi, double eta, double phi[6], double dphi[6][2]) {
  const double A = 0.5 * (1.0 + 2.0 * xi + eta), B = 0.5 * (1.0 - eta);
  phi[0] = 1.0;
  phi[1] = A;
  phi[2] = 0.5 * (1.0 + 3.0 * eta);
  phi[3] = 0.5 * (3.0 * A * A - B * B);
  phi[4] = 0.5 * A * (3.0 + 5.0 * eta);
  phi[5] = 0.5 * (5.0 * eta * eta + 2.0 * eta - 1.0);
  if (dphi) {
    dphi[0][0] = 0.0; dphi[0][1] = 0.0;
    dphi[1][0] = 1.0; dphi[1][1] = 0.5;
    dphi[2][0] = 0.0; dphi[2][1] = 1.5;
    dphi[3][0] = 3.0 * A; dphi[3][1] = 0.5 * (3.0 * A + B);
    dphi[4][0] = 0.5 * (3.0 + 5.0 * eta); dphi[4][1] = 0.25 * (3.0 + 5.0 * eta) + 2.5 * A;
    dphi[5][0] = 0.0; dphi[5][1] = 5.0 * eta + 1.0;
  }
}

/* P2 READING: area rule of degree 4 with 6 points (Dunavant): two orbits of
 * barycentric points (a, b, b) with their permutations; edge rule: 4-point
 * Gauss-Lobatto (s = -1, -1/sqrt5, 1/sqrt5, 1; weights 1/6, 5/6, 5/6, 1/6),
 * exact to degree 5 = 2p + 1. */
static const double D4_A1 = 0.10810301816807022736, D4_B1 = 0.44594849091596488632, D4_W1 = 0.22338158967801146570;
static const double D4_A2 = 0.81684757298045851308, D4_B2 = 0.09157621350977074346, D4_W2 = 0.10995174365532186764;
static double AREA2_BARY[6][3], AREA2_W[6], EDGE2_S[4], EDGE2_W[4];
static int tables2_ready = 0;

static void tables2(void) {
  if (tables2_ready) return;
  const double orb[2][3] = {{D4_A1, D4_B1, D4_W1}, {D4_A2, D4_B2, D4_W2}};
  for (int o = 0; o < 2; ++o)
    for (int r = 0; r < 3; ++r) {
      int q = 3 * o + r;
      for (int v = 0; v < 3; ++v) AREA2_BARY[q][v] = (v == r) ? orb[o][0] : orb[o][1];
      AREA2_W[q] = orb[o][2];
    }
  const double r5 = 1.0 / sqrt(5.0);
  EDGE2_S[0] = -1.0; EDGE2_S[1] = -r5; EDGE2_S[2] = r5; EDGE2_S[3] = 1.0;
  EDGE2_W[0] = 1.0 / 6.0; EDGE2_W[1] = 5.0 / 6.0; EDGE2_W[2] = 5.0 / 6.0; EDGE2_W[3] = 1.0 / 6.0;
  tables2_ready = 1;
}

void or_area_rule2(double bary[18], double wfrac[6]) {
  tables2();
  for (int q = 0; q < 6; ++q) {
    for (int v = 0; v < 3; ++v) bary[q * 3 + v] = AREA2_BARY[q][v];
    wfrac[q] = AREA2_W[q];
  }
}

void or_edge_rule2(double s[4], double w[4]) {
  tables2();
  for (int g = 0; g < 4; ++g) { s[g] = EDGE2_S[g]; w[g] = EDGE2_W[g]; }
}

/* diagonal of the physical mass matrix divided by the area: the reference
 * norms 2 / ((2i+1)(i+j+1)) over the reference area 2 */
static const double MU2[6] = {1.0, 1.0 / 6.0, 1.0 / 2.0, 1.0 / 15.0, 1.0 / 9.0, 1.0 / 3.0};

void or_mass2(double mu[6]) { for (int k = 0; k < 6; ++k) mu[k] = MU2[k]; }

static void edge_basis2(int l, double s, double phi[6]) {
  static const double V[3][2] = {{-1.0, -1.0}, {1.0, -1.0}, {-1.0, 1.0}};
  int a = (l + 1) % 3, b = (l + 2) % 3;
  double xi = V[a][0] * 0.5 * (1.0 - s) + V[b][0] * 0.5 * (1.0 + s);
  double eta = V[a][1] * 0.5 * (1.0 - s) + V[b][1] * 0.5 * (1.0 + s);
  or_basis2(xi, eta, phi, NULL);
}

#define W6(w, m, k, e, ne) (w)[((size_t)((m) * 6 + (k))) * (ne) + (e)]

static void eval_state2(const double *w, int32_t e, int32_t ne, const double phi[6], double out[3]) {
  for (int m = 0; m < 3; ++m) {
    double s = 0.0;
    for (int k = 0; k < 6; ++k) s += W6(w, m, k, e, ne) * phi[k];
    out[m] = s;
  }
}

/* switch a mesh to p = 2 (before its state is set); the state becomes
 * [3][6][ne] and the area quadrature has 6 points per element */
int32_t or_set_order(or_mesh *M, int32_t p) {
  if (p != 1 && p != 2) return OR_E_INVALID;
  const int32_t ne = M->ne;
  int32_t nm = p == 2 ? 6 : 3, nq = p == 2 ? 6 : 3;
  tables2();
  size_t sw = sizeof(double) * 3 * (size_t)nm * ne;
  free(M->w); free(M->w1); free(M->wt); free(M->dw); free(M->slot); free(M->qxy); free(M->jit); free(M->extra);
  M->extra = NULL; M->src_fn = NULL;
  M->w = calloc(1, sw); M->w1 = calloc(1, sw); M->wt = calloc(1, sw); M->dw = calloc(1, sw);
  M->slot = calloc(1, sizeof(double) * 9 * (size_t)nm * ne);
  M->qxy = malloc(sizeof(double) * 2 * (size_t)nq * ne);
  M->jit = malloc(sizeof(double) * 4 * (size_t)ne);
  if (!M->w || !M->w1 || !M->wt || !M->dw || !M->slot || !M->qxy || !M->jit) return OR_E_NOMEM;
  M->nm = nm; M->nq = nq;
  for (int32_t e = 0; e < ne; ++e) {
    const int32_t *v = M->tri + 3 * e;
    double x1 = M->xy[2 * v[0]], y1 = M->xy[2 * v[0] + 1];
    double x2 = M->xy[2 * v[1]], y2 = M->xy[2 * v[1] + 1];
    double x3 = M->xy[2 * v[2]], y3 = M->xy[2 * v[2] + 1];
    double J11 = 0.5 * (x2 - x1), J12 = 0.5 * (x3 - x1), J21 = 0.5 * (y2 - y1), J22 = 0.5 * (y3 - y1);
    double det = J11 * J22 - J12 * J21;
    /* J^{-T} = 1/det [[J22, -J21], [-J12, J11]] */
    M->jit[4 * e] = J22 / det; M->jit[4 * e + 1] = -J21 / det;
    M->jit[4 * e + 2] = -J12 / det; M->jit[4 * e + 3] = J11 / det;
    for (int q = 0; q < nq; ++q) {
      const double *L = p == 2 ? AREA2_BARY[q] : AREA_BARY[q];
      M->qxy[2 * ((size_t)nq * e + q)] = L[0] * x1 + L[1] * x2 + L[2] * x3;
      M->qxy[2 * ((size_t)nq * e + q) + 1] = L[0] * y1 + L[1] * y2 + L[2] * y3;
    }
  }
  return OR_OK;
}

/* EDGE for p = 2: as edge_integrals with the 4-point rule and the six-mode
 * traces; slot[e][l][k][m] (54 values per element) */
static void edge_integrals2(or_mesh *M, const double *w, double t) {
  const double g = M->prm.g, h0 = M->prm.h0;
  const int32_t ne = M->ne, ned = M->ned;
  const double zb = tide_level(&M->frc, t);
#pragma omp parallel for schedule(static)
  for (int32_t d = 0; d < ned; ++d) {
    int32_t ep = M->ed_el[2 * d], em = M->ed_el[2 * d + 1];
    int lp = M->ed_loc[2 * d], lm = M->ed_loc[2 * d + 1];
    int type = M->ed_type[d];
    double nx = M->ed_n[2 * d], ny = M->ed_n[2 * d + 1], len = M->ed_len[d];
    int32_t na = M->tri[3 * ep + (lp + 1) % 3], nb = M->tri[3 * ep + (lp + 2) % 3];
    double Fp[4][3], Fm[4][3], php[4][6], phm[4][6], wp[4][3], wm[4][3], hbq[4];
    int wetp = is_wet(M, w, ep), wetm = 0;
    for (int gq = 0; gq < 4; ++gq) {
      double s = EDGE2_S[gq];
      edge_basis2(lp, s, php[gq]);
      eval_state2(w, ep, ne, php[gq], wp[gq]);
      hbq[gq] = M->hb[na] * 0.5 * (1.0 - s) + M->hb[nb] * 0.5 * (1.0 + s);
      if (type == 0) {
        edge_basis2(lm, -s, phm[gq]);
        eval_state2(w, em, ne, phm[gq], wm[gq]);
      } else {
        wm[gq][0] = zb; wm[gq][1] = wp[gq][1]; wm[gq][2] = wp[gq][2];
      }
    }
    if (type == 0) wetm = is_wet(M, w, em);
    else if (type == BC_OCEAN) wetm = M->prm.wetdry ? (zb + 0.5 * (M->hb[na] + M->hb[nb]) > h0) : 1;
    if (type == BC_LAND) {
      for (int gq = 0; gq < 4; ++gq) {
        or_wall(g, wp[gq], hbq[gq], nx, ny, wetp, Fp[gq]);
        for (int m = 0; m < 3; ++m) Fm[gq][m] = 0.0;
      }
    } else if (!wetp && !wetm) {
      for (int gq = 0; gq < 4; ++gq)
        for (int m = 0; m < 3; ++m) { Fp[gq][m] = 0.0; Fm[gq][m] = 0.0; }
    } else {
      double F[4][3];
      for (int gq = 0; gq < 4; ++gq) {
        if (M->prm.flux == 1 && wetp && wetm) or_roe(g, wp[gq], wm[gq], hbq[gq], nx, ny, F[gq]);
        else or_llf(g, wp[gq], wm[gq], hbq[gq], nx, ny, wetp, wetm, F[gq]);
      }
      int flood = 1;
      if (!(wetp && wetm)) {
        double mflux = 0.0;
        for (int gq = 0; gq < 4; ++gq) mflux += EDGE2_W[gq] * F[gq][0];
        flood = wetp ? (mflux > 0.0) : (mflux < 0.0);
      }
      if (flood) {
        for (int gq = 0; gq < 4; ++gq)
          for (int m = 0; m < 3; ++m) { Fp[gq][m] = F[gq][m]; Fm[gq][m] = -F[gq][m]; }
      } else if (wetp) {
        for (int gq = 0; gq < 4; ++gq) {
          or_wall(g, wp[gq], hbq[gq], nx, ny, 1, Fp[gq]);
          for (int m = 0; m < 3; ++m) Fm[gq][m] = 0.0;
        }
      } else {
        for (int gq = 0; gq < 4; ++gq) {
          or_wall(g, wm[gq], hbq[gq], -nx, -ny, 1, Fm[gq]);
          for (int m = 0; m < 3; ++m) Fp[gq][m] = 0.0;
        }
      }
    }
    double *sp = M->slot + 54 * (size_t)ep + 18 * lp;
    for (int k = 0; k < 6; ++k)
      for (int m = 0; m < 3; ++m) {
        double s = 0.0;
        for (int gq = 0; gq < 4; ++gq) s += 0.5 * len * EDGE2_W[gq] * php[gq][k] * Fp[gq][m];
        sp[3 * k + m] = s;
      }
    if (type == 0) {
      double *sm = M->slot + 54 * (size_t)em + 18 * lm;
      for (int k = 0; k < 6; ++k)
        for (int m = 0; m < 3; ++m) {
          double s = 0.0;
          for (int gq = 0; gq < 4; ++gq) s += 0.5 * len * EDGE2_W[gq] * phm[gq][k] * Fm[gq][m];
          sm[3 * k + m] = s;
        }
    }
  }
}

/* AREA + GATHER for p = 2: 6-point rule; the basis gradients vary over the
 * element: grad phi_k(x_q) = J^{-T} grad_ref phi_k(xi_q, eta_q) */
static void element_rhs2(or_mesh *M, const double *w, double t, double *dw) {
  const double g = M->prm.g, h0 = M->prm.h0, rho0 = M->prm.rho0;
  const int32_t ne = M->ne;
  if (M->src_fn) M->src_fn(t, 6 * ne, M->qxy, M->extra, M->src_ctx);
#pragma omp parallel for schedule(static)
  for (int32_t e = 0; e < ne; ++e) {
    const int32_t *v = M->tri + 3 * e;
    double A = M->area[e];
    const double *jt = M->jit + 4 * e;
    const double *gl = M->glam + 6 * e;
    double hbv[3], tx[3], ty[3], pa[3];
    for (int i = 0; i < 3; ++i) {
      hbv[i] = M->hb[v[i]];
      tx[i] = M->nodal[3 * v[i]]; ty[i] = M->nodal[3 * v[i] + 1]; pa[i] = M->nodal[3 * v[i] + 2];
    }
    double dhx = 0.0, dhy = 0.0, dpx = 0.0, dpy = 0.0;
    for (int i = 1; i < 3; ++i) {
      dhx += (hbv[i] - hbv[0]) * gl[2 * i]; dhy += (hbv[i] - hbv[0]) * gl[2 * i + 1];
      dpx += (pa[i] - pa[0]) * gl[2 * i]; dpy += (pa[i] - pa[0]) * gl[2 * i + 1];
    }
    double n = M->frc.manning_elem ? M->frc.manning_elem[e] : M->frc.manning_n;
    int wet = is_wet(M, w, e);
    double R[3][6];
    for (int m = 0; m < 3; ++m)
      for (int k = 0; k < 6; ++k) R[m][k] = 0.0;
    for (int q = 0; q < 6; ++q) {
      double xi, eta, phq[6], dref[6][2], wq[3];
      ref_point(AREA2_BARY[q], &xi, &eta);
      or_basis2(xi, eta, phq, dref);
      eval_state2(w, e, ne, phq, wq);
      double hq = AREA2_BARY[q][0] * hbv[0] + AREA2_BARY[q][1] * hbv[1] + AREA2_BARY[q][2] * hbv[2];
      double wA = AREA2_W[q] * A;
      /* volume term */
      double F[3][2];
      phys_flux(g, wq[0], wq[1], wq[2], hq, wet, F);
      for (int k = 1; k < 6; ++k) {
        double gx = jt[0] * dref[k][0] + jt[1] * dref[k][1];
        double gy = jt[2] * dref[k][0] + jt[3] * dref[k][1];
        for (int m = 0; m < 3; ++m) R[m][k] += wA * (gx * F[m][0] + gy * F[m][1]);
      }
      /* source term */
      double ze = wq[0], qx = wq[1], qy = wq[2];
      double H = ze + hq;
      double S[3] = {0.0, 0.0, 0.0};
      if (wet) {
        double Hf = fmax(H, h0);
        double qm = sqrt(qx * qx + qy * qy);
        double fr = g * n * n * qm / pow(Hf, 7.0 / 3.0);
        double txq = AREA2_BARY[q][0] * tx[0] + AREA2_BARY[q][1] * tx[1] + AREA2_BARY[q][2] * tx[2];
        double tyq = AREA2_BARY[q][0] * ty[0] + AREA2_BARY[q][1] * ty[1] + AREA2_BARY[q][2] * ty[2];
        S[1] = g * ze * dhx - fr * qx + txq / rho0 - H / rho0 * dpx + M->frc.coriolis * qy;
        S[2] = g * ze * dhy - fr * qy + tyq / rho0 - H / rho0 * dpy - M->frc.coriolis * qx;
      }
      S[0] += M->frc.rain;
      if (M->extra)
        for (int m = 0; m < 3; ++m) S[m] += M->extra[(size_t)m * 6 * ne + 6 * (size_t)e + q];
      for (int m = 0; m < 3; ++m)
        for (int k = 0; k < 6; ++k) R[m][k] += wA * phq[k] * S[m];
    }
    const double *sl = M->slot + 54 * (size_t)e;
    for (int l = 0; l < 3; ++l)
      for (int k = 0; k < 6; ++k)
        for (int m = 0; m < 3; ++m) R[m][k] -= sl[18 * l + 3 * k + m];
    if (!wet)
      for (int k = 0; k < 6; ++k) { R[1][k] = 0.0; R[2][k] = 0.0; }
    for (int m = 0; m < 3; ++m)
      for (int k = 0; k < 6; ++k) W6(dw, m, k, e, ne) = R[m][k] / (A * MU2[k]);
  }
}

/* values of a six-mode field at the vertices (0..2) and the edge midpoints
 * (3..5: local edges 0, 1, 2) */
static void to_points2(const double u[6], double v[6]) {
  static const double P[6][2] = {{-1.0, -1.0}, {1.0, -1.0}, {-1.0, 1.0}, {0.0, 0.0}, {-1.0, 0.0}, {0.0, -1.0}};
  for (int i = 0; i < 6; ++i) {
    double phi[6];
    or_basis2(P[i][0], P[i][1], phi, NULL);
    double s = 0.0;
    for (int k = 0; k < 6; ++k) s += u[k] * phi[k];
    v[i] = s;
  }
}

/* Post-processing for p = 2 (P2 READINGS).  Both operations keep every
 * element mean and are continuous in their inputs, so that a rounding-level
 * change of the input (FP32 momentum, another summation order) changes the
 * output at rounding level only.
 *
 * Limiter, per variable u (Barth-Jespersen over the six Lagrange nodes of a
 * quadratic): [lo, hi] is the range of the element's and its face
 * neighbours' means, d_i the deviation of the field from its mean u0 at the
 * three vertices and the three edge midpoints, and
 *   theta = min(1, min_i r_i),  r_i = (hi - u0)/d_i (d_i > 0),
 *                               r_i = (lo - u0)/d_i (d_i < 0);
 * modes 1-5 are multiplied by theta.  A linear field takes its extremes at
 * the vertices, so with zero quadratic modes this is the p = 1 limiter.
 *
 * Wet/dry with threshold H0: the depth H = zeta + h_b is a quadratic whose
 * modes are H_k = zeta_k + b_k, b_k the modes of the linear bed (b_k = 0 for
 * k >= 3), with mean Hm = zeta_0 + b_0.
 *   Hm <= H0 -> dry: flat depth Hm, all momentum set to 0 (as p = 1);
 *   else, with Hmin the smallest depth over every point at which the stage
 *   evaluates the element's state (the vertices, the two interior
 *   Gauss-Lobatto points of each edge and the six area points), if
 *   Hmin < H0 the depth's deviation from its mean is scaled by
 *   theta = (Hm - H0)/(Hm - Hmin), which lifts the lowest point to H0:
 *   H_k <- theta H_k for k >= 1, zeta_k = H_k - b_k; momentum unchanged. */
static void depth_points2(double pts[15][2]) {
  static const double V[3][2] = {{-1.0, -1.0}, {1.0, -1.0}, {-1.0, 1.0}};
  int n = 0;
  for (int i = 0; i < 3; ++i) { pts[n][0] = V[i][0]; pts[n][1] = V[i][1]; ++n; }
  for (int l = 0; l < 3; ++l) {
    const int a = (l + 1) % 3, b = (l + 2) % 3;
    for (int g = 1; g <= 2; ++g) {
      const double s = EDGE2_S[g];
      pts[n][0] = V[a][0] * 0.5 * (1.0 - s) + V[b][0] * 0.5 * (1.0 + s);
      pts[n][1] = V[a][1] * 0.5 * (1.0 - s) + V[b][1] * 0.5 * (1.0 + s);
      ++n;
    }
  }
  for (int q = 0; q < 6; ++q) { ref_point(AREA2_BARY[q], &pts[n][0], &pts[n][1]); ++n; }
}

static int32_t postprocess2(or_mesh *M, const double *wt, double *out) {
  if (M->prm.limiter == 2) return OR_E_INVALID;  /* the vertex-based limiter is p = 1 only */
  const int32_t ne = M->ne;
  const double h0 = M->prm.h0;
  double dpts[15][2];
  tables2();
  depth_points2(dpts);
#pragma omp parallel for schedule(static)
  for (int32_t e = 0; e < ne; ++e) {
    double u[3][6];
    for (int m = 0; m < 3; ++m)
      for (int k = 0; k < 6; ++k) u[m][k] = W6(wt, m, k, e, ne);
    if (M->prm.limiter) {
      for (int m = 0; m < 3; ++m) {
        double mean = u[m][0], hi = mean, lo = mean;
        for (int l = 0; l < 3; ++l) {
          int32_t f = M->el_nb[3 * e + l];
          if (f < 0) continue;
          double nbm = W6(wt, m, 0, f, ne);
          if (nbm > hi) hi = nbm;
          if (nbm < lo) lo = nbm;
        }
        double pv[6];
        to_points2(u[m], pv);
        double theta = 1.0;
        for (int i = 0; i < 6; ++i) {
          double d = pv[i] - mean, r = 1.0;
          if (d > 0.0) r = (hi - mean) / d;
          else if (d < 0.0) r = (lo - mean) / d;
          if (r < theta) theta = r;
        }
        for (int k = 1; k < 6; ++k) u[m][k] *= theta;
      }
    }
    if (M->prm.wetdry) {
      const int32_t *vt = M->tri + 3 * e;
      double hbv[3] = {M->hb[vt[0]], M->hb[vt[1]], M->hb[vt[2]]};
      const double b0 = hb_mean(M, e);
      const double b[6] = {b0, 0.5 * (hbv[1] - hbv[0]), 0.5 * (hbv[2] - b0), 0.0, 0.0, 0.0};
      double Hk[6];
      for (int k = 0; k < 6; ++k) Hk[k] = u[0][k] + b[k];
      const double Hm = u[0][0] + b0;
      if (Hm <= h0) {
        /* flat depth: zeta = Hm - h_b, i.e. zeta_k = -b_k for k >= 1 */
        u[0][1] = -b[1]; u[0][2] = -b[2];
        u[0][3] = 0.0; u[0][4] = 0.0; u[0][5] = 0.0;
        for (int k = 0; k < 6; ++k) { u[1][k] = 0.0; u[2][k] = 0.0; }
      } else {
        double Hmin = INFINITY;
        for (int i = 0; i < 15; ++i) {
          double phi[6], s = 0.0;
          or_basis2(dpts[i][0], dpts[i][1], phi, NULL);
          for (int k = 0; k < 6; ++k) s += Hk[k] * phi[k];
          if (s < Hmin) Hmin = s;
        }
        if (Hmin < h0) {
          const double theta = (Hm - h0) / (Hm - Hmin);
          for (int k = 1; k < 6; ++k) u[0][k] = theta * Hk[k] - b[k];
        }
      }
    }
    for (int m = 0; m < 3; ++m)
      for (int k = 0; k < 6; ++k) W6(out, m, k, e, ne) = u[m][k];
  }
  return OR_OK;
}
