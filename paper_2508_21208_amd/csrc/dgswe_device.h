// Device helpers shared by the p = 1 and p = 2 kernels of the gfx950 DG
// shallow-water library: fast reciprocal / root sequences, the time step
// control, the tide, the edge fluxes of both sides, the CFL candidate,
// state views, chunk records and the XCD-aware block mapping.
#pragma once

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

// Reciprocal, square root and cube root for the flux and source arithmetic.
// FP64: the hardware estimates refined by Newton (reciprocal, square root)
// or Halley (cube root) iterations, within about 1 ulp instead of the
// correctly rounded library sequences.  FP32: the hardware instructions
// (about 1 ulp).  Arguments are finite and in the normal range (depths >=
// h0, lengths and areas of a mesh).
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
HD float rcp_nr(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
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
HD float sqrt_nr(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_sqrtf(x);
#else
  return sqrtf(x);
#endif
}

// cube root of x > 0: float estimate 2^(log2(x)/3); FP64 adds one Halley
// step y <- y (y^3 + 2x) / (2y^3 + x) (cubic convergence)
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
HD float cbrt_nr(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 3.0f));
#else
  return cbrtf(x);
#endif
}

// Cache policy of the stage kernel's global accesses.  ld_once: records a
// launch reads exactly once (packed chunk records, element geometry); st_out:
// stage results no kernel of this launch reads back.  With the non-temporal
// forms they do not displace the state arrays that neighbouring chunks
// re-read from L2.
#ifndef DGSWE_NT_LOAD
#define DGSWE_NT_LOAD 1
#endif
#ifndef DGSWE_NT_STORE
#define DGSWE_NT_STORE 0
#endif
#if defined(__HIP_DEVICE_COMPILE__) && DGSWE_NT_LOAD
typedef double dgswe_d2v __attribute__((ext_vector_type(2)));
typedef int dgswe_i4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double2 ld_once(const double2 *p) {
  const dgswe_d2v v = __builtin_nontemporal_load((const dgswe_d2v *)p);
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ int4 ld_once(const int4 *p) {
  const dgswe_i4v v = __builtin_nontemporal_load((const dgswe_i4v *)p);
  return make_int4(v.x, v.y, v.z, v.w);
}
template <class T>
__device__ __forceinline__ T ld_once(const T *p) { return __builtin_nontemporal_load(p); }
#else
template <class T>
HD T ld_once(const T *p) { return *p; }
#endif
#if defined(__HIP_DEVICE_COMPILE__) && DGSWE_NT_STORE
template <class T>
__device__ __forceinline__ void st_out(T *p, T v) { __builtin_nontemporal_store(v, p); }
#else
template <class T>
HD void st_out(T *p, T v) { *p = v; }
#endif

// dt of the current step: fixed, or cfl x the CFL minimum of w^n (capped),
// from the bit pattern of that minimum.  Returns false when no wet element
// defines it and there is no cap.
HD bool dt_from_bits(const Params &p, unsigned long long bits, double &dt) {
  if (p.dt_fixed > 0.0) { dt = p.dt_fixed; return true; }
  double raw = bits_to_double(bits);
  if (raw == INFINITY) {
    if (p.dt_max > 0.0) { dt = p.dt_max; return true; }
    return false;
  }
  double d = p.cfl * raw;
  if (p.dt_max > 0.0 && d > p.dt_max) d = p.dt_max;
  dt = d;
  return true;
}
HD bool step_dt(const Ctrl *c, const Params &p, int slot, double &dt) { return dt_from_bits(p, c->dtmin[slot], dt); }

// (unrolled over the constituent slots, so the constants are read with
// constant offsets - scalar loads - and no vector load inside a loop makes
// the kernel wait for every load it has in flight)
HD double tide_level(const Member &f, double t) {
  double z = f.tide_offset;
#pragma unroll
  for (int i = 0; i < kMaxTide; ++i)
    if (i < f.n_tide) z += f.tide_amp[i] * cos(f.tide_omega[i] * t + f.tide_phase[i]);
  return z;
}

// hydrostatic flux g/2 (H^2 - h_b^2) written as g/2 zeta (zeta + 2 h_b), FP64
HD double p_hydro(double g, double ze, double hb) { return 0.5 * g * ze * (ze + 2.0 * hb); }

// normal physical flux F(w).n of one side; u = 0 on a dry side.  zeta and
// h_b FP64; momentum, normal and result in R.
template <class R>
HD void flux_n(double g, double ze, R qx, R qy, double hb, bool wet, R nx, R ny, R &un, R f[3]) {
  const R H = (R)(ze + hb);
  const R qn = qx * nx + qy * ny;
  un = wet ? qn * rcp_nr(H) : (R)0;
  const R p = (R)p_hydro(g, ze, hb);
  f[0] = qn;
  f[1] = qx * un + p * nx;
  f[2] = qy * un + p * ny;
}

// local Lax-Friedrichs flux from side L (normal n points from L to R); the
// zeta jump is formed in FP64
template <class R>
HD void llf(double g, double zl, R qlx, R qly, double zr, R qrx, R qry, double hb, R nx, R ny, bool wetl,
            bool wetr, R out[3]) {
  R unl, unr, fl[3], fr[3];
  flux_n<R>(g, zl, qlx, qly, hb, wetl, nx, ny, unl, fl);
  flux_n<R>(g, zr, qrx, qry, hb, wetr, nx, ny, unr, fr);
  const R cl = sqrt_nr((R)(g * fmax(zl + hb, 0.0)));
  const R cr = sqrt_nr((R)(g * fmax(zr + hb, 0.0)));
  const R lam = fmax(fabs(unl) + cl, fabs(unr) + cr);
  const R jump[3] = {(R)(zr - zl), qrx - qlx, qry - qly};
  for (int m = 0; m < 3; ++m) out[m] = (R)0.5 * (fl[m] + fr[m]) - (R)0.5 * lam * jump[m];
}

// Roe flux from side L (normal n from L to R) for two wet sides: Roe
// averages of the normal and tangential velocity (square-root depth
// weights) and c = sqrt(g (H_L + H_R)/2); waves u_n - c, u_n, u_n + c on
// (H, q_n, q_t) with Harten-Hyman entropy fixes on the two acoustic waves.
// Depths and the zeta jump are formed in FP64; a side without positive
// depth at the point falls back to LLF.
template <class R>
HD void roe(double g, double zl, R qlx, R qly, double zr, R qrx, R qry, double hb, R nx, R ny, R out[3]) {
  const double Hld = zl + hb, Hrd = zr + hb;
  if (!(Hld > 0.0 && Hrd > 0.0)) {
    llf<R>(g, zl, qlx, qly, zr, qrx, qry, hb, nx, ny, true, true, out);
    return;
  }
  R unl, unr, fl[3], fr[3];
  flux_n<R>(g, zl, qlx, qly, hb, true, nx, ny, unl, fl);
  flux_n<R>(g, zr, qrx, qry, hb, true, nx, ny, unr, fr);
  const R Hl = (R)Hld, Hr = (R)Hrd;
  const R utl = (qly * nx - qlx * ny) * rcp_nr(Hl), utr = (qry * nx - qrx * ny) * rcp_nr(Hr);
  const R sl = sqrt_nr(Hl), sr = sqrt_nr(Hr);
  const R isum = rcp_nr(sl + sr);
  const R un = (sl * unl + sr * unr) * isum, ut = (sl * utl + sr * utr) * isum;
  const R c = sqrt_nr((R)(0.5 * g * (Hld + Hrd)));
  const R dH = (R)(zr - zl);
  const R dqx = qrx - qlx, dqy = qry - qly;
  const R dqn = dqx * nx + dqy * ny, dqt = dqy * nx - dqx * ny;
  const R i2c = rcp_nr((R)2 * c);
  const R a1 = ((un + c) * dH - dqn) * i2c, a2 = dqt - ut * dH, a3 = (dqn - (un - c) * dH) * i2c;
  const R l1 = un - c, l3 = un + c;
  const R cl = sqrt_nr((R)(g * Hld)), cr = sqrt_nr((R)(g * Hrd));
  const R d1 = fmax((R)0, fmax(l1 - (unl - cl), (unr - cr) - l1));
  const R d3 = fmax((R)0, fmax(l3 - (unl + cl), (unr + cr) - l3));
  R m1 = fabs(l1), m3 = fabs(l3);
  const R m2 = fabs(un);
  if (m1 < d1) m1 = (l1 * l1 + d1 * d1) * rcp_nr((R)2 * d1);
  if (m3 < d3) m3 = (l3 * l3 + d3 * d3) * rcp_nr((R)2 * d3);
  const R DH = m1 * a1 + m3 * a3;
  const R Dn = m1 * a1 * l1 + m3 * a3 * l3;
  const R Dt = (m1 * a1 + m3 * a3) * ut + m2 * a2;
  out[0] = (R)0.5 * (fl[0] + fr[0]) - (R)0.5 * DH;
  out[1] = (R)0.5 * (fl[1] + fr[1]) - (R)0.5 * (Dn * nx - Dt * ny);
  out[2] = (R)0.5 * (fl[2] + fr[2]) - (R)0.5 * (Dn * ny + Dt * nx);
}

// land wall: LLF against the mirror state, closed form, zero mass flux
template <class R>
HD void wall(double g, double ze, R qx, R qy, double hb, R nx, R ny, bool wet, R out[3]) {
  const R p = (R)p_hydro(g, ze, hb);
  R f = p;
  if (wet) {
    const double Hd = ze + hb;
    const R iH = rcp_nr((R)Hd);
    const R qn = qx * nx + qy * ny;
    const R lam = fabs(qn) * iH + sqrt_nr((R)(g * fmax(Hd, 0.0)));
    f = qn * qn * iH + p + lam * qn;
  }
  out[0] = (R)0;
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

HD void holland(const Member &f, double x, double y, double t, double out[3]) {
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

HD double mean3(const double h[3]) { return (h[0] + h[1] + h[2]) / 3.0; }

// CFL candidate 2 r_e / (|Q_mean| / H_mean + sqrt(g H_mean)) of a state
// (INFINITY when dry); unchanged by the post-processing.
HD double cfl_candidate(double z0, double qx0, double qy0, double hmean, double inr2, const Params &p) {
  const double Hm = z0 + hmean;
  const bool wet = p.wetdry ? (Hm > p.h0) : true;
  if (!wet) return INFINITY;
  const double lam = sqrt(qx0 * qx0 + qy0 * qy0) / Hm + sqrt(p.g * Hm);
  return inr2 / lam;
}

// ---------------------------------------------------------------- global-memory views
// A state buffer: zeta modes [3][ne] FP64, then momentum modes [6][ne] of
// type QT (Qx modes 0-2, Qy modes 0-2), each mode contiguous.
template <class QT>
struct St {
  double *z;
  QT *q;
};
template <class QT>
struct CSt {
  const double *z;
  const QT *q;
};

struct ChunkInfo {
  int c, c0, cc, h1o, n1, h2o, n2, leo, ne_loc, lo, member, first, man_base, man_step;
  HD int nl() const { return cc + n1; }
};

HD ChunkInfo chunk_info(const DevMesh &m, int c) {
  const int *r = m.chunk_rec + (size_t)c * kChunkRec;
  ChunkInfo k;
  k.c = c;
  k.c0 = r[0]; k.cc = r[1];
  k.h1o = r[2]; k.n1 = r[3];
  k.h2o = r[4]; k.n2 = r[5];
  k.leo = r[6]; k.ne_loc = r[7];
  k.lo = r[8];
  k.member = r[9];
  k.first = r[10];
  k.man_base = r[11];
  k.man_step = r[12];
  return k;
}

// Manning n of element i of a chunk
HD double manning_of(const DevMesh &m, const ChunkInfo &k, int i, double) {
  return m.man[(size_t)k.man_base + (size_t)i * k.man_step];
}
HD float manning_of(const DevMesh &m, const ChunkInfo &k, int i, float) {
  return m.manf[(size_t)k.man_base + (size_t)i * k.man_step];
}

// ---------------------------------------------------------------- block helpers
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

// views of a state buffer: zeta modes first, then the momentum modes
template <class QT>
inline St<QT> split(void *buf, size_t ne) {
  return {(double *)buf, (QT *)((double *)buf + 3 * ne)};
}
template <class QT>
inline CSt<QT> csplit(const void *buf, size_t ne) {
  return {(const double *)buf, (const QT *)((const double *)buf + 3 * ne)};
}

}  // namespace dgswe
