// C ABI of the gfx950 DG shallow-water step: solver lifetime, host<->device
// transfers (with the internal element permutation), the per-step launch
// sequence and HIP-event kernel timing.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "dgswe_internal.h"
#include "../../include/dgswe.h"

using namespace dgswe;

namespace {
thread_local std::string g_create_error = "no error";

enum KernelId { K_FORCING = 0, K_STAGE, K_COUNT };
const char *kKernelNames[K_COUNT] = {"k_forcing", "k_stage"};
}  // namespace

struct dgswe_solver {
  dgswe_params uprm{};
  Params prm{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  int nn = 0, ne = 0, ned = 0, nbnd = 0;
  std::vector<int> perm;  // internal -> caller element
  std::vector<void *> allocs;
  DevMesh m{};
  DevState s{};
  double *d_manning = nullptr;   // per-element Manning n (internal order)
  float *d_manningf = nullptr;
  double *d_manning1 = nullptr;  // one uniform Manning n
  float *d_manning1f = nullptr;
  double *d_diag = nullptr;
  int precision = DGSWE_FP64;
  double *rb = nullptr;  // FP64 [9][ne] read-back buffer (mixed path)
  long long steps_enq = 0;
  int block = 256;         // workgroup size of the stage kernel
  int cur = 0;             // buffer holding w^n (unlimited unless cur_is_pp)
  bool cur_is_pp = false;  // w^n is already post-processed (set_state without post-processing)
  bool forcing_dynamic = false;
  std::string err = "no error";
  std::vector<double> stage_buf;
  std::vector<unsigned char> stage_raw;
  // kernel timing
  bool prof = false;
  struct Rec { int k; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double prof_ms[K_COUNT] = {0, 0};
  long long prof_n[K_COUNT] = {0, 0};
};

namespace {

dgswe_status fail(dgswe_solver *s, dgswe_status st, const std::string &msg) {
  if (s) s->err = msg;
  else g_create_error = msg;
  return st;
}

dgswe_status hip_fail(dgswe_solver *s, hipError_t e, const char *what) {
  return fail(s, DGSWE_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
hipError_t dev_alloc(dgswe_solver *S, T **p, size_t n) {
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, n * sizeof(T) + 16);
  if (e == hipSuccess) S->allocs.push_back(q);
  *p = (T *)q;
  return e;
}

template <class T>
hipError_t upload(dgswe_solver *S, const T **dst, const std::vector<T> &v) {
  T *p = nullptr;
  hipError_t e = dev_alloc(S, &p, v.size());
  if (e != hipSuccess) return e;
  e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  *dst = p;
  return e;
}

// Host image of a caller-order FP64 [9][ne] state in the internal order and
// the solver's buffer layout (zeta FP64, momentum FP64 or FP32).
void pack_state(dgswe_solver *S, const double *w) {
  const size_t ne = S->ne;
  S->stage_raw.resize(state_bytes(ne, S->precision));
  double *z = (double *)S->stage_raw.data();
  for (size_t j = 0; j < 3; ++j)
    for (size_t i = 0; i < ne; ++i) z[j * ne + i] = w[j * ne + (size_t)S->perm[i]];
  if (S->precision == DGSWE_MIXED) {
    float *q = (float *)(z + 3 * ne);
    for (size_t j = 0; j < 6; ++j)
      for (size_t i = 0; i < ne; ++i) q[j * ne + i] = (float)w[(3 + j) * ne + (size_t)S->perm[i]];
  } else {
    double *q = z + 3 * ne;
    for (size_t j = 0; j < 6; ++j)
      for (size_t i = 0; i < ne; ++i) q[j * ne + i] = w[(3 + j) * ne + (size_t)S->perm[i]];
  }
}

void free_all(dgswe_solver *S) {
  for (void *p : S->allocs) (void)hipFree(p);
  S->allocs.clear();
  for (auto &r : S->recs) { S->pool.push_back(r.a); S->pool.push_back(r.b); }
  S->recs.clear();
  for (hipEvent_t ev : S->pool) (void)hipEventDestroy(ev);
  S->pool.clear();
  if (S->own_stream && S->stream) (void)hipStreamDestroy(S->stream);
  S->stream = nullptr;
}

bool validate_params(const dgswe_params *p, std::string &msg) {
  if (!p) { msg = "params is NULL"; return false; }
  if (p->p != 1) { msg = "only p = 1 is supported"; return false; }
  if (p->precision != DGSWE_FP64 && p->precision != DGSWE_MIXED) {
    msg = "precision must be DGSWE_FP64 or DGSWE_MIXED";
    return false;
  }
  if (!(p->g > 0) || !(p->rho0 > 0) || !(p->h0 > 0)) { msg = "g, rho0 and h0 must be positive"; return false; }
  if (!(p->dt_fixed > 0) && !(p->cfl > 0)) { msg = "cfl must be positive when dt_fixed <= 0"; return false; }
  return true;
}

// event-bracketed launch helper
struct Timed {
  dgswe_solver *S;
  int k;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(dgswe_solver *S_, int k_) : S(S_), k(k_) {
    if (!S->prof) return;
    a = take();
    b = take();
    if (a && b) (void)hipEventRecord(a, S->stream);
  }
  hipEvent_t take() {
    if (!S->pool.empty()) { hipEvent_t ev = S->pool.back(); S->pool.pop_back(); return ev; }
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    return ev;
  }
  ~Timed() {
    if (!S->prof) return;
    if (a && b) {
      (void)hipEventRecord(b, S->stream);
      S->recs.push_back({k, a, b});
    } else {
      if (a) S->pool.push_back(a);
      if (b) S->pool.push_back(b);
    }
  }
};

dgswe_status drain_profile(dgswe_solver *S) {
  hipError_t e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "hipStreamSynchronize");
  for (auto &r : S->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      S->prof_ms[r.k] += ms;
      S->prof_n[r.k] += 1;
    }
    S->pool.push_back(r.a);
    S->pool.push_back(r.b);
  }
  S->recs.clear();
  return DGSWE_OK;
}

}  // namespace

extern "C" {

void dgswe_default_params(dgswe_params *p) {
  if (!p) return;
  p->p = 1;
  p->precision = DGSWE_FP64;
  p->g = 9.81;
  p->rho0 = 1000.0;
  p->h0 = 0.01;
  p->cfl = 0.2;
  p->dt_fixed = 0.0;
  p->dt_max = 0.0;
  p->limiter = 1;
  p->wetdry = 1;
}

dgswe_status dgswe_create_mesh(int32_t n_nodes, const double *node_xy, const double *node_hb,
                               int32_t n_elems, const int32_t *tri, int32_t n_bnd,
                               const int32_t *bnd_nodes, const int32_t *bnd_type,
                               const dgswe_params *prm, void *hip_stream, dgswe_solver **out) {
  if (!out) return fail(nullptr, DGSWE_E_INVALID, "out is NULL");
  *out = nullptr;
  std::string msg;
  if (!validate_params(prm, msg)) return fail(nullptr, DGSWE_E_INVALID, msg);
  Prep P;
  int rc = prepare_mesh(n_nodes, node_xy, node_hb, n_elems, tri, n_bnd, bnd_nodes, bnd_type, P, msg);
  if (rc != DGSWE_OK) return fail(nullptr, (dgswe_status)rc, msg);

  dgswe_solver *S = new (std::nothrow) dgswe_solver();
  if (!S) return fail(nullptr, DGSWE_E_NOMEM, "host allocation failed");
  hipError_t e = hipGetDevice(&S->device);
  if (e != hipSuccess) { delete S; return fail(nullptr, DGSWE_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e)); }
  if (hip_stream) {
    S->stream = (hipStream_t)hip_stream;
  } else {
    e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
    if (e != hipSuccess) { delete S; return fail(nullptr, DGSWE_E_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e)); }
    S->own_stream = true;
  }
  S->uprm = *prm;
  S->nn = P.nn; S->ne = P.ne; S->ned = P.ned; S->nbnd = P.nbnd;
  S->perm = P.perm;
  S->precision = prm->precision;
  const bool mixed = S->precision == DGSWE_MIXED;
  Params &pp = S->prm;
  pp.g = prm->g; pp.rho0 = prm->rho0; pp.h0 = prm->h0; pp.cfl = prm->cfl;
  pp.dt_fixed = prm->dt_fixed; pp.dt_max = prm->dt_max;
  pp.limiter = prm->limiter ? 1 : 0; pp.wetdry = prm->wetdry ? 1 : 0;
  pp.manning_n = 0.0; pp.n_tide = 0; pp.tide_offset = 0.0; pp.holland = 0; pp.pn = 101300.0;

  DevMesh &m = S->m;
  m.ne = P.ne; m.nn = P.nn; m.ned = P.ned;
  const size_t ne = P.ne, ned = P.ned, nn = P.nn;
  bool ok = true;
  auto chk = [&](hipError_t x) { if (x != hipSuccess) ok = false; };
  chk(upload(S, &m.area, P.area)); chk(upload(S, &m.inr2, P.inr2));
  chk(upload(S, &m.hbv, P.hbv));
  chk(upload(S, &m.el_nb, P.el_nb));
  chk(upload(S, &m.node_x, P.node_x)); chk(upload(S, &m.node_y, P.node_y));
  chk(dev_alloc(S, &S->d_manning1, 1));
  chk(dev_alloc(S, &S->d_manning1f, 1));
  m.manning = S->d_manning1;
  m.manningf = S->d_manning1f;
  m.manning_step = 0;
  // chunk size and workgroup size of the stage kernel
  int chunk = 256, block = 256;
  if (const char *ev = std::getenv("DGSWE_CHUNK")) chunk = std::atoi(ev);
  if (const char *ev = std::getenv("DGSWE_BLOCK")) block = std::atoi(ev);
  if (!stage_block_ok(block) || chunk < 64 || chunk > block) {
    free_all(S);
    delete S;
    return fail(nullptr, DGSWE_E_INVALID, "unsupported chunk/block configuration");
  }
  S->block = block;
  build_chunks(P, chunk);
  m.C = P.C; m.nch = P.nch; m.nl_max = P.nl_max; m.nm_max = P.nm_max; m.ed_max = P.ed_max;
  m.n2_max = P.n2_max;
  chk(upload(S, &m.h1_off, P.h1_off)); chk(upload(S, &m.lgid, P.lgid));
  chk(upload(S, &m.h2_off, P.h2_off)); chk(upload(S, &m.h2, P.h2));
  chk(upload(S, &m.le_off, P.le_off)); chk(upload(S, &m.lo_off, P.lo_off));
  chk(upload(S, &m.eai, P.eai)); chk(upload(S, &m.enode, P.enode));
  chk(upload(S, &m.lhb01, P.lhb01)); chk(upload(S, &m.lhb2, P.lhb2)); chk(upload(S, &m.lnb, P.lnb));
  m.eg1 = m.eg2 = m.le_a = m.le_b = nullptr;
  m.egf = m.le_f = nullptr;
  if (mixed) {
    chk(upload(S, &m.egf, P.egf));
    chk(upload(S, &m.le_f, P.le_f));
  } else {
    chk(upload(S, &m.eg1, P.eg1)); chk(upload(S, &m.eg2, P.eg2));
    chk(upload(S, &m.le_a, P.le_a)); chk(upload(S, &m.le_b, P.le_b));
  }
  const size_t lds = stage_lds_bytes(m, S->precision);
  if (lds > 80 * 1024 || P.nl_max > 2 * block || P.ed_max > 2 * block) {
    free_all(S);
    delete S;
    return fail(nullptr, DGSWE_E_MESH, "element chunks have halos too large for the LDS (" +
                                           std::to_string(lds) + " bytes)");
  }
  DevState &st = S->s;
  const size_t sb = state_bytes(ne, S->precision);
  for (int b = 0; b < 3; ++b) {
    unsigned char *q = nullptr;
    chk(dev_alloc(S, &q, sb));
    st.buf[b] = q;
  }
  {
    unsigned char *q = nullptr;
    chk(dev_alloc(S, &q, sb));
    st.wpp = q;
  }
  if (mixed) chk(dev_alloc(S, &S->rb, 9 * ne));
  chk(dev_alloc(S, &st.nodal, 3 * nn)); chk(dev_alloc(S, &st.partial, 3 * (size_t)diag_blocks(P.ne)));
  chk(dev_alloc(S, &st.ctrl, 1)); chk(dev_alloc(S, &S->d_diag, 4));
  if (!ok) {
    free_all(S);
    delete S;
    return fail(nullptr, DGSWE_E_NOMEM, "device allocation or upload failed");
  }
  // zero state and forcing, dt of the zero state
  chk(hipMemsetAsync(st.buf[0], 0, sb, S->stream));
  chk(hipMemsetAsync(st.nodal, 0, 3 * nn * sizeof(double), S->stream));
  chk(hipMemsetAsync(S->d_manning1, 0, sizeof(double), S->stream));
  chk(hipMemsetAsync(S->d_manning1f, 0, sizeof(float), S->stream));
  chk(launch_init_state(m, st, pp, st.buf[0], 0.0, S->precision, S->stream));
  chk(hipStreamSynchronize(S->stream));
  S->cur = 0;
  S->cur_is_pp = true;
  if (!ok) {
    free_all(S);
    delete S;
    return fail(nullptr, DGSWE_E_DEVICE, "device initialisation failed");
  }
  *out = S;
  return DGSWE_OK;
}

dgswe_status dgswe_set_state(dgswe_solver *S, double t, const double *w, int32_t postprocess) {
  if (!S) return fail(nullptr, DGSWE_E_INVALID, "solver is NULL");
  if (!w) return fail(S, DGSWE_E_INVALID, "state is NULL");
  if (!std::isfinite(t)) return fail(S, DGSWE_E_INVALID, "time is not finite");
  pack_state(S, w);
  // The stored state is post-processed by the first stage that reads it;
  // a state given without post-processing is marked as already done.
  S->cur = 0;
  S->cur_is_pp = postprocess == 0;
  hipError_t e = hipMemcpyAsync(S->s.buf[0], S->stage_raw.data(), S->stage_raw.size(), hipMemcpyHostToDevice,
                                S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "hipMemcpyAsync");
  S->steps_enq = 0;
  e = launch_init_state(S->m, S->s, S->prm, S->s.buf[0], t, S->precision, S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "init kernel");
  e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "hipStreamSynchronize");
  return DGSWE_OK;
}

dgswe_status dgswe_set_forcing(dgswe_solver *S, const dgswe_forcing *f) {
  if (!S) return fail(nullptr, DGSWE_E_INVALID, "solver is NULL");
  if (!f) return fail(S, DGSWE_E_INVALID, "forcing is NULL");
  if (f->n_tide < 0 || f->n_tide > kMaxTide) return fail(S, DGSWE_E_INVALID, "at most 8 tidal constituents");
  if (f->n_tide > 0 && (!f->tide_amp || !f->tide_omega || !f->tide_phase))
    return fail(S, DGSWE_E_INVALID, "tidal arrays are NULL");
  if (f->holland && !(f->rmax > 0 && f->B > 0 && f->rho_air > 0))
    return fail(S, DGSWE_E_INVALID, "Holland rmax, B and rho_air must be positive");
  const size_t ne = S->ne, nn = S->nn;
  hipError_t e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "hipStreamSynchronize");
  Params &p = S->prm;
  p.manning_n = f->manning_n;
  p.n_tide = f->n_tide;
  for (int i = 0; i < f->n_tide; ++i) {
    p.tide_amp[i] = f->tide_amp[i]; p.tide_omega[i] = f->tide_omega[i]; p.tide_phase[i] = f->tide_phase[i];
  }
  p.tide_offset = f->tide_offset;
  p.holland = f->holland ? 1 : 0;
  p.x0 = f->x0; p.y0 = f->y0; p.vx = f->vx; p.vy = f->vy; p.dp = f->dp; p.pn = f->pn;
  p.rmax = f->rmax; p.B = f->B; p.rho_air = f->rho_air; p.coriolis_f = f->coriolis_f; p.wind_factor = f->wind_factor;
  if (f->manning_n_elem) {
    if (!S->d_manning) {
      e = dev_alloc(S, &S->d_manning, ne);
      if (e != hipSuccess) return fail(S, DGSWE_E_NOMEM, "device allocation failed");
    }
    std::vector<double> tmp(ne);
    for (size_t i = 0; i < ne; ++i) tmp[i] = f->manning_n_elem[S->perm[i]];
    e = hipMemcpy(S->d_manning, tmp.data(), ne * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
    S->m.manning = S->d_manning;
    S->m.manning_step = 1;
    if (S->precision == DGSWE_MIXED) {
      if (!S->d_manningf) {
        e = dev_alloc(S, &S->d_manningf, ne);
        if (e != hipSuccess) return fail(S, DGSWE_E_NOMEM, "device allocation failed");
      }
      std::vector<float> tf(ne);
      for (size_t i = 0; i < ne; ++i) tf[i] = (float)tmp[i];
      e = hipMemcpy(S->d_manningf, tf.data(), ne * sizeof(float), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
      S->m.manningf = S->d_manningf;
    }
  } else {
    const float nf = (float)f->manning_n;
    e = hipMemcpy(S->d_manning1, &f->manning_n, sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(S->d_manning1f, &nf, sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
    S->m.manning = S->d_manning1;
    S->m.manningf = S->d_manning1f;
    S->m.manning_step = 0;
  }
  S->forcing_dynamic = p.holland != 0;
  if (!p.holland) {
    // (tau_x, tau_y) pairs per node, then p_a per node
    std::vector<double> tmp(3 * nn, 0.0);
    for (size_t i = 0; i < nn; ++i) {
      if (f->wind_tau) { tmp[2 * i] = f->wind_tau[2 * i]; tmp[2 * i + 1] = f->wind_tau[2 * i + 1]; }
      if (f->patm) tmp[2 * nn + i] = f->patm[i];
    }
    e = hipMemcpy(S->s.nodal, tmp.data(), 3 * nn * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
  }
  return DGSWE_OK;
}

dgswe_status dgswe_step(dgswe_solver *S, int32_t n_steps) {
  if (!S) return fail(nullptr, DGSWE_E_INVALID, "solver is NULL");
  if (n_steps < 0) return fail(S, DGSWE_E_INVALID, "n_steps < 0");
  const DevMesh &m = S->m;
  DevState &st = S->s;
  const Params &p = S->prm;
  const int want_dt = (p.dt_fixed > 0.0) ? 0 : 1;
  for (int i = 0; i < n_steps; ++i) {
    const int slot = (int)(S->steps_enq & 1);
    // rotation: w^n in cur, stage 1 -> s1, stage 2 -> nx (both unlimited)
    const int cur = S->cur, s1 = (cur + 1) % 3, nx = (cur + 2) % 3;
    const int pp_cur = S->cur_is_pp ? 0 : 1;
    hipError_t e = hipSuccess;
    for (int stage = 0; stage < 2 && e == hipSuccess; ++stage) {
      if (S->forcing_dynamic) {
        Timed t(S, K_FORCING);
        e = launch_forcing(m, st, p, slot, stage, S->stream);
      }
      if (e != hipSuccess) break;
      Timed t(S, K_STAGE);
      if (stage == 0)
        e = launch_stage(m, st, p, st.buf[cur], nullptr, st.buf[s1], st.wpp, slot, 0, pp_cur, 0, S->block,
                         S->precision, S->stream);
      else
        e = launch_stage(m, st, p, st.buf[s1], st.wpp, st.buf[nx], nullptr, slot, 1, 1, want_dt, S->block,
                         S->precision, S->stream);
    }
    if (e != hipSuccess) return hip_fail(S, e, "kernel launch");
    S->cur = nx;
    S->cur_is_pp = false;
    S->steps_enq += 1;
  }
  return DGSWE_OK;
}

dgswe_status dgswe_read_state(dgswe_solver *S, double *w_out, dgswe_diag *d) {
  if (!S) return fail(nullptr, DGSWE_E_INVALID, "solver is NULL");
  hipError_t e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "hipStreamSynchronize");
  const size_t ne = S->ne;
  if (w_out) {
    // the state at the boundary is post-processed FP64 [9][ne]; in FP64 a
    // free state buffer takes the post-processed copy
    const void *src = S->s.buf[S->cur];
    if (!S->cur_is_pp || S->precision == DGSWE_MIXED) {
      double *tmp = S->precision == DGSWE_MIXED ? S->rb : (double *)S->s.buf[(S->cur + 1) % 3];
      e = launch_post_only(S->m, S->prm, src, S->cur_is_pp ? 0 : 1, tmp, S->precision, S->stream);
      if (e != hipSuccess) return hip_fail(S, e, "post-processing kernel");
      src = tmp;
    }
    S->stage_buf.resize(9 * ne);
    e = hipMemcpyAsync(S->stage_buf.data(), src, 9 * ne * sizeof(double), hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
    for (size_t j = 0; j < 9; ++j)
      for (size_t i = 0; i < ne; ++i) w_out[j * ne + (size_t)S->perm[i]] = S->stage_buf[j * ne + i];
  }
  Ctrl c{};
  if (d) {
    e = launch_diag(S->m, S->s, S->prm, S->s.buf[S->cur], S->d_diag, S->stream);
    if (e != hipSuccess) return hip_fail(S, e, "diagnostics kernel");
    double out4[4];
    e = hipMemcpyAsync(out4, S->d_diag, sizeof out4, hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
    d->mass = out4[0];
    d->volume = out4[1];
    d->n_wet = (int32_t)out4[2];
    d->n_dry = (int32_t)(S->ne - d->n_wet);
  }
  e = hipMemcpy(&c, S->s.ctrl, sizeof c, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
  if (d) {
    d->t = c.t[c.steps & 1];
    d->dt_last = c.dt_last;
    d->steps = c.steps;
  }
  if (c.status == DGSWE_E_NONFINITE) return fail(S, DGSWE_E_NONFINITE, "non-finite value in the state");
  if (c.status == DGSWE_E_ALLDRY) return fail(S, DGSWE_E_ALLDRY, "no wet element defines the CFL time step");
  if (c.status) return fail(S, DGSWE_E_DEVICE, "device status " + std::to_string(c.status));
  return DGSWE_OK;
}

void dgswe_destroy(dgswe_solver *S) {
  if (!S) return;
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  free_all(S);
  delete S;
}

const char *dgswe_last_error(const dgswe_solver *S) {
  return S ? S->err.c_str() : g_create_error.c_str();
}

dgswe_status dgswe_profile(dgswe_solver *S, int32_t enable) {
  if (!S) return fail(nullptr, DGSWE_E_INVALID, "solver is NULL");
  dgswe_status st = drain_profile(S);
  if (st != DGSWE_OK) return st;
  for (int k = 0; k < K_COUNT; ++k) { S->prof_ms[k] = 0.0; S->prof_n[k] = 0; }
  S->prof = enable != 0;
  return DGSWE_OK;
}

dgswe_status dgswe_profile_read(dgswe_solver *S, int32_t max_kernels, char *names, double *total_ms,
                                int64_t *launches, int32_t *n_out) {
  if (!S) return fail(nullptr, DGSWE_E_INVALID, "solver is NULL");
  if (max_kernels < 0 || (max_kernels > 0 && (!names || !total_ms || !launches)) || !n_out)
    return fail(S, DGSWE_E_INVALID, "bad output buffers");
  dgswe_status st = drain_profile(S);
  if (st != DGSWE_OK) return st;
  int n = 0;
  for (int k = 0; k < K_COUNT && n < max_kernels; ++k) {
    std::strncpy(names + 32 * n, kKernelNames[k], 31);
    names[32 * n + 31] = 0;
    total_ms[n] = S->prof_ms[k];
    launches[n] = S->prof_n[k];
    ++n;
  }
  *n_out = n;
  return DGSWE_OK;
}

dgswe_status dgswe_mesh_info(const dgswe_solver *S, int64_t out[4]) {
  if (!S || !out) return DGSWE_E_INVALID;
  out[0] = S->nn;
  out[1] = S->ne;
  out[2] = S->ned;
  out[3] = S->nbnd;
  return DGSWE_OK;
}

}  // extern "C"
