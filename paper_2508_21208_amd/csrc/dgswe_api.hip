// C ABI of the gfx950 DG shallow-water step: solver lifetime for a batch
// of independent meshes (a single mesh is a batch of one), host<->device
// transfers (with each mesh's internal element permutation), the per-step
// launch sequence and HIP-event kernel timing.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "dgswe_internal.h"
#include "../../include/dgswe.h"

using namespace dgswe;

namespace {
thread_local std::string g_create_error = "no error";

enum KernelId { K_FORCING = 0, K_STAGE, K_PP2, K_RHS2, K_COUNT };
const char *kKernelNames[K_COUNT] = {"k_forcing", "k_stage", "k_pp2", "k_rhs2"};

// Host view of one member of a batch.
struct MemberHost {
  std::vector<int> perm;   // internal (member-local) -> caller element
  int ne = 0, nn = 0, ned = 0, nbnd = 0;
  bool cur_is_pp = true;   // its stored state is already post-processed
  bool holland = false;    // moving vortex (nodal forcing recomputed per stage)
};
}  // namespace

struct dgswe_solver {
  dgswe_params uprm{};
  Params prm{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  int nn = 0, ne = 0, ned = 0, nbnd = 0;
  std::vector<MemberHost> mh;
  std::vector<Member> mem;      // host mirror of the device member table
  Member *d_mem = nullptr;
  int *d_fblk_off = nullptr;
  double *d_man = nullptr;      // Manning n: per element [ne], then per member [nmem]
  float *d_manf = nullptr;
  std::vector<int> chunk_rec;   // host copy of the chunk records
  int *d_chunk_rec = nullptr;
  int nfblk = 0;                // forcing blocks of this step
  std::vector<void *> allocs;
  DevMesh m{};
  DevState s{};
  double *d_diag = nullptr;
  double *rb = nullptr;         // FP64 [3 nm][largest member] read-back buffer
  long long steps_enq = 0;
  int block = 256;              // workgroup size of the stage kernel
  int cur = 0;                  // buffer holding w^n
  int precision = DGSWE_FP64;
  int order = 1;                // polynomial degree p
  int nm = 3;                   // modes per variable
  std::string err = "no error";
  std::vector<double> stage_buf;
  std::vector<unsigned char> stage_raw;
  // kernel timing
  bool prof = false;
  struct Rec { int k; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double prof_ms[K_COUNT] = {};
  long long prof_n[K_COUNT] = {};
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
  // (shared by every member of a batch)
  if (!p) { msg = "params is NULL"; return false; }
  if (p->p != 1 && p->p != 2) { msg = "p must be 1 or 2"; return false; }
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


// Upload the member table and the forcing block offsets (after a forcing
// change).  Members with a moving vortex get ceil(nn / kBlock) blocks.
dgswe_status sync_members(dgswe_solver *S) {
  std::vector<int> off(S->mem.size() + 1, 0);
  for (size_t i = 0; i < S->mem.size(); ++i)
    off[i + 1] = off[i] + (S->mh[i].holland ? (S->mem[i].nn + kBlock - 1) / kBlock : 0);
  S->nfblk = off.back();
  hipError_t e = hipMemcpy(S->d_mem, S->mem.data(), S->mem.size() * sizeof(Member), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(S->d_fblk_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
  return DGSWE_OK;
}

dgswe_status check_member(dgswe_solver *S, int32_t member) {
  if (!S) return fail(nullptr, DGSWE_E_INVALID, "solver is NULL");
  if (member < 0 || member >= (int32_t)S->mh.size()) return fail(S, DGSWE_E_INVALID, "member out of range");
  return DGSWE_OK;
}

dgswe_status create_impl(int32_t n_members, const dgswe_mesh *meshes, const dgswe_params *prm, void *hip_stream,
                         dgswe_solver **out) {
  if (!out) return fail(nullptr, DGSWE_E_INVALID, "out is NULL");
  *out = nullptr;
  if (n_members < 1 || !meshes) return fail(nullptr, DGSWE_E_INVALID, "a batch needs at least one mesh");
  std::string msg;
  if (!validate_params(prm, msg)) return fail(nullptr, DGSWE_E_INVALID, msg);
  // chunk size and workgroup size of the stage kernel
  int chunk = 256, block = 256;
  if (const char *ev = std::getenv("DGSWE_CHUNK")) chunk = std::atoi(ev);
  if (const char *ev = std::getenv("DGSWE_BLOCK")) block = std::atoi(ev);
  if (!stage_block_ok(block) || chunk < 64 || chunk > block)
    return fail(nullptr, DGSWE_E_INVALID, "unsupported chunk/block configuration");
  std::vector<Prep> parts((size_t)n_members);
  long long ne_total = 0;
  for (int32_t i = 0; i < n_members; ++i) ne_total += meshes[i].n_elems > 0 ? meshes[i].n_elems : 0;
  if (ne_total > 0x7fffffffLL) return fail(nullptr, DGSWE_E_INVALID, "more than 2^31 - 1 elements in the batch");
  // host preprocessing of the meshes, several at a time (each thread owns
  // whole meshes; the first failing mesh in order is reported)
  std::vector<int> rcs((size_t)n_members, DGSWE_OK);
  std::vector<std::string> msgs((size_t)n_members);
  {
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const int nt = (int)std::min<unsigned>(hw, (unsigned)n_members);
    auto work = [&](int t0) {
      for (int i = t0; i < n_members; i += nt) {
        const dgswe_mesh &d = meshes[i];
        rcs[i] = prepare_mesh(d.n_nodes, d.node_xy, d.node_hb, d.n_elems, d.tri, d.n_bnd, d.bnd_nodes, d.bnd_type,
                              parts[i], msgs[i]);
        if (rcs[i] != DGSWE_OK) continue;
        build_chunks(parts[i], chunk);
        // (the p = 2 kernels use only the chunk ranges, not the halos)
        if (prm->p == 1 && (parts[i].nl_max > 2 * block || parts[i].ed_max > 2 * block)) {
          rcs[i] = DGSWE_E_MESH;
          msgs[i] = "element chunks have halos too large for the stage kernel";
        }
      }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work, t);
    work(0);
    for (auto &x : th) x.join();
  }
  for (int32_t i = 0; i < n_members; ++i)
    if (rcs[i] != DGSWE_OK) {
      msg = n_members > 1 ? "mesh " + std::to_string(i) + ": " + msgs[i] : msgs[i];
      return fail(nullptr, (dgswe_status)rcs[i], msg);
    }
  Prep P;
  merge_meshes(parts, P);
  if (prm->p == 2) p2_records(P);

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
  S->precision = prm->precision;
  S->order = prm->p;
  S->nm = prm->p == 2 ? 6 : 3;
  S->block = block;
  const bool mixed = S->precision == DGSWE_MIXED;
  S->nn = P.nn; S->ne = P.ne; S->ned = P.ned; S->nbnd = P.nbnd;
  Params &pp = S->prm;
  pp.g = prm->g; pp.rho0 = prm->rho0; pp.h0 = prm->h0; pp.cfl = prm->cfl;
  pp.dt_fixed = prm->dt_fixed; pp.dt_max = prm->dt_max;
  pp.limiter = prm->limiter ? 1 : 0; pp.wetdry = prm->wetdry ? 1 : 0;

  bool ok = true;
  auto chk = [&](hipError_t x) { if (x != hipSuccess) ok = false; };
  // members
  S->mh.resize((size_t)n_members);
  S->mem.resize((size_t)n_members);
  std::vector<int> chunk_member;
  chunk_member.reserve((size_t)P.nch);
  int e0 = 0, n0 = 0, c0 = 0, big = 0;
  for (int32_t i = 0; i < n_members; ++i) {
    MemberHost &h = S->mh[i];
    const Prep &q = parts[i];
    h.perm = q.perm;
    h.ne = q.ne; h.nn = q.nn; h.ned = q.ned; h.nbnd = q.nbnd;
    big = std::max(big, q.ne);
    Member f{};
    f.e0 = e0; f.ne = q.ne; f.n0 = n0; f.nn = q.nn; f.chunk0 = c0; f.nchunk = q.nch;
    f.holland = 0; f.n_tide = 0; f.tide_offset = 0.0; f.pn = 101300.0;
    S->mem[i] = f;
    for (int c = 0; c < q.nch; ++c) chunk_member.push_back(i);
    e0 += q.ne; n0 += q.nn; c0 += q.nch;
  }
  parts.clear();
  DevMesh &m = S->m;
  m.ne = P.ne; m.nn = P.nn; m.ned = P.ned;
  const size_t ne = P.ne, nn = P.nn;
  chk(upload(S, &m.area, P.area)); chk(upload(S, &m.inr2, P.inr2));
  chk(upload(S, &m.hbv, P.hbv));
  chk(upload(S, &m.el_nb, P.el_nb));
  chk(upload(S, &m.node_x, P.node_x)); chk(upload(S, &m.node_y, P.node_y));
  m.C = P.C; m.nch = P.nch; m.nl_max = P.nl_max; m.nm_max = P.nm_max; m.ed_max = P.ed_max;
  m.n2_max = P.n2_max;
  chunk_records(P, chunk_member, S->chunk_rec);
  chk(dev_alloc(S, &S->d_chunk_rec, S->chunk_rec.size()));
  chk(hipMemcpy(S->d_chunk_rec, S->chunk_rec.data(), S->chunk_rec.size() * sizeof(int), hipMemcpyHostToDevice));
  m.chunk_rec = S->d_chunk_rec;
  chk(dev_alloc(S, &S->d_man, ne + (size_t)n_members));
  chk(dev_alloc(S, &S->d_manf, ne + (size_t)n_members));
  m.man = S->d_man;
  m.manf = S->d_manf;
  chk(upload(S, &m.lgid, P.lgid)); chk(upload(S, &m.h2, P.h2));
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
  m.e2edge = nullptr;
  m.ed2a = m.ed2b = nullptr;
  m.hmean = nullptr;
  if (S->order == 2) {
    chk(upload(S, &m.e2edge, P.el_edge));
    chk(upload(S, &m.ed2a, P.ed2a)); chk(upload(S, &m.ed2b, P.ed2b));
    chk(upload(S, &m.hmean, P.hmean));
  }
  m.nmem = n_members;
  chk(dev_alloc(S, &S->d_mem, (size_t)n_members));
  chk(dev_alloc(S, &S->d_fblk_off, (size_t)n_members + 1));
  m.mem = S->d_mem;
  m.fblk_off = S->d_fblk_off;
  const size_t lds = stage_lds_bytes(m, S->precision);
  if (S->order == 1 && lds > 80 * 1024) {
    free_all(S);
    delete S;
    return fail(nullptr, DGSWE_E_MESH, "element chunks have halos too large for the LDS (" +
                                           std::to_string(lds) + " bytes)");
  }
  DevState &st = S->s;
  const size_t sb = state_bytes(ne, S->precision, S->order);
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
  chk(dev_alloc(S, &S->rb, 3 * (size_t)S->nm * (size_t)big));
  chk(dev_alloc(S, &st.nodal, 3 * nn)); chk(dev_alloc(S, &st.partial, 3 * (size_t)diag_blocks(big)));
  chk(dev_alloc(S, &st.ctrl, (size_t)n_members)); chk(dev_alloc(S, &S->d_diag, 4));
  if (!ok) {
    free_all(S);
    delete S;
    return fail(nullptr, DGSWE_E_NOMEM, "device allocation or upload failed");
  }
  // zero state and forcing, dt of the zero state
  chk(hipMemsetAsync(st.buf[0], 0, sb, S->stream));
  chk(hipMemsetAsync(st.nodal, 0, 3 * nn * sizeof(double), S->stream));
  chk(hipMemsetAsync(S->d_man, 0, (ne + (size_t)n_members) * sizeof(double), S->stream));
  chk(hipMemsetAsync(S->d_manf, 0, (ne + (size_t)n_members) * sizeof(float), S->stream));
  for (int32_t i = 0; i < n_members; ++i) {
    chk(launch_init_state(m, st, pp, st.buf[0], i, S->mem[i].e0, S->mem[i].ne, 0.0, 0, 0, S->precision,
                          S->order, S->stream));
  }
  chk(hipStreamSynchronize(S->stream));
  if (ok && sync_members(S) != DGSWE_OK) ok = false;
  S->cur = 0;
  if (!ok) {
    free_all(S);
    delete S;
    return fail(nullptr, DGSWE_E_DEVICE, "device initialisation failed");
  }
  *out = S;
  return DGSWE_OK;
}

dgswe_status set_state_impl(dgswe_solver *S, int32_t member, double t, const double *w, int32_t postprocess) {
  dgswe_status st0 = check_member(S, member);
  if (st0 != DGSWE_OK) return st0;
  if (!w) return fail(S, DGSWE_E_INVALID, "state is NULL");
  if (!std::isfinite(t)) return fail(S, DGSWE_E_INVALID, "time is not finite");
  MemberHost &h = S->mh[member];
  const Member &f = S->mem[member];
  const size_t ne = (size_t)h.ne, NE = (size_t)S->ne, nm = (size_t)S->nm;
  const bool mixed = S->precision == DGSWE_MIXED;
  // member-order image: zeta modes FP64, momentum modes FP64 or FP32
  S->stage_raw.resize(state_bytes(ne, S->precision, S->order));
  double *z = (double *)S->stage_raw.data();
  for (size_t j = 0; j < nm; ++j)
    for (size_t i = 0; i < ne; ++i) z[j * ne + i] = w[j * ne + (size_t)h.perm[i]];
  if (mixed) {
    float *q = (float *)(z + nm * ne);
    for (size_t j = 0; j < 2 * nm; ++j)
      for (size_t i = 0; i < ne; ++i) q[j * ne + i] = (float)w[(nm + j) * ne + (size_t)h.perm[i]];
  } else {
    double *q = z + nm * ne;
    for (size_t j = 0; j < 2 * nm; ++j)
      for (size_t i = 0; i < ne; ++i) q[j * ne + i] = w[(nm + j) * ne + (size_t)h.perm[i]];
  }
  // into the member's range of every mode array of the current buffer
  unsigned char *base = (unsigned char *)S->s.buf[S->cur];
  const size_t qs = mixed ? sizeof(float) : sizeof(double);
  hipError_t e = hipSuccess;
  for (size_t j = 0; j < nm && e == hipSuccess; ++j)
    e = hipMemcpyAsync(base + (j * NE + (size_t)f.e0) * sizeof(double), z + j * ne, ne * sizeof(double),
                       hipMemcpyHostToDevice, S->stream);
  const unsigned char *qsrc = (const unsigned char *)(z + nm * ne);
  unsigned char *qdst = base + nm * NE * sizeof(double);
  for (size_t j = 0; j < 2 * nm && e == hipSuccess; ++j)
    e = hipMemcpyAsync(qdst + (j * NE + (size_t)f.e0) * qs, qsrc + j * ne * qs, ne * qs, hipMemcpyHostToDevice,
                       S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "hipMemcpyAsync");
  // The stored state is post-processed by the first stage that reads it; a
  // state given without post-processing is marked as already done.
  h.cur_is_pp = postprocess == 0;
  e = launch_init_state(S->m, S->s, S->prm, S->s.buf[S->cur], member, f.e0, f.ne, t, (int)(S->steps_enq & 1),
                        postprocess ? 1 : 0, S->precision, S->order, S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "init kernel");
  e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "hipStreamSynchronize");
  return DGSWE_OK;
}

dgswe_status set_forcing_impl(dgswe_solver *S, int32_t member, const dgswe_forcing *fr) {
  dgswe_status st0 = check_member(S, member);
  if (st0 != DGSWE_OK) return st0;
  if (!fr) return fail(S, DGSWE_E_INVALID, "forcing is NULL");
  if (fr->n_tide < 0 || fr->n_tide > kMaxTide) return fail(S, DGSWE_E_INVALID, "at most 8 tidal constituents");
  if (fr->n_tide > 0 && (!fr->tide_amp || !fr->tide_omega || !fr->tide_phase))
    return fail(S, DGSWE_E_INVALID, "tidal arrays are NULL");
  if (fr->holland && !(fr->rmax > 0 && fr->B > 0 && fr->rho_air > 0))
    return fail(S, DGSWE_E_INVALID, "Holland rmax, B and rho_air must be positive");
  MemberHost &h = S->mh[member];
  Member &f = S->mem[member];
  const size_t ne = (size_t)h.ne, nn = (size_t)h.nn, NN = (size_t)S->nn;
  hipError_t e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "hipStreamSynchronize");
  f.n_tide = fr->n_tide;
  for (int i = 0; i < kMaxTide; ++i) {
    const bool on = i < fr->n_tide;
    f.tide_amp[i] = on ? fr->tide_amp[i] : 0.0;
    f.tide_omega[i] = on ? fr->tide_omega[i] : 0.0;
    f.tide_phase[i] = on ? fr->tide_phase[i] : 0.0;
  }
  f.tide_offset = fr->tide_offset;
  f.holland = fr->holland ? 1 : 0;
  f.x0 = fr->x0; f.y0 = fr->y0; f.vx = fr->vx; f.vy = fr->vy; f.dp = fr->dp; f.pn = fr->pn;
  f.rmax = fr->rmax; f.B = fr->B; f.rho_air = fr->rho_air; f.coriolis_f = fr->coriolis_f;
  f.wind_factor = fr->wind_factor;
  // Manning n: the member's per-element range, or its uniform slot after
  // the per-element values; its chunk records point at the one that applies
  const bool per_elem = fr->manning_n_elem != nullptr;
  if (per_elem) {
    std::vector<double> tmp(ne);
    std::vector<float> tf(ne);
    for (size_t i = 0; i < ne; ++i) {
      tmp[i] = fr->manning_n_elem[h.perm[i]];
      tf[i] = (float)tmp[i];
    }
    e = hipMemcpy(S->d_man + f.e0, tmp.data(), ne * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(S->d_manf + f.e0, tf.data(), ne * sizeof(float), hipMemcpyHostToDevice);
  } else {
    const float nf = (float)fr->manning_n;
    e = hipMemcpy(S->d_man + S->ne + member, &fr->manning_n, sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(S->d_manf + S->ne + member, &nf, sizeof(float), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
  for (int c = f.chunk0; c < f.chunk0 + f.nchunk; ++c) {
    int *r = &S->chunk_rec[(size_t)c * kChunkRec];
    r[11] = per_elem ? r[0] : S->ne + member;
    r[12] = per_elem ? 1 : 0;
  }
  e = hipMemcpy(S->d_chunk_rec + (size_t)f.chunk0 * kChunkRec, &S->chunk_rec[(size_t)f.chunk0 * kChunkRec],
                (size_t)f.nchunk * kChunkRec * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
  h.holland = fr->holland != 0;
  if (!h.holland) {
    // static fields of this member's nodes: (tau_x, tau_y) pairs, then p_a
    std::vector<double> tau(2 * nn, 0.0), pa(nn, 0.0);
    for (size_t i = 0; i < nn; ++i) {
      if (fr->wind_tau) { tau[2 * i] = fr->wind_tau[2 * i]; tau[2 * i + 1] = fr->wind_tau[2 * i + 1]; }
      if (fr->patm) pa[i] = fr->patm[i];
    }
    e = hipMemcpy(S->s.nodal + 2 * (size_t)f.n0, tau.data(), 2 * nn * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(S->s.nodal + 2 * NN + (size_t)f.n0, pa.data(), nn * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
  }
  return sync_members(S);
}

dgswe_status read_state_impl(dgswe_solver *S, int32_t member, double *w_out, dgswe_diag *d) {
  dgswe_status st0 = check_member(S, member);
  if (st0 != DGSWE_OK) return st0;
  hipError_t e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "hipStreamSynchronize");
  MemberHost &h = S->mh[member];
  const Member &f = S->mem[member];
  const size_t ne = (size_t)h.ne;
  if (w_out) {
    // the state at the boundary is post-processed, FP64
    const size_t nv = 3 * (size_t)S->nm;
    if (S->order == 2)
      e = launch_post_only2(S->m, S->prm, S->s.buf[S->cur], h.cur_is_pp ? 0 : 1, f.e0, f.ne, S->rb, S->precision,
                            S->stream);
    else
      e = launch_post_only(S->m, S->prm, S->s.buf[S->cur], h.cur_is_pp ? 0 : 1, f.e0, f.ne, S->rb, S->precision,
                           S->stream);
    if (e != hipSuccess) return hip_fail(S, e, "post-processing kernel");
    S->stage_buf.resize(nv * ne);
    e = hipMemcpyAsync(S->stage_buf.data(), S->rb, nv * ne * sizeof(double), hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
    for (size_t j = 0; j < nv; ++j)
      for (size_t i = 0; i < ne; ++i) w_out[j * ne + (size_t)h.perm[i]] = S->stage_buf[j * ne + i];
  }
  Ctrl c{};
  if (d) {
    e = launch_diag(S->m, S->s, S->prm, S->s.buf[S->cur], f.e0, f.ne, S->d_diag, S->stream);
    if (e != hipSuccess) return hip_fail(S, e, "diagnostics kernel");
    double out4[4];
    e = hipMemcpyAsync(out4, S->d_diag, sizeof out4, hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
    d->mass = out4[0];
    d->volume = out4[1];
    d->n_wet = (int32_t)out4[2];
    d->n_dry = (int32_t)(h.ne - d->n_wet);
  }
  e = hipMemcpy(&c, S->s.ctrl + member, sizeof c, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
  if (d) {
    d->t = c.t[S->steps_enq & 1];
    d->dt_last = c.dt_last;
    d->steps = c.steps;
  }
  if (c.status == DGSWE_E_NONFINITE) return fail(S, DGSWE_E_NONFINITE, "non-finite value in the state");
  if (c.status == DGSWE_E_ALLDRY) return fail(S, DGSWE_E_ALLDRY, "no wet element defines the CFL time step");
  if (c.status) return fail(S, DGSWE_E_DEVICE, "device status " + std::to_string(c.status));
  return DGSWE_OK;
}

dgswe_status single(dgswe_solver *S) {
  if (!S) return fail(nullptr, DGSWE_E_INVALID, "solver is NULL");
  if (S->mh.size() != 1) return fail(S, DGSWE_E_INVALID, "a batch of several meshes needs the dgswe_member_* calls");
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
  dgswe_mesh d{n_nodes, node_xy, node_hb, n_elems, tri, n_bnd, bnd_nodes, bnd_type};
  return create_impl(1, &d, prm, hip_stream, out);
}

dgswe_status dgswe_create_batch(int32_t n_meshes, const dgswe_mesh *meshes, const dgswe_params *prm,
                                void *hip_stream, dgswe_solver **out) {
  return create_impl(n_meshes, meshes, prm, hip_stream, out);
}

dgswe_status dgswe_set_state(dgswe_solver *S, double t, const double *w, int32_t postprocess) {
  dgswe_status st = single(S);
  return st != DGSWE_OK ? st : set_state_impl(S, 0, t, w, postprocess);
}

dgswe_status dgswe_member_set_state(dgswe_solver *S, int32_t member, double t, const double *w,
                                    int32_t postprocess) {
  return set_state_impl(S, member, t, w, postprocess);
}

dgswe_status dgswe_set_forcing(dgswe_solver *S, const dgswe_forcing *f) {
  dgswe_status st = single(S);
  return st != DGSWE_OK ? st : set_forcing_impl(S, 0, f);
}

dgswe_status dgswe_member_set_forcing(dgswe_solver *S, int32_t member, const dgswe_forcing *f) {
  return set_forcing_impl(S, member, f);
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
    hipError_t e = hipSuccess;
    for (int stage = 0; stage < 2 && e == hipSuccess; ++stage) {
      if (S->nfblk > 0) {
        Timed t(S, K_FORCING);
        e = launch_forcing(m, st, p, S->nfblk, slot, stage, S->stream);
      }
      if (e != hipSuccess) break;
      if (S->order == 2) {
        // records of the stage input: w^n's go to wpp (the RK base of the
        // second stage), the first stage result's to the buffer of w^n,
        // which is no longer read
        void *rec = stage == 0 ? st.wpp : st.buf[cur];
        {
          Timed t(S, K_PP2);
          e = launch_pp2(m, st, p, stage == 0 ? st.buf[cur] : st.buf[s1], rec, slot, stage, S->precision, S->stream);
        }
        if (e != hipSuccess) break;
        Timed t(S, K_RHS2);
        e = launch_rhs2(m, st, p, rec, stage == 0 ? nullptr : st.wpp, stage == 0 ? st.buf[s1] : st.buf[nx], slot,
                        stage, stage == 0 ? 0 : want_dt, S->precision, S->stream);
        continue;
      }
      Timed t(S, K_STAGE);
      if (stage == 0)
        e = launch_stage(m, st, p, st.buf[cur], nullptr, st.buf[s1], st.wpp, slot, 0, 0, S->block, S->precision,
                         S->stream);
      else
        e = launch_stage(m, st, p, st.buf[s1], st.wpp, st.buf[nx], nullptr, slot, 1, want_dt, S->block,
                         S->precision, S->stream);
    }
    if (e != hipSuccess) return hip_fail(S, e, "kernel launch");
    S->cur = nx;
    for (MemberHost &h : S->mh) h.cur_is_pp = false;
    S->steps_enq += 1;
  }
  return DGSWE_OK;
}

dgswe_status dgswe_read_state(dgswe_solver *S, double *w_out, dgswe_diag *d) {
  dgswe_status st = single(S);
  return st != DGSWE_OK ? st : read_state_impl(S, 0, w_out, d);
}

dgswe_status dgswe_member_read_state(dgswe_solver *S, int32_t member, double *w_out, dgswe_diag *d) {
  return read_state_impl(S, member, w_out, d);
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

dgswe_status dgswe_member_info(const dgswe_solver *S, int32_t member, int64_t out[4]) {
  if (!S || !out || member < 0 || member >= (int32_t)S->mh.size()) return DGSWE_E_INVALID;
  const MemberHost &h = S->mh[member];
  out[0] = h.nn;
  out[1] = h.ne;
  out[2] = h.ned;
  out[3] = h.nbnd;
  return DGSWE_OK;
}

int32_t dgswe_member_count(const dgswe_solver *S) { return S ? (int32_t)S->mh.size() : 0; }

}  // extern "C"
