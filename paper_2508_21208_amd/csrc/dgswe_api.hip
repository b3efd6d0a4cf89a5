// C ABI of the gfx950 DG shallow-water step: solver lifetime for a batch
// of independent meshes (a single mesh is a batch of one) or a serving pool
// whose members join and leave between steps, host<->device transfers (with
// each mesh's internal element permutation), the per-step launch sequence
// and HIP-event kernel timing.
//
// Device memory layout.  Every per-element, per-node, per-local-element,
// per-local-edge, ring-2 and per-edge array of the kernels is one arena of
// fixed capacity; a member occupies one contiguous range of each arena
// (first fit, freed ranges coalesce), with every stored id shifted into the
// arena's index space.  Structure-of-arrays rows have the arena capacity as
// their stride.  The chunk records list the chunks of the active members
// only and are rebuilt when a member joins or leaves, so a step launches one
// grid over exactly the active work.  A batch is a pool sized to its meshes.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "dgswe_internal.h"
#include "../../include/dgswe.h"

using namespace dgswe;

namespace dgswe {
// Shu-Osher forms: SSPRK(2,2) and SSPRK(3,3) (Shu and Osher 1988), and the
// optimal second-order SSPRK(s,2) (s - 1 forward-Euler steps of dt/(s-1),
// then the average with w^n weighted 1/s), whose SSP coefficient s - 1
// allows a CFL number s - 1 times that of a single Euler step.
int rk_stages(int rk, StageCoef out[5]) {
  if (rk == 22) {
    out[0] = {0.0, 1.0, 1.0, 0.0, 0};
    out[1] = {0.5, 0.5, 1.0, 1.0, 1};
    return 2;
  }
  if (rk == 33) {
    out[0] = {0.0, 1.0, 1.0, 0.0, 0};
    out[1] = {0.75, 0.25, 1.0, 1.0, 0};
    out[2] = {1.0 / 3.0, 2.0 / 3.0, 1.0, 0.5, 1};
    return 3;
  }
  if (rk == 32 || rk == 42 || rk == 52) {
    const int s = rk / 10;
    const double h = 1.0 / (s - 1);
    for (int i = 0; i < s - 1; ++i) out[i] = {0.0, 1.0, h, i * h, 0};
    out[s - 1] = {1.0 / s, (double)(s - 1) / s, h, 1.0, 1};
    return s;
  }
  return 0;
}
}  // namespace dgswe

namespace {
thread_local std::string g_create_error = "no error";

// Scratch of dgswe_member_read_state_device, the read-back for callers that
// cannot allocate: the diagnostics' per-block partial sums of a member of
// up to DGSWE_NOALLOC_MAX_ELEMS elements (3 per block of 256 elements)
// followed by their three totals, 1.5 MiB.  Each GPU holds its own copy
// until the process ends.  Host code never passes the array's name to a
// kernel or a copy: it uses the device address hipGetSymbolAddress gives
// for the device, looked up once per device with that device current.
constexpr int kNoAllocBlocks = DGSWE_NOALLOC_MAX_ELEMS / 256;
constexpr size_t kNoAllocDoubles = 3 * (size_t)kNoAllocBlocks + 4;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on `device`
hipError_t scratch_on(int device, double **out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *addr = nullptr;
    e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!addr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = (double *)addr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

enum KernelId { K_FORCING = 0, K_STAGE, K_PP2, K_RHS2, K_VBOUNDS, K_STAGE12, K_STAGE1PP2, K_COUNT };
const char *kKernelNames[K_COUNT] = {"k_forcing", "k_stage",   "k_pp2",      "k_rhs2",
                                     "k_vbounds", "k_stage12", "k_stage1pp2"};


// First-fit allocator over [0, cap) with coalescing of freed ranges.
class Arena {
 public:
  void init(long long cap) {
    cap_ = cap;
    free_.clear();
    if (cap > 0) free_[0] = cap;
  }
  bool take(long long n, long long &off) {
    if (n <= 0) { off = 0; return true; }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      off = it->first;
      const long long rest = it->second - n;
      free_.erase(it);
      if (rest > 0) free_[off + n] = rest;
      return true;
    }
    return false;
  }
  void give(long long off, long long n) {
    if (n <= 0) return;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  long long cap() const { return cap_; }
  long long free_total() const {
    long long t = 0;
    for (auto &kv : free_) t += kv.second;
    return t;
  }

 private:
  long long cap_ = 0;
  std::map<long long, long long> free_;
};

// arenas: elements, nodes, local elements (chunk + ring 1 of each chunk),
// chunk-local edges, ring-2 entries (+1 sentinel per member)
enum ArenaId { A_ELEM = 0, A_NODE, A_LOC, A_LEDGE, A_RING2, A_COUNT };

// Host view of one member (slot).
struct MemberHost {
  bool active = false;
  std::vector<int> perm;   // internal (member-local) -> caller element
  int ne = 0, nn = 0, ned = 0, nbnd = 0;
  bool cur_is_pp = true;   // its stored state is already post-processed
  bool holland = false;    // moving vortex (nodal forcing recomputed per stage)
  bool man_elem = false;   // per-element Manning n (else the member's uniform slot)
  long long off[A_COUNT] = {}, len[A_COUNT] = {};
  // chunks relative to the member's ranges: c0, cc, n1, h2o, n2, leo, ne_loc, lo
  std::vector<int> chunks;
  int nl_max = 0, nm_max = 0, ed_max = 0, n2_max = 0, C = 0;
};
constexpr int kChunkHost = 8;
}  // namespace

// A mesh after host preprocessing, not yet on the device.
struct dgswe_prepared {
  dgswe::Prep P;
  int order = 1;
};

struct dgswe_solver {
  dgswe_params uprm{};
  Params prm{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  int nn = 0, ne = 0, ned = 0, nbnd = 0;   // sums over the active members
  Arena arena[A_COUNT];
  int chunk_cap = 0;            // capacity of the chunk-record array
  bool is_pool = false;         // members may join and leave
  // the nodal forcing buffer holds the forcing at the time the next step
  // starts (the last stage of the previous step ran at t + 1.0 dt, which is
  // that time bit for bit); cleared by anything that changes times or fields
  bool forcing_fresh = false;
  bool forcing_every_stage = false;  // DGSWE_FORCING_EVERY_STAGE=1: never reuse
  size_t dev_bytes = 0;         // device memory held
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
  double *rb = nullptr;         // FP64 [3 nm][rb_elems] read-back buffer (grown on demand)
  size_t rb_elems = 0;
  long long steps_enq = 0;
  int block = 256;              // workgroup size of the stage kernel
  int cur = 0;                  // buffer holding w^n
  int precision = DGSWE_FP64;
  int order = 1;                // polynomial degree p
  int nm = 3;                   // modes per variable
  std::string err = "no error";
  // pinned host staging for state uploads and read-backs (grown on demand)
  void *stage_in = nullptr, *stage_out = nullptr;
  size_t stage_in_bytes = 0, stage_out_bytes = 0;
  // step graphs: G steps captured once per (buffer rotation, step parity)
  // and replayed; dropped whenever the launch tables change
  int graph_steps = 0;
  bool capturing = false;
  hipGraphExec_t graph[6] = {};
  // graphs of dgswe_step_pair (this solver the p = 1 side): per (rotation,
  // parity) of both solvers, for the partner with id pair_id as it was at
  // generation pair_gen
  hipGraphExec_t pair_graph[36] = {};
  unsigned long long id = 0;       // unique per solver of the process
  unsigned long long pair_id = 0;
  unsigned gen = 0;                // bumped whenever this solver's graphs are dropped
  unsigned pair_gen = 0;
  hipEvent_t pair_ev = nullptr;    // orders this solver's stream around dgswe_step_pair
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
  if (e == hipSuccess) {
    S->allocs.push_back(q);
    S->dev_bytes += n * sizeof(T) + 16;
  }
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

void drop_pair_graphs(dgswe_solver *S) {
  for (hipGraphExec_t &g : S->pair_graph) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  S->pair_id = 0;
}

void drop_graphs(dgswe_solver *S) {
  S->forcing_fresh = false;
  ++S->gen;
  for (hipGraphExec_t &g : S->graph) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  drop_pair_graphs(S);
}

void free_all(dgswe_solver *S) {
  drop_graphs(S);
  if (S->pair_ev) (void)hipEventDestroy(S->pair_ev);
  S->pair_ev = nullptr;
  if (S->stage_in) (void)hipHostFree(S->stage_in);
  if (S->stage_out) (void)hipHostFree(S->stage_out);
  S->stage_in = S->stage_out = nullptr;
  S->stage_in_bytes = S->stage_out_bytes = 0;
  for (void *p : S->allocs) (void)hipFree(p);
  S->allocs.clear();
  if (S->rb) (void)hipFree(S->rb);
  S->rb = nullptr;
  S->rb_elems = 0;
  for (auto &r : S->recs) { S->pool.push_back(r.a); S->pool.push_back(r.b); }
  S->recs.clear();
  for (hipEvent_t ev : S->pool) (void)hipEventDestroy(ev);
  S->pool.clear();
  if (S->own_stream && S->stream) (void)hipStreamDestroy(S->stream);
  S->stream = nullptr;
}

// A pinned host buffer of at least `bytes` (kept and grown across calls).
hipError_t pinned(void *&buf, size_t &have, size_t bytes) {
  if (have >= bytes) return hipSuccess;
  if (buf) (void)hipHostFree(buf);
  buf = nullptr;
  have = 0;
  const hipError_t e = hipHostMalloc(&buf, bytes, hipHostMallocDefault);
  if (e == hipSuccess) have = bytes;
  return e;
}

// f(j) for every plane j < nplanes of a state of ne elements; large states
// spread the planes over host threads (the permutation between the caller's
// and the internal element order is a gather over the whole plane).
template <class F>
void for_planes(size_t nplanes, size_t ne, F &&f) {
  const size_t hw = std::max(1u, std::thread::hardware_concurrency());
  const size_t nt = ne < 65536 ? 1 : std::min({nplanes, hw, (size_t)16});
  if (nt > 1) {
    std::vector<std::thread> th;
    try {
      for (size_t t = 0; t < nt; ++t)
        th.emplace_back([&f, t, nt, nplanes] {
          for (size_t j = t; j < nplanes; j += nt) f(j);
        });
    } catch (...) {
      // no threads to be had: the planes not started run here (each plane
      // is written by one thread only)
      const size_t started = th.size();
      for (std::thread &x : th) x.join();
      for (size_t t = started; t < nt; ++t)
        for (size_t j = t; j < nplanes; j += nt) f(j);
      return;
    }
    for (std::thread &x : th) x.join();
    return;
  }
  for (size_t j = 0; j < nplanes; ++j) f(j);
}

bool validate_params(const dgswe_params *p, std::string &msg) {
  // (shared by every member of a batch)
  if (!p) { msg = "params is NULL"; return false; }
  if (p->p != 1 && p->p != 2) { msg = "p must be 1 or 2"; return false; }
  StageCoef sc[5];
  if (rk_stages(p->rk, sc) == 0) { msg = "rk must be 22, 33, 32, 42 or 52"; return false; }
  if (p->flux != 0 && p->flux != 1) { msg = "flux must be 0 (LLF) or 1 (Roe)"; return false; }
  if (p->chunk != 0 && (p->chunk < 64 || p->chunk > 256)) { msg = "chunk must be 0 or in [64, 256]"; return false; }
  if (p->waves < 0 || p->waves > 4) { msg = "waves must be in [0, 4]"; return false; }
  if (p->persistent < 0 || p->persistent > 8) { msg = "persistent must be in [0, 8]"; return false; }
  if (p->limiter < 0 || p->limiter > 2) { msg = "limiter must be 0, 1 or 2"; return false; }
  if (p->limiter == 2 && p->p != 1) { msg = "the vertex-based limiter (limiter = 2) needs p = 1"; return false; }
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
    if (!S->prof || S->capturing) return;
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
    if (!S->prof || S->capturing) return;
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
  if (!S->mh[(size_t)member].active) return fail(S, DGSWE_E_INVALID, "member slot is empty");
  return DGSWE_OK;
}

// Whether the chunks of P fit the p = 1 stage kernel: at most 2 x block
// local elements (chunk + ring 1) and local edges per chunk (each lane
// holds two), and the chunk's LDS within kStageLdsMax.
bool chunks_fit(const Prep &P, int precision, int block) {
  if (P.nl_max > 2 * block || P.ed_max > 2 * block) return false;
  DevMesh t{};
  t.nl_max = P.nl_max; t.nm_max = P.nm_max; t.ed_max = P.ed_max; t.n2_max = P.n2_max; t.C = P.C;
  return stage_lds_bytes(t, precision) <= kStageLdsMax;
}

// Host preprocessing of one mesh for the solver's order and chunking.  A
// mesh whose chunks of `chunk` elements have halos too large for the stage
// kernel is chunked again with 32 fewer elements per chunk, and so on: at
// 64 every mesh fits (at most 256 local elements, 192 local edges, about
// 50 KB of LDS at p = 1), so no valid mesh is refused.  The p = 2 kernels
// take a chunk's local edges (two per lane) but not its halo elements.
//
// chunk = 0 (the default) at p = 1: the largest chunk size of at most 256 -
// down to 160, in steps of 8 - whose LDS lets the most workgroups share a
// compute unit (kStageWgPerCu: 3 in FP64, 4 in mixed precision, the number
// the stage kernel's registers allow), else 256.  On the 4M hurricane mesh
// that is 232 in FP64 (3 workgroups per CU instead of 2 at 256: 373 against
// 415 us per stage launch) and 256 in mixed precision.  At p = 2: 256.
int auto_chunk(Prep &P, int order, int precision, int block) {
  if (order != 1) return 256;
  const int want = precision == DGSWE_MIXED ? kStageWgPerCuMixed : kStageWgPerCuFp64;
  const size_t cap = kLdsPerCu / (size_t)want - kLdsSlack;
  for (int c = 256; c >= 160; c -= 8) {
    build_chunks(P, c);
    if (!chunks_fit(P, precision, block)) continue;
    DevMesh t{};
    t.nl_max = P.nl_max; t.nm_max = P.nm_max; t.ed_max = P.ed_max; t.n2_max = P.n2_max; t.C = P.C;
    if (stage_lds_bytes(t, precision) <= cap) return c;
  }
  return 256;
}

int prep_one(const dgswe_mesh &d, int order, int precision, int chunk, int block, Prep &P, std::string &msg) {
  int rc = prepare_mesh(d.n_nodes, d.node_xy, d.node_hb, d.n_elems, d.tri, d.n_bnd, d.bnd_nodes, d.bnd_type, P, msg);
  if (rc != DGSWE_OK) return rc;
  if (chunk == 0) chunk = std::min(auto_chunk(P, order, precision, block), block);
  for (int c = chunk;; c = std::max(64, c - 32)) {
    build_chunks(P, c);
    if (order == 2 ? P.ed_max <= 2 * block : chunks_fit(P, precision, block)) break;
    if (c == 64) {
      msg = "element chunks have halos too large for the stage kernel";
      return DGSWE_E_MESH;
    }
  }
  if (order == 2) p2_records(P);
  return DGSWE_OK;
}

// entries each arena needs for a prepared mesh
void arena_need(const Prep &q, int order, long long need[A_COUNT]) {
  need[A_ELEM] = q.ne;
  need[A_NODE] = q.nn;
  need[A_LOC] = q.lo_off[q.nch];
  need[A_LEDGE] = q.le_off[q.nch];
  need[A_RING2] = (long long)q.h2_off[q.nch] + 1;
}

bool chunk_config(const dgswe_params *prm, int &chunk, int &block) {
  chunk = prm && prm->chunk > 0 ? prm->chunk : 0;  // 0: chosen per mesh (auto_chunk)
  block = 256;
  if (const char *ev = std::getenv("DGSWE_CHUNK")) chunk = std::atoi(ev);
  if (const char *ev = std::getenv("DGSWE_BLOCK")) block = std::atoi(ev);
  return stage_block_ok(block) && (chunk == 0 || (chunk >= 64 && chunk <= block));
}

// Device arrays for the given arena capacities, `slots` members and
// `chunk_cap` chunk records.
dgswe_status alloc_solver(const dgswe_params *prm, int block, const long long cap[A_COUNT], int chunk_cap, int slots,
                          void *hip_stream, dgswe_solver **out) {
  dgswe_solver *S = new (std::nothrow) dgswe_solver();
  if (!S) return fail(nullptr, DGSWE_E_NOMEM, "host allocation failed");
  static std::atomic<unsigned long long> next_id{1};
  S->id = next_id++;
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
  if (const char *ev = std::getenv("DGSWE_FORCING_EVERY_STAGE")) S->forcing_every_stage = std::atoi(ev) != 0;
  // measured alternatives (see Params)
  {
    const char *ev = std::getenv("DGSWE_RHS2_MFMA");
    S->prm.rhs2_mfma = ev && std::atoi(ev) == 1;
    ev = std::getenv("DGSWE_PAIR_SPLIT");
    S->prm.pair_split = !(ev && std::atoi(ev) == 0);
  }
  S->precision = prm->precision;
  S->order = prm->p;
  S->nm = prm->p == 2 ? 6 : 3;
  S->block = block;
  const bool mixed = S->precision == DGSWE_MIXED;
  Params &pp = S->prm;
  pp.g = prm->g; pp.rho0 = prm->rho0; pp.h0 = prm->h0; pp.cfl = prm->cfl;
  pp.dt_fixed = prm->dt_fixed; pp.dt_max = prm->dt_max;
  pp.limiter = prm->limiter; pp.wetdry = prm->wetdry ? 1 : 0;
  pp.flux = prm->flux;
  pp.waves = prm->waves;
  pp.persistent = prm->persistent;
  pp.n_cu = 0;
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, S->device) == hipSuccess) pp.n_cu = ncu;
  }
  for (int a = 0; a < A_COUNT; ++a) S->arena[a].init(cap[a]);
  S->chunk_cap = chunk_cap;
  S->mh.resize((size_t)slots);
  S->mem.assign((size_t)slots, Member{});
  for (Member &f : S->mem) f.pn = 101300.0;

  bool ok = true;
  auto chk = [&](hipError_t x) { if (x != hipSuccess) ok = false; };
  const size_t E = (size_t)std::max(1LL, cap[A_ELEM]), N = (size_t)std::max(1LL, cap[A_NODE]);
  const size_t L = (size_t)std::max(1LL, cap[A_LOC]), LE = (size_t)std::max(1LL, cap[A_LEDGE]);
  const size_t R2 = (size_t)std::max(1LL, cap[A_RING2]);
  DevMesh &m = S->m;
  m = DevMesh{};
  m.ne = (int)E; m.nn = (int)N; m.ned = 0;
  auto al = [&](auto **ptr, size_t n) {
    using T = std::remove_const_t<std::remove_pointer_t<std::remove_reference_t<decltype(*ptr)>>>;
    T *q = nullptr;
    chk(dev_alloc(S, &q, n));
    *ptr = q;
  };
  al(&m.area, E); al(&m.inr2, E); al(&m.hbv, 3 * E); al(&m.el_nb, 3 * E); al(&m.perm, E);
  al(&m.node_x, N); al(&m.node_y, N);
  al(&m.eai, E); al(&m.enode, E);
  if (mixed) { al(&m.egf, E); al(&m.le_f, LE); }
  else { al(&m.eg1, E); al(&m.eg2, E); al(&m.le_a, LE); al(&m.le_b, LE); }
  al(&m.lgid, L); al(&m.lhb01, L); al(&m.lhb2, L); al(&m.lnb, L);
  al(&m.h2, R2);
  if (S->order == 2) { al(&m.hmean, E); al(&m.le_g, LE); }
  if (pp.limiter == 2 && 3 * E > 0x7fffffffULL) ok = false;  // incidence positions are int
  if (pp.limiter == 2) { al(&m.nd_rng, N); al(&m.nd_el, 3 * E); al(&m.evb, E); }
  chk(dev_alloc(S, &S->d_chunk_rec, (size_t)std::max(1, chunk_cap) * kChunkRec));
  m.chunk_rec = S->d_chunk_rec;
  chk(dev_alloc(S, &S->d_man, E + (size_t)slots));
  chk(dev_alloc(S, &S->d_manf, E + (size_t)slots));
  m.man = S->d_man;
  m.manf = S->d_manf;
  m.C = 0; m.nch = 0; m.nl_max = m.nm_max = m.ed_max = m.n2_max = 1;
  m.nmem = slots;
  chk(dev_alloc(S, &S->d_mem, (size_t)slots));
  chk(dev_alloc(S, &S->d_fblk_off, (size_t)slots + 1));
  m.mem = S->d_mem;
  m.fblk_off = S->d_fblk_off;
  DevState &st = S->s;
  const size_t sb = state_bytes(E, S->precision, S->order);
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
  chk(dev_alloc(S, &st.nodal, 3 * N)); chk(dev_alloc(S, &st.partial, 3 * (size_t)diag_blocks((int)E)));
  chk(dev_alloc(S, &st.ctrl, (size_t)slots)); chk(dev_alloc(S, &S->d_diag, 4));
  if (pp.limiter == 2) chk(dev_alloc(S, &st.vb, 6 * N));
  if (ok) {
    // ring-2 entries are read clamped, so every entry is a valid element id
    chk(hipMemset((void *)m.h2, 0, R2 * sizeof(int)));
    chk(hipMemset(S->d_man, 0, (E + (size_t)slots) * sizeof(double)));
    chk(hipMemset(S->d_manf, 0, (E + (size_t)slots) * sizeof(float)));
    // node ranges of unused node slots: empty; element ids: valid
    if (pp.limiter == 2) {
      chk(hipMemset((void *)m.nd_rng, 0, N * sizeof(int2)));
      chk(hipMemset((void *)m.nd_el, 0, 3 * E * sizeof(int)));
    }
  }
  if (!ok) {
    free_all(S);
    delete S;
    return fail(nullptr, DGSWE_E_NOMEM, "device allocation failed");
  }
  S->cur = 0;
  *out = S;
  return DGSWE_OK;
}

template <class T>
hipError_t put(const T *dst, size_t off, const T *src, size_t n) {
  if (n == 0) return hipSuccess;
  return hipMemcpy((T *)dst + off, src, n * sizeof(T), hipMemcpyHostToDevice);
}

// Place a prepared mesh into free ranges of every arena as member `slot`
// (state zero at t = 0, no forcing).  DGSWE_E_NOMEM when some arena has no
// room; the solver is then unchanged.
// Give a member's store ranges back and empty its slot (no table rebuild).
void release_slot(dgswe_solver *S, int slot) {
  MemberHost &h = S->mh[(size_t)slot];
  for (int a = 0; a < A_COUNT; ++a) S->arena[a].give(h.off[a], h.len[a]);
  h = MemberHost{};
}

dgswe_status place_member(dgswe_solver *S, int slot, const Prep &q) {
  long long need[A_COUNT], off[A_COUNT];
  arena_need(q, S->order, need);
  for (int a = 0; a < A_COUNT; ++a) {
    if (!S->arena[a].take(need[a], off[a])) {
      for (int b = 0; b < a; ++b) S->arena[b].give(off[b], need[b]);
      return fail(S, DGSWE_E_NOMEM, "no room for a mesh of " + std::to_string(q.ne) + " elements (" +
                                        std::to_string(S->arena[A_ELEM].free_total()) + " elements free)");
    }
  }
  if (S->order == 1) {
    DevMesh t = S->m;
    t.nl_max = std::max(t.nl_max, q.nl_max); t.nm_max = std::max(t.nm_max, q.nm_max);
    t.ed_max = std::max(t.ed_max, q.ed_max); t.n2_max = std::max(t.n2_max, q.n2_max);
    t.C = std::max(t.C, q.C);
    if (stage_lds_bytes(t, S->precision) > kStageLdsMax) {
      for (int a = 0; a < A_COUNT; ++a) S->arena[a].give(off[a], need[a]);
      return fail(S, DGSWE_E_MESH, "element chunks have halos too large for the LDS");
    }
  }
  const bool mixed = S->precision == DGSWE_MIXED;
  const DevMesh &m = S->m;
  const size_t E = (size_t)m.ne, N = (size_t)m.nn, ne = (size_t)q.ne, nn = (size_t)q.nn;
  const int e0 = (int)off[A_ELEM], n0 = (int)off[A_NODE];
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  chk(put(m.area, e0, q.area.data(), ne));
  chk(put(m.inr2, e0, q.inr2.data(), ne));
  chk(put(m.perm, e0, q.perm.data(), ne));
  {
    std::vector<int> nb(ne);
    for (size_t k = 0; k < 3; ++k) {
      chk(put(m.hbv, k * E + e0, q.hbv.data() + k * ne, ne));
      for (size_t i = 0; i < ne; ++i) {
        const int f = q.el_nb[k * ne + i];
        nb[i] = f < 0 ? -1 : f + e0;
      }
      chk(put(m.el_nb, k * E + e0, nb.data(), ne));
    }
  }
  chk(put(m.node_x, n0, q.node_x.data(), nn));
  chk(put(m.node_y, n0, q.node_y.data(), nn));
  chk(put(m.eai, e0, q.eai.data(), ne));
  {
    std::vector<int4> en(q.enode);
    for (int4 &v : en) { v.x += n0; v.y += n0; v.z += n0; }
    chk(put(m.enode, e0, en.data(), ne));
  }
  if (S->prm.limiter == 2) {
    // node -> element incidence for the vertex-based limiter: range slots
    // in order of first appearance in the element list (unused nodes
    // last), the member's 3 ne entries at positions [3 e0, 3 e0 + 3 ne)
    std::vector<int> slot_of(nn, -1);
    int na = 0;
    for (const int4 &v : q.enode)
      for (int n : {v.x, v.y, v.z})
        if (slot_of[(size_t)n] < 0) slot_of[(size_t)n] = na++;
    for (int &a : slot_of)
      if (a < 0) a = na++;
    std::vector<int2> rng(nn, make_int2(0, 0));
    for (const int4 &v : q.enode)
      for (int n : {v.x, v.y, v.z}) ++rng[(size_t)slot_of[(size_t)n]].y;
    int at = 3 * e0;
    for (int2 &r : rng) { r.x = at; at += r.y; r.y = 0; }
    std::vector<int> inc(3 * ne);
    std::vector<int4> evb(ne);
    for (size_t i = 0; i < ne; ++i) {
      const int4 v = q.enode[i];
      const int a[3] = {slot_of[(size_t)v.x], slot_of[(size_t)v.y], slot_of[(size_t)v.z]};
      for (int j = 0; j < 3; ++j) {
        int2 &r = rng[(size_t)a[j]];
        inc[(size_t)(r.x - 3 * e0 + r.y)] = (int)i + e0;
        ++r.y;
      }
      evb[i] = make_int4(a[0] + n0, a[1] + n0, a[2] + n0, 0);
    }
    chk(put(m.nd_rng, (size_t)n0, rng.data(), nn));
    chk(put(m.nd_el, 3 * (size_t)e0, inc.data(), 3 * ne));
    chk(put(m.evb, (size_t)e0, evb.data(), ne));
  }
  if (mixed) {
    chk(put(m.egf, e0, q.egf.data(), ne));
    chk(put(m.le_f, (size_t)off[A_LEDGE], q.le_f.data(), (size_t)need[A_LEDGE]));
  } else {
    chk(put(m.eg1, e0, q.eg1.data(), ne));
    chk(put(m.eg2, e0, q.eg2.data(), ne));
    chk(put(m.le_a, (size_t)off[A_LEDGE], q.le_a.data(), (size_t)need[A_LEDGE]));
    chk(put(m.le_b, (size_t)off[A_LEDGE], q.le_b.data(), (size_t)need[A_LEDGE]));
  }
  {
    std::vector<int> g(q.lgid.begin(), q.lgid.begin() + need[A_LOC]);
    for (int &x : g) x += e0;
    chk(put(m.lgid, (size_t)off[A_LOC], g.data(), g.size()));
    chk(put(m.lhb01, (size_t)off[A_LOC], q.lhb01.data(), (size_t)need[A_LOC]));
    chk(put(m.lhb2, (size_t)off[A_LOC], q.lhb2.data(), (size_t)need[A_LOC]));
    chk(put(m.lnb, (size_t)off[A_LOC], q.lnb.data(), (size_t)need[A_LOC]));
    // ring-2 list and a sentinel (the member's first element)
    std::vector<int> r2((size_t)need[A_RING2], e0);
    for (int i = 0; i < q.h2_off[q.nch]; ++i) r2[(size_t)i] = q.h2[(size_t)i] + e0;
    chk(put(m.h2, (size_t)off[A_RING2], r2.data(), r2.size()));
  }
  if (S->order == 2) {
    chk(put(m.hmean, e0, q.hmean.data(), ne));
    std::vector<int2> g(q.le_g.begin(), q.le_g.begin() + need[A_LEDGE]);
    for (int2 &x : g) { x.x += e0; x.y += e0; }
    chk(put(m.le_g, (size_t)off[A_LEDGE], g.data(), g.size()));
  }
  if (e != hipSuccess) {
    for (int a = 0; a < A_COUNT; ++a) S->arena[a].give(off[a], need[a]);
    return hip_fail(S, e, "upload");
  }
  MemberHost &h = S->mh[(size_t)slot];
  h = MemberHost{};
  h.active = true;
  h.perm = q.perm;  // copied: a prepared mesh stays whole until its admission has succeeded
  h.ne = q.ne; h.nn = q.nn; h.ned = q.ned; h.nbnd = q.nbnd;
  for (int a = 0; a < A_COUNT; ++a) { h.off[a] = off[a]; h.len[a] = need[a]; }
  h.chunks.resize((size_t)q.nch * kChunkHost);
  for (int c = 0; c < q.nch; ++c) {
    int *r = &h.chunks[(size_t)c * kChunkHost];
    r[0] = q.ch_off[c]; r[1] = q.ch_off[c + 1] - q.ch_off[c];
    r[2] = q.h1_off[c + 1] - q.h1_off[c];
    r[3] = q.h2_off[c]; r[4] = q.h2_off[c + 1] - q.h2_off[c];
    r[5] = q.le_off[c]; r[6] = q.le_off[c + 1] - q.le_off[c];
    r[7] = q.lo_off[c];
  }
  h.nl_max = q.nl_max; h.nm_max = q.nm_max; h.ed_max = q.ed_max; h.n2_max = q.n2_max;
  h.C = q.C;
  S->m.C = std::max(S->m.C, q.C);
  Member f{};
  f.e0 = e0; f.ne = q.ne; f.n0 = n0; f.nn = q.nn;
  f.pn = 101300.0;
  S->mem[(size_t)slot] = f;
  // zero state (every mode row of the current buffer), forcing and Manning
  const size_t nm = (size_t)S->nm, qs = mixed ? sizeof(float) : sizeof(double);
  unsigned char *base = (unsigned char *)S->s.buf[S->cur];
  for (size_t j = 0; j < nm && e == hipSuccess; ++j)
    e = hipMemsetAsync(base + (j * E + e0) * sizeof(double), 0, ne * sizeof(double), S->stream);
  for (size_t j = 0; j < 2 * nm && e == hipSuccess; ++j)
    e = hipMemsetAsync(base + nm * E * sizeof(double) + (j * E + e0) * qs, 0, ne * qs, S->stream);
  if (e == hipSuccess) e = hipMemsetAsync(S->s.nodal + 2 * (size_t)n0, 0, 2 * nn * sizeof(double), S->stream);
  if (e == hipSuccess) e = hipMemsetAsync(S->s.nodal + 2 * N + n0, 0, nn * sizeof(double), S->stream);
  if (e == hipSuccess) e = hipMemsetAsync(S->d_man + E + slot, 0, sizeof(double), S->stream);
  if (e == hipSuccess) e = hipMemsetAsync(S->d_manf + E + slot, 0, sizeof(float), S->stream);
  if (e == hipSuccess)
    e = launch_init_state(S->m, S->s, S->prm, S->s.buf[S->cur], slot, e0, q.ne, 0.0, (int)(S->steps_enq & 1), 0,
                          S->precision, S->order, S->stream);
  if (e != hipSuccess) {
    release_slot(S, slot);
    return hip_fail(S, e, "member initialisation");
  }
  return DGSWE_OK;
}

// Chunk records of the active members (slot order), member table, forcing
// blocks and the mesh maxima; waits for the stream first (the kernels read
// these tables).
dgswe_status rebuild(dgswe_solver *S) {
  hipError_t e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "hipStreamSynchronize");
  drop_graphs(S);
  DevMesh &m = S->m;
  const int E = m.ne;
  S->chunk_rec.clear();
  int nch = 0;
  S->nn = S->ne = S->ned = S->nbnd = 0;
  m.nl_max = m.nm_max = m.ed_max = m.n2_max = 1;
  m.C = 1;
  for (size_t i = 0; i < S->mh.size(); ++i) {
    MemberHost &h = S->mh[i];
    Member &f = S->mem[i];
    if (!h.active) {
      f = Member{};
      f.pn = 101300.0;
      continue;
    }
    const int nc = (int)(h.chunks.size() / kChunkHost);
    f.chunk0 = nch;
    f.nchunk = nc;
    for (int c = 0; c < nc; ++c) {
      const int *r = &h.chunks[(size_t)c * kChunkHost];
      int rec[kChunkRec] = {};
      rec[0] = f.e0 + r[0]; rec[1] = r[1];
      rec[2] = 0; rec[3] = r[2];
      rec[4] = (int)h.off[A_RING2] + r[3]; rec[5] = r[4];
      rec[6] = (int)h.off[A_LEDGE] + r[5]; rec[7] = r[6];
      rec[8] = (int)h.off[A_LOC] + r[7];
      rec[9] = (int)i;
      rec[10] = c == 0 ? 1 : 0;
      rec[11] = h.man_elem ? f.e0 + r[0] : E + (int)i;
      rec[12] = h.man_elem ? 1 : 0;
      S->chunk_rec.insert(S->chunk_rec.end(), rec, rec + kChunkRec);
      ++nch;
    }
    S->nn += h.nn; S->ne += h.ne; S->ned += h.ned; S->nbnd += h.nbnd;
    m.nl_max = std::max(m.nl_max, h.nl_max); m.nm_max = std::max(m.nm_max, h.nm_max);
    m.ed_max = std::max(m.ed_max, h.ed_max); m.n2_max = std::max(m.n2_max, h.n2_max);
    m.C = std::max(m.C, h.C);
  }
  if (nch > S->chunk_cap) return fail(S, DGSWE_E_NOMEM, "chunk table full");
  m.nch = nch;
  m.ned = S->ned;
  if (nch > 0) {
    e = hipMemcpy(S->d_chunk_rec, S->chunk_rec.data(), S->chunk_rec.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
  }
  return sync_members(S);
}

// capacities of the arenas for a pool of max_elems elements and `slots` members
void pool_caps(long long max_elems, int slots, int order, long long cap[A_COUNT], int &chunk_cap) {
  const long long E = max_elems, M = slots;
  cap[A_ELEM] = E;
  cap[A_NODE] = E + 3 * M;
  cap[A_LOC] = 2 * E + 512 * M;
  cap[A_LEDGE] = 2 * E + 512 * M;
  cap[A_RING2] = E + 256 * M;
  chunk_cap = (int)(E / 64 + 2 * M + 1);
}

dgswe_status create_impl(int32_t n_members, const dgswe_mesh *meshes, const dgswe_params *prm, void *hip_stream,
                         dgswe_solver **out) {
  if (!out) return fail(nullptr, DGSWE_E_INVALID, "out is NULL");
  *out = nullptr;
  if (n_members < 1 || !meshes) return fail(nullptr, DGSWE_E_INVALID, "a batch needs at least one mesh");
  std::string msg;
  if (!validate_params(prm, msg)) return fail(nullptr, DGSWE_E_INVALID, msg);
  int chunk, block;
  if (!chunk_config(prm, chunk, block)) return fail(nullptr, DGSWE_E_INVALID, "unsupported chunk/block configuration");
  long long ne_total = 0;
  for (int32_t i = 0; i < n_members; ++i) ne_total += meshes[i].n_elems > 0 ? meshes[i].n_elems : 0;
  if (ne_total > 0x7fffffffLL) return fail(nullptr, DGSWE_E_INVALID, "more than 2^31 - 1 elements in the batch");
  std::vector<Prep> parts((size_t)n_members);
  // host preprocessing of the meshes, several at a time (each thread owns
  // whole meshes; the first failing mesh in order is reported)
  std::vector<int> rcs((size_t)n_members, DGSWE_OK);
  std::vector<std::string> msgs((size_t)n_members);
  {
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const int nt = (int)std::min<unsigned>(hw, (unsigned)n_members);
    auto work = [&](int t0) {
      for (int i = t0; i < n_members; i += nt) rcs[i] = prep_one(meshes[i], prm->p, prm->precision, chunk, block, parts[i], msgs[i]);
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
  // arenas sized to the meshes
  long long cap[A_COUNT] = {};
  int chunk_cap = 0;
  for (const Prep &q : parts) {
    long long need[A_COUNT];
    arena_need(q, prm->p, need);
    for (int a = 0; a < A_COUNT; ++a) cap[a] += need[a];
    chunk_cap += q.nch;
  }
  dgswe_solver *S = nullptr;
  dgswe_status st = alloc_solver(prm, block, cap, chunk_cap, n_members, hip_stream, &S);
  if (st != DGSWE_OK) return st;
  for (int32_t i = 0; i < n_members; ++i) {
    st = place_member(S, i, parts[(size_t)i]);
    parts[(size_t)i] = Prep();
    if (st != DGSWE_OK) {
      msg = S->err;
      free_all(S);
      delete S;
      return fail(nullptr, st, msg);
    }
  }
  st = rebuild(S);
  if (st == DGSWE_OK && hipStreamSynchronize(S->stream) != hipSuccess) st = DGSWE_E_DEVICE;
  if (st != DGSWE_OK) {
    msg = S->err;
    free_all(S);
    delete S;
    return fail(nullptr, st, "device initialisation failed: " + msg);
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
  const size_t ne = (size_t)h.ne, NE = (size_t)S->m.ne, nm = (size_t)S->nm;
  const bool mixed = S->precision == DGSWE_MIXED;
  // member-order image: zeta modes FP64, momentum modes FP64 or FP32
  {
    const hipError_t e0 = pinned(S->stage_in, S->stage_in_bytes, state_bytes(ne, S->precision, S->order));
    if (e0 != hipSuccess) return hip_fail(S, e0, "hipHostMalloc");
  }
  double *z = (double *)S->stage_in;
  const int *perm = h.perm.data();
  for_planes(3 * nm, ne, [&](size_t j) {
    if (j < nm) {
      for (size_t i = 0; i < ne; ++i) z[j * ne + i] = w[j * ne + (size_t)perm[i]];
    } else if (mixed) {
      float *q = (float *)(z + nm * ne) + (j - nm) * ne;
      for (size_t i = 0; i < ne; ++i) q[i] = (float)w[j * ne + (size_t)perm[i]];
    } else {
      double *q = z + nm * ne + (j - nm) * ne;
      for (size_t i = 0; i < ne; ++i) q[i] = w[j * ne + (size_t)perm[i]];
    }
  });
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
  S->forcing_fresh = false;
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
  const size_t ne = (size_t)h.ne, nn = (size_t)h.nn, NN = (size_t)S->m.nn, NE = (size_t)S->m.ne;
  hipError_t e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "hipStreamSynchronize");
  S->forcing_fresh = false;
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
  f.coriolis = fr->coriolis;
  f.rain = fr->rain;
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
    e = hipMemcpy(S->d_man + NE + member, &fr->manning_n, sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(S->d_manf + NE + member, &nf, sizeof(float), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
  // the member's chunk records point at the Manning values that apply
  h.man_elem = per_elem;
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
  return rebuild(S);
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
    if (S->rb_elems < ne) {
      if (S->rb) (void)hipFree(S->rb);
      S->rb = nullptr;
      S->rb_elems = 0;
      e = hipMalloc(&S->rb, nv * ne * sizeof(double));
      if (e != hipSuccess) return hip_fail(S, e, "hipMalloc");
      S->rb_elems = ne;
    }
    if (S->order == 2)
      e = launch_post_only2(S->m, S->prm, S->s.buf[S->cur], h.cur_is_pp ? 0 : 1, f.e0, f.ne, S->rb, nullptr,
                            S->precision, S->stream);
    else
      e = launch_post_only(S->m, S->s, S->prm, S->s.buf[S->cur], h.cur_is_pp ? 0 : 1, f.e0, f.ne, S->rb, nullptr,
                           S->precision, S->stream);
    if (e != hipSuccess) return hip_fail(S, e, "post-processing kernel");
    e = pinned(S->stage_out, S->stage_out_bytes, nv * ne * sizeof(double));
    if (e != hipSuccess) return hip_fail(S, e, "hipHostMalloc");
    const double *sb = (const double *)S->stage_out;
    e = hipMemcpyAsync(S->stage_out, S->rb, nv * ne * sizeof(double), hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) return hip_fail(S, e, "hipMemcpy");
    const int *perm = h.perm.data();
    for_planes(nv, ne, [&](size_t j) {
      for (size_t i = 0; i < ne; ++i) w_out[j * ne + (size_t)perm[i]] = sb[j * ne + i];
    });
  }
  Ctrl c{};
  if (d) {
    e = launch_diag(S->m, S->prm, S->s.buf[S->cur], f.e0, f.ne, S->s.partial, S->d_diag, S->stream);
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

// Enqueue n steps launch by launch (also the body of a captured graph).
dgswe_status enqueue_steps(dgswe_solver *S, int32_t n_steps) {
  const DevMesh &m = S->m;
  DevState &st = S->s;
  const Params &p = S->prm;
  const int want_dt = (p.dt_fixed > 0.0) ? 0 : 1;
  StageCoef sc[5];
  const int ns = rk_stages(S->uprm.rk, sc);
  // a captured graph may be replayed after the forcing changed: it always
  // computes its first stage's forcing
  bool fresh = S->forcing_fresh && !S->capturing;
  const bool reuse = sc[ns - 1].c == 1.0 && !S->forcing_every_stage;
  for (int i = 0; i < n_steps; ++i) {
    const int slot = (int)(S->steps_enq & 1);
    // buffers: stage k reads buf[(cur + k) % 3] and writes buf[(cur + k + 1)
    // % 3] (unlimited); wpp holds the post-processed w^n (RK base), so the
    // buffer of w^n is free from the second stage on
    const int cur = S->cur;
    hipError_t e = hipSuccess;
    for (int stage = 0; stage < ns && e == hipSuccess; ++stage) {
      void *in = st.buf[(cur + stage) % 3], *out = st.buf[(cur + stage + 1) % 3];
      const int wd = sc[stage].last ? want_dt : 0;
      if (S->nfblk > 0 && !(stage == 0 && fresh)) {
        Timed t(S, K_FORCING);
        e = launch_forcing(m, st, p, S->nfblk, slot, sc[stage].c, S->stream);
      }
      if (e != hipSuccess) break;
      if (S->order == 2) {
        // records of the stage input: w^n's go to wpp (the RK base), a later
        // stage's to the one buffer it neither reads nor writes
        void *rec = stage == 0 ? st.wpp : st.buf[(cur + stage + 2) % 3];
        {
          Timed t(S, K_PP2);
          e = launch_pp2(m, st, p, in, rec, slot, stage == 0 ? 0 : 1, S->precision, S->stream);
        }
        if (e != hipSuccess) break;
        Timed t(S, K_RHS2);
        e = launch_rhs2(m, st, p, rec, stage == 0 ? nullptr : st.wpp, out, slot, stage == 0, sc[stage], wd,
                        S->precision, S->stream);
        continue;
      }
      if (p.limiter == 2) {
        Timed t(S, K_VBOUNDS);
        e = launch_vbounds(m, st, in, S->precision, S->stream);
        if (e != hipSuccess) break;
      }
      Timed t(S, K_STAGE);
      e = launch_stage(m, st, p, in, stage == 0 ? nullptr : st.wpp, out, stage == 0 ? st.wpp : nullptr, slot,
                       stage == 0, sc[stage], wd, S->block, S->precision, S->stream);
    }
    if (e != hipSuccess) return hip_fail(S, e, "kernel launch");
    S->cur = (cur + ns) % 3;
    for (MemberHost &h : S->mh) h.cur_is_pp = false;
    S->steps_enq += 1;
    fresh = reuse;
  }
  if (!S->capturing) S->forcing_fresh = fresh;
  return DGSWE_OK;
}

// One graph launch of graph_steps steps from the current (rotation,
// parity), captured on first use.  graph_steps is a multiple of 6, so the
// buffer rotation and the step parity are back where they started.
dgswe_status graph_steps(dgswe_solver *S) {
  const int key = S->cur * 2 + (int)(S->steps_enq & 1);
  if (!S->graph[key]) {
    const int cur = S->cur;
    const long long se = S->steps_enq;
    hipError_t e = hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(S, e, "hipStreamBeginCapture");
    S->capturing = true;
    dgswe_status st = enqueue_steps(S, S->graph_steps);
    S->capturing = false;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(S->stream, &g);
    // the capture only recorded: put the bookkeeping back
    S->cur = cur;
    S->steps_enq = se;
    if (st != DGSWE_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(S, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&S->graph[key], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      S->graph[key] = nullptr;
      return hip_fail(S, e, "hipGraphInstantiate");
    }
  }
  hipError_t e = hipGraphLaunch(S->graph[key], S->stream);
  if (e != hipSuccess) return hip_fail(S, e, "hipGraphLaunch");
  for (MemberHost &h : S->mh) h.cur_is_pp = false;
  {
    StageCoef sc[5];
    const int ns = rk_stages(S->uprm.rk, sc);
    S->forcing_fresh = sc[ns - 1].c == 1.0 && !S->forcing_every_stage;
  }
  S->steps_enq += S->graph_steps;
  return DGSWE_OK;
}

// Enqueue n steps of a p = 1 solver A and a p = 2 solver B on A's stream,
// each stage one k_pp2 launch for B's stage input and one launch of both
// solvers' stage work (launch_stage12); forcing and bookkeeping per solver
// as in enqueue_steps.
dgswe_status enqueue_pair(dgswe_solver *A, dgswe_solver *B, int32_t n_steps) {
  StageCoef sc[5];
  const int ns = rk_stages(A->uprm.rk, sc);
  const int wda = A->prm.dt_fixed > 0.0 ? 0 : 1, wdb = B->prm.dt_fixed > 0.0 ? 0 : 1;
  bool fa = A->forcing_fresh && !A->capturing, fb = B->forcing_fresh && !B->capturing;
  const bool ra = sc[ns - 1].c == 1.0 && !A->forcing_every_stage;
  const bool rb = sc[ns - 1].c == 1.0 && !B->forcing_every_stage;
  DevState &sa = A->s, &sb = B->s;
  for (int i = 0; i < n_steps; ++i) {
    const int la = (int)(A->steps_enq & 1), lb = (int)(B->steps_enq & 1);
    const int ca = A->cur, cb = B->cur;
    hipError_t e = hipSuccess;
    for (int stage = 0; stage < ns && e == hipSuccess; ++stage) {
      if (A->nfblk > 0 && !(stage == 0 && fa)) {
        Timed t(A, K_FORCING);
        e = launch_forcing(A->m, sa, A->prm, A->nfblk, la, sc[stage].c, A->stream);
      }
      if (e == hipSuccess && B->nfblk > 0 && !(stage == 0 && fb)) {
        Timed t(A, K_FORCING);
        e = launch_forcing(B->m, sb, B->prm, B->nfblk, lb, sc[stage].c, A->stream);
      }
      if (e != hipSuccess) break;
      void *rec = stage == 0 ? sb.wpp : sb.buf[(cb + stage + 2) % 3];
      if (A->prm.pair_split) {
        // the p = 1 stage with the p = 2 post-processing, then the p = 2
        // right-hand side (the default: measured faster than the other
        // arrangement below, whose post-processing launch runs alone)
        {
          Timed t(A, K_STAGE1PP2);
          e = launch_stage1pp2(A->m, sa, A->prm, sa.buf[(ca + stage) % 3], stage == 0 ? nullptr : sa.wpp,
                               sa.buf[(ca + stage + 1) % 3], stage == 0 ? sa.wpp : nullptr, la,
                               sc[stage].last ? wda : 0, B->m, sb, B->prm, sb.buf[(cb + stage) % 3], rec, lb,
                               stage == 0, sc[stage], A->precision, A->stream);
        }
        if (e != hipSuccess) break;
        Timed t(A, K_RHS2);
        e = launch_rhs2(B->m, sb, B->prm, rec, stage == 0 ? nullptr : sb.wpp, sb.buf[(cb + stage + 1) % 3], lb,
                        stage == 0, sc[stage], sc[stage].last ? wdb : 0, B->precision, A->stream);
        continue;
      }
      {
        Timed t(A, K_PP2);
        e = launch_pp2(B->m, sb, B->prm, sb.buf[(cb + stage) % 3], rec, lb, stage == 0 ? 0 : 1, B->precision,
                       A->stream);
      }
      if (e != hipSuccess) break;
      Timed t(A, K_STAGE12);
      e = launch_stage12(A->m, sa, A->prm, sa.buf[(ca + stage) % 3], stage == 0 ? nullptr : sa.wpp,
                         sa.buf[(ca + stage + 1) % 3], stage == 0 ? sa.wpp : nullptr, la,
                         sc[stage].last ? wda : 0, B->m, sb, B->prm, rec, stage == 0 ? nullptr : sb.wpp,
                         sb.buf[(cb + stage + 1) % 3], lb, sc[stage].last ? wdb : 0, stage == 0, sc[stage],
                         A->precision, A->stream);
    }
    if (e != hipSuccess) return hip_fail(A, e, "kernel launch");
    A->cur = (ca + ns) % 3;
    B->cur = (cb + ns) % 3;
    for (MemberHost &h : A->mh) h.cur_is_pp = false;
    for (MemberHost &h : B->mh) h.cur_is_pp = false;
    A->steps_enq += 1;
    B->steps_enq += 1;
    fa = ra;
    fb = rb;
  }
  if (!A->capturing) {
    A->forcing_fresh = fa;
    B->forcing_fresh = fb;
  }
  return DGSWE_OK;
}

// One graph launch of A's graph_steps steps of the pair, captured on first
// use per (rotation, parity) of both solvers.
dgswe_status pair_graph_steps(dgswe_solver *A, dgswe_solver *B) {
  if (A->pair_id != B->id || A->pair_gen != B->gen) {
    drop_pair_graphs(A);
    A->pair_id = B->id;
    A->pair_gen = B->gen;
  }
  const int key = ((A->cur * 2 + (int)(A->steps_enq & 1)) * 3 + B->cur) * 2 + (int)(B->steps_enq & 1);
  if (!A->pair_graph[key]) {
    const int ca = A->cur, cb = B->cur;
    const long long ea = A->steps_enq, eb = B->steps_enq;
    hipError_t e = hipStreamBeginCapture(A->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(A, e, "hipStreamBeginCapture");
    A->capturing = B->capturing = true;
    dgswe_status st = enqueue_pair(A, B, A->graph_steps);
    A->capturing = B->capturing = false;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(A->stream, &g);
    // the capture only recorded: put the bookkeeping back
    A->cur = ca; B->cur = cb;
    A->steps_enq = ea; B->steps_enq = eb;
    if (st != DGSWE_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(A, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&A->pair_graph[key], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      A->pair_graph[key] = nullptr;
      return hip_fail(A, e, "hipGraphInstantiate");
    }
  }
  hipError_t e = hipGraphLaunch(A->pair_graph[key], A->stream);
  if (e != hipSuccess) return hip_fail(A, e, "hipGraphLaunch");
  StageCoef sc[5];
  const int ns = rk_stages(A->uprm.rk, sc);
  for (dgswe_solver *S : {A, B}) {
    for (MemberHost &h : S->mh) h.cur_is_pp = false;
    S->forcing_fresh = sc[ns - 1].c == 1.0 && !S->forcing_every_stage;
    S->cur = (S->cur + ns * A->graph_steps) % 3;
    S->steps_enq += A->graph_steps;
  }
  return DGSWE_OK;
}

// Entry points return a status and never let an exception cross the C ABI:
// a failed host allocation (std::bad_alloc) becomes DGSWE_E_NOMEM, anything
// else DGSWE_E_DEVICE, with the message in dgswe_last_error.
template <class F>
dgswe_status guard(dgswe_solver *S, F &&f) noexcept {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    try {
      return fail(S, DGSWE_E_NOMEM, "host allocation failed");
    } catch (...) {
      return DGSWE_E_NOMEM;
    }
  } catch (...) {
    try {
      return fail(S, DGSWE_E_DEVICE, "unexpected host error");
    } catch (...) {
      return DGSWE_E_DEVICE;
    }
  }
}

}  // namespace

extern "C" {

void dgswe_default_params(dgswe_params *p) {
  if (!p) return;
  p->rk = 22;
  p->flux = 0;
  p->chunk = 0;
  p->waves = 0;
  p->persistent = 0;
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
  return guard(nullptr, [&]() -> dgswe_status {
    dgswe_mesh d{n_nodes, node_xy, node_hb, n_elems, tri, n_bnd, bnd_nodes, bnd_type};
    return create_impl(1, &d, prm, hip_stream, out);
  });
}

dgswe_status dgswe_create_batch(int32_t n_meshes, const dgswe_mesh *meshes, const dgswe_params *prm,
                                void *hip_stream, dgswe_solver **out) {
  return guard(nullptr, [&]() -> dgswe_status {
    return create_impl(n_meshes, meshes, prm, hip_stream, out);
  });
}

dgswe_status dgswe_set_state(dgswe_solver *S, double t, const double *w, int32_t postprocess) {
  return guard(S, [&]() -> dgswe_status {
    dgswe_status st = single(S);
    return st != DGSWE_OK ? st : set_state_impl(S, 0, t, w, postprocess);
  });
}

dgswe_status dgswe_member_set_state(dgswe_solver *S, int32_t member, double t, const double *w,
                                    int32_t postprocess) {
  return guard(S, [&]() -> dgswe_status {
    return set_state_impl(S, member, t, w, postprocess);
  });
}

dgswe_status dgswe_set_forcing(dgswe_solver *S, const dgswe_forcing *f) {
  return guard(S, [&]() -> dgswe_status {
    dgswe_status st = single(S);
    return st != DGSWE_OK ? st : set_forcing_impl(S, 0, f);
  });
}

dgswe_status dgswe_member_set_forcing(dgswe_solver *S, int32_t member, const dgswe_forcing *f) {
  return guard(S, [&]() -> dgswe_status {
    return set_forcing_impl(S, member, f);
  });
}

dgswe_status dgswe_step(dgswe_solver *S, int32_t n_steps) {
  return guard(S, [&]() -> dgswe_status {
    if (!S) return fail(nullptr, DGSWE_E_INVALID, "solver is NULL");
    if (n_steps < 0) return fail(S, DGSWE_E_INVALID, "n_steps < 0");
    if (S->m.nch == 0) return DGSWE_OK;  // no member
    int32_t left = n_steps;
    if (S->graph_steps > 0 && !S->prof) {
      while (left >= S->graph_steps) {
        dgswe_status st = graph_steps(S);
        if (st != DGSWE_OK) return st;
        left -= S->graph_steps;
      }
    }
    return enqueue_steps(S, left);
  });
}

dgswe_status dgswe_step_pair(dgswe_solver *A, dgswe_solver *B, int32_t n_steps) {
  return guard(A, [&]() -> dgswe_status {
    if (!A || !B) return fail(A, DGSWE_E_INVALID, "solver is NULL");
    if (n_steps < 0) return fail(A, DGSWE_E_INVALID, "n_steps < 0");
    if (A->order != 1 || B->order != 2) return fail(A, DGSWE_E_INVALID, "the pair is a p = 1 and a p = 2 solver");
    if (A->device != B->device) return fail(A, DGSWE_E_INVALID, "the pair must share a device");
    if (A == B) return fail(A, DGSWE_E_INVALID, "the pair needs two solvers");
    if (A->precision != B->precision || A->uprm.rk != B->uprm.rk)
      return fail(A, DGSWE_E_INVALID, "the pair must share the precision and the time stepper");
    if (A->prm.limiter == 2) return fail(A, DGSWE_E_INVALID, "the pair does not take the vertex-based limiter");
    if (A->block != 256 || B->block != 256) return fail(A, DGSWE_E_INVALID, "the pair needs 256-lane workgroups");
    if (A->prm.persistent != B->prm.persistent)
      return fail(A, DGSWE_E_INVALID, "the pair must share the persistent setting");
    if (B->m.nch == 0) return dgswe_step(A, n_steps);
    if (A->m.nch == 0) return dgswe_step(B, n_steps);
    // everything runs on A's stream; B's stream (if another) is ordered
    // before and after it with events
    const bool two = A->stream != B->stream;
    hipError_t e = hipSuccess;
    if (two) {
      for (hipEvent_t *ev : {&A->pair_ev, &B->pair_ev})
        if (!*ev && (e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess)
          return hip_fail(A, e, "hipEventCreate");
      e = hipEventRecord(B->pair_ev, B->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(A->stream, B->pair_ev, 0);
      if (e != hipSuccess) return hip_fail(A, e, "stream ordering");
    }
    int32_t left = n_steps;
    dgswe_status st = DGSWE_OK;
    if (A->graph_steps > 0 && !A->prof) {
      while (st == DGSWE_OK && left >= A->graph_steps) {
        st = pair_graph_steps(A, B);
        left -= A->graph_steps;
      }
    }
    if (st == DGSWE_OK) st = enqueue_pair(A, B, left);
    if (two) {
      e = hipEventRecord(A->pair_ev, A->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(B->stream, A->pair_ev, 0);
      if (e != hipSuccess && st == DGSWE_OK) return hip_fail(A, e, "stream ordering");
    }
    return st;
  });
}

dgswe_status dgswe_use_graphs(dgswe_solver *S, int32_t steps_per_graph) {
  return guard(S, [&]() -> dgswe_status {
    if (!S) return fail(nullptr, DGSWE_E_INVALID, "solver is NULL");
    if (steps_per_graph < 0) return fail(S, DGSWE_E_INVALID, "steps_per_graph < 0");
    hipError_t e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) return hip_fail(S, e, "hipStreamSynchronize");
    drop_graphs(S);
    S->graph_steps = steps_per_graph == 0 ? 0 : (steps_per_graph + 5) / 6 * 6;
    return DGSWE_OK;
  });
}

dgswe_status dgswe_read_state(dgswe_solver *S, double *w_out, dgswe_diag *d) {
  return guard(S, [&]() -> dgswe_status {
    dgswe_status st = single(S);
    return st != DGSWE_OK ? st : read_state_impl(S, 0, w_out, d);
  });
}

dgswe_status dgswe_member_read_state(dgswe_solver *S, int32_t member, double *w_out, dgswe_diag *d) {
  return guard(S, [&]() -> dgswe_status {
    return read_state_impl(S, member, w_out, d);
  });
}

dgswe_status dgswe_member_read_state_device(dgswe_solver *S, int32_t member, double *w_dev, double *diag_dev) {
  return guard(S, [&]() -> dgswe_status {
    const dgswe_status st = check_member(S, member);
    if (st != DGSWE_OK) return st;
    const MemberHost &h = S->mh[member];
    const Member &f = S->mem[member];
    if (h.ne > DGSWE_NOALLOC_MAX_ELEMS)
      return fail(S, DGSWE_E_INVALID, "member has " + std::to_string(h.ne) +
                                          " elements; the allocation-free read-back takes at most " +
                                          std::to_string(DGSWE_NOALLOC_MAX_ELEMS));
    double *scr = nullptr;
    hipError_t e = scratch_on(S->device, &scr);
    if (e != hipSuccess) return hip_fail(S, e, "hipGetSymbolAddress (read-back scratch)");
    const int pp = h.cur_is_pp ? 0 : 1;
    if (w_dev) {
      if (S->order == 2)
        e = launch_post_only2(S->m, S->prm, S->s.buf[S->cur], pp, f.e0, f.ne, w_dev, S->m.perm, S->precision,
                              S->stream);
      else
        e = launch_post_only(S->m, S->s, S->prm, S->s.buf[S->cur], pp, f.e0, f.ne, w_dev, S->m.perm, S->precision,
                             S->stream);
      if (e != hipSuccess) return hip_fail(S, e, "post-processing kernel");
    }
    if (diag_dev) {
      double *sums = scr + 3 * (size_t)kNoAllocBlocks;
      e = launch_diag(S->m, S->prm, S->s.buf[S->cur], f.e0, f.ne, scr, sums, S->stream);
      if (e == hipSuccess)
        e = launch_diag_pack(S->s.ctrl + member, (int)(S->steps_enq & 1), f.ne, sums, diag_dev, S->stream);
      if (e != hipSuccess) return hip_fail(S, e, "diagnostics kernel");
    }
    return DGSWE_OK;
  });
}

void dgswe_destroy(dgswe_solver *S) {
  if (!S) return;
  try {
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    free_all(S);
  } catch (...) {
  }
  delete S;
}

const char *dgswe_last_error(const dgswe_solver *S) {
  return S ? S->err.c_str() : g_create_error.c_str();
}

dgswe_status dgswe_profile(dgswe_solver *S, int32_t enable) {
  return guard(S, [&]() -> dgswe_status {
    if (!S) return fail(nullptr, DGSWE_E_INVALID, "solver is NULL");
    dgswe_status st = drain_profile(S);
    if (st != DGSWE_OK) return st;
    for (int k = 0; k < K_COUNT; ++k) { S->prof_ms[k] = 0.0; S->prof_n[k] = 0; }
    S->prof = enable != 0;
    return DGSWE_OK;
  });
}

dgswe_status dgswe_profile_read(dgswe_solver *S, int32_t max_kernels, char *names, double *total_ms,
                                int64_t *launches, int32_t *n_out) {
  return guard(S, [&]() -> dgswe_status {
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
  });
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
  if (!S || !out || member < 0 || member >= (int32_t)S->mh.size() || !S->mh[(size_t)member].active)
    return DGSWE_E_INVALID;
  const MemberHost &h = S->mh[member];
  out[0] = h.nn;
  out[1] = h.ne;
  out[2] = h.ned;
  out[3] = h.nbnd;
  return DGSWE_OK;
}

int32_t dgswe_member_count(const dgswe_solver *S) { return S ? (int32_t)S->mh.size() : 0; }

dgswe_status dgswe_create_pool(int64_t max_elems, int32_t max_members, const dgswe_params *prm, void *hip_stream,
                               dgswe_solver **out) {
  return guard(nullptr, [&]() -> dgswe_status {
    if (!out) return fail(nullptr, DGSWE_E_INVALID, "out is NULL");
    *out = nullptr;
    std::string msg;
    if (!validate_params(prm, msg)) return fail(nullptr, DGSWE_E_INVALID, msg);
    if (max_elems < 1 || max_elems > 0x3fffffffLL || max_members < 1 || max_members > 65536)
      return fail(nullptr, DGSWE_E_INVALID, "pool capacity out of range");
    int chunk, block;
    if (!chunk_config(prm, chunk, block)) return fail(nullptr, DGSWE_E_INVALID, "unsupported chunk/block configuration");
    long long cap[A_COUNT];
    int chunk_cap = 0;
    pool_caps(max_elems, max_members, prm->p, cap, chunk_cap);
    dgswe_solver *S = nullptr;
    dgswe_status st = alloc_solver(prm, block, cap, chunk_cap, max_members, hip_stream, &S);
    if (st != DGSWE_OK) return st;
    S->is_pool = true;
    st = rebuild(S);
    if (st != DGSWE_OK) {
      msg = S->err;
      free_all(S);
      delete S;
      return fail(nullptr, st, msg);
    }
    *out = S;
    return DGSWE_OK;
  });
}

dgswe_status dgswe_prepare_mesh(const dgswe_mesh *mesh, const dgswe_params *prm, dgswe_prepared **out) {
  return guard(nullptr, [&]() -> dgswe_status {
    if (!out) return fail(nullptr, DGSWE_E_INVALID, "out is NULL");
    *out = nullptr;
    std::string msg;
    if (!mesh) return fail(nullptr, DGSWE_E_INVALID, "mesh is NULL");
    if (!validate_params(prm, msg)) return fail(nullptr, DGSWE_E_INVALID, msg);
    int chunk, block;
    if (!chunk_config(prm, chunk, block)) return fail(nullptr, DGSWE_E_INVALID, "unsupported chunk/block configuration");
    dgswe_prepared *P = new (std::nothrow) dgswe_prepared();
    if (!P) return fail(nullptr, DGSWE_E_NOMEM, "host allocation failed");
    P->order = prm->p;
    const int rc = prep_one(*mesh, prm->p, prm->precision, chunk, block, P->P, msg);
    if (rc != DGSWE_OK) {
      delete P;
      return fail(nullptr, (dgswe_status)rc, msg);
    }
    *out = P;
    return DGSWE_OK;
  });
}

void dgswe_prepared_free(dgswe_prepared *P) { delete P; }

int64_t dgswe_prepared_elems(const dgswe_prepared *P) { return P ? P->P.ne : 0; }

dgswe_status dgswe_member_add_prepared(dgswe_solver *S, dgswe_prepared *P, int32_t *member) {
  return guard(S, [&]() -> dgswe_status {
    if (!S) return fail(nullptr, DGSWE_E_INVALID, "solver is NULL");
    if (!P || !member) return fail(S, DGSWE_E_INVALID, "prepared mesh or member is NULL");
    if (!S->is_pool) return fail(S, DGSWE_E_INVALID, "members join only a pool (dgswe_create_pool)");
    if (P->order != S->order) return fail(S, DGSWE_E_INVALID, "the mesh was prepared for another order p");
    int slot = -1;
    for (size_t i = 0; i < S->mh.size(); ++i)
      if (!S->mh[i].active) { slot = (int)i; break; }
    if (slot < 0) return fail(S, DGSWE_E_NOMEM, "every member slot is taken");
    hipError_t e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) return hip_fail(S, e, "hipStreamSynchronize");
    dgswe_status st = place_member(S, slot, P->P);
    if (st != DGSWE_OK) return st;
    st = rebuild(S);
    if (st != DGSWE_OK) {
      // not admitted after all: the slot is emptied and the caller keeps P
      const std::string msg = S->err;
      release_slot(S, slot);
      (void)rebuild(S);
      return fail(S, st, msg);
    }
    delete P;  // owned by the pool from here on
    *member = slot;
    return DGSWE_OK;
  });
}

dgswe_status dgswe_member_add(dgswe_solver *S, const dgswe_mesh *mesh, int32_t *member) {
  return guard(S, [&]() -> dgswe_status {
    if (!S) return fail(nullptr, DGSWE_E_INVALID, "solver is NULL");
    dgswe_prepared *P = nullptr;
    dgswe_status st = dgswe_prepare_mesh(mesh, &S->uprm, &P);
    if (st != DGSWE_OK) return fail(S, st, g_create_error);
    st = dgswe_member_add_prepared(S, P, member);
    if (st != DGSWE_OK) dgswe_prepared_free(P);
    return st;
  });
}

dgswe_status dgswe_member_remove(dgswe_solver *S, int32_t member) {
  return guard(S, [&]() -> dgswe_status {
    dgswe_status st = check_member(S, member);
    if (st != DGSWE_OK) return st;
    if (!S->is_pool) return fail(S, DGSWE_E_INVALID, "members leave only a pool (dgswe_create_pool)");
    hipError_t e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) return hip_fail(S, e, "hipStreamSynchronize");
    release_slot(S, member);
    return rebuild(S);
  });
}

dgswe_status dgswe_pool_usage(const dgswe_solver *S, int64_t out[5]) {
  if (!S || !out) return DGSWE_E_INVALID;
  const Arena &a = S->arena[A_ELEM];
  out[0] = a.cap() - a.free_total();
  out[1] = a.cap();
  int64_t act = 0;
  for (const MemberHost &h : S->mh) act += h.active ? 1 : 0;
  out[2] = act;
  out[3] = (int64_t)S->mh.size();
  out[4] = (int64_t)S->dev_bytes;
  return DGSWE_OK;
}

}  // extern "C"
