// Internal declarations of the gfx950 DG shallow-water library: device data
// layout, kernel argument blocks and the launch entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace dgswe {

constexpr int kMaxTide = 8;
constexpr int kBlock = 256;
// One chunk record: first element, element count, ring-1 offset and count,
// ring-2 offset and count, local-edge offset and count, local-element
// offset, member, 1 if first chunk of its member, Manning index base and
// stride (element i of the chunk reads man[base + i * stride]), padding
// (64 bytes, one scalar load).
constexpr int kChunkRec = 16;

// Device control block: one per member of a batch, read by every kernel of
// a step.  Step n of the batch reads t[n & 1] and dtmin[n & 1]; its last
// kernel writes t[(n + 1) & 1] and the CFL candidates of step n + 1 into
// dtmin[(n + 1) & 1], so no kernel writes a value another block of the same
// kernel reads.
struct Ctrl {
  double t[2];                   // model time at the start of a step, per parity
  double dt_last;                // dt of the last completed step
  unsigned long long dtmin[2];   // bit pattern of the raw CFL minimum, per parity
  long long steps;               // completed steps since the member's state was set
  int status;                    // first error detected on the device (0 = none)
  int pp_in;                     // the stored state still needs post-processing
};

// Forcing and bookkeeping of one member of a batch (device copy).  Members
// occupy disjoint, contiguous ranges of the batch's element, node and chunk
// arrays; every chunk belongs to one member.
struct Member {
  int e0, ne, n0, nn;            // element and node ranges
  int chunk0, nchunk;            // chunk range
  int holland, n_tide;
  double tide_amp[kMaxTide], tide_omega[kMaxTide], tide_phase[kMaxTide], tide_offset;
  double x0, y0, vx, vy, dp, pn, rmax, B, rho_air, coriolis_f, wind_factor;
  double coriolis, rain;          // momentum Coriolis parameter, rainfall rate
};

// Mesh on the device (internal order).  Arrays read by the stage kernel are
// packed as 16-byte records in paired structure-of-arrays form (lane i reads
// record i with one 16-byte load, a wavefront one contiguous 1 KiB block).
struct DevMesh {
  int ne, nn, ned;
  // elements, structure of arrays (initialisation, read-back, diagnostics)
  const double *area;                   // A_e
  const double *inr2;                   // 2 x inradius
  const double *hbv;                    // [3][ne] bathymetry at the element's vertices
  const int *el_nb;                     // [3][ne] neighbour across local edge, -1 none
  const int *perm;                      // [ne] the caller's index of each element within its member
  // nodes
  const double *node_x, *node_y;
  // vertex-based limiter only.  Its node ranges are numbered in the order
  // the nodes first appear in the (Hilbert-ordered) element list, so that
  // both passes over them read compact stretches: range slot a covers the
  // elements nd_el[nd_rng[a].x .. nd_rng[a].x + nd_rng[a].y) (ascending
  // ids); evb[e] holds the slots of element e's three vertices.
  const int2 *nd_rng;
  const int *nd_el;
  const int4 *evb;
  // members of the batch
  int nmem;
  const Member *mem;
  const int *fblk_off;                  // [nmem + 1] first forcing block of each member
  // Manning n: per element [ne], then one uniform value per member [nmem];
  // the chunk records say which applies
  const double *man;
  const float *manf;                    // the same in FP32 (mixed path)
  // chunks of the stage kernel (see build_chunks)
  int C, nch, nl_max, nm_max, ed_max, n2_max;
  const int *chunk_rec;                  // [nch][kChunkRec] chunk records (see chunk_records)
  const int *h2;                         // ring-2 element ids
  // chunk elements
  const double2 *eg1, *eg2;  // (d phi_10/dx, d phi_10/dy), (d phi_01/dx, d phi_01/dy), FP64 path
  const float4 *egf;         // the four gradients in FP32, mixed path
  const double2 *eai;        // (A_e, 2 x inradius)
  const int4 *enode;         // node ids; w: local edge codes of the 3 local edges, 10 bits each
  // local elements (chunk + ring 1) of each chunk
  const int *lgid;           // global element id
  const double2 *lhb01;      // vertex bathymetry 0, 1
  const double *lhb2;        // vertex bathymetry 2
  const unsigned long long *lnb;  // local neighbour index across local edge q in bits 16q (0xFFFF: none)
  // local edges of each chunk; packed ids = e+ | e- << 12 | (lp | lm << 2 | type << 4) << 24
  // (the bathymetry at the edge ends is the e+ element's, read from LDS)
  const double2 *le_a, *le_b;  // FP64: (nx, ny), (len/2, ids as bits)
  const float4 *le_f;          // mixed: (nx, ny, len/2, ids as bits)
  // p = 2: mean bathymetry per element (the wet/dry test of a neighbour)
  const double *hmean;
  // p = 2: global ids (e+, e-) of each local edge (e- = e+ on a boundary),
  // so the edge pass reaches the two records without the local-id lookup
  const int2 *le_g;
};

// One stage of an SSP Runge-Kutta scheme in Shu-Osher form: the stage
// result is a * w^n + b * (w_in + h dt L(w_in)) (post-processed w^n; a = 0:
// w_in + h dt L(w_in)), with the forcing and tide at time t^n + c dt.  last:
// the step's final stage (advances the member's time and step count and
// forms the next step's CFL minimum).
struct StageCoef {
  double a, b, h, c;
  int last;
};

// The stages of scheme `rk` (22, 33, 32, 42, 52: SSPRK(s, q)); returns the
// stage count, 0 for an unknown scheme.
int rk_stages(int rk, StageCoef out[5]);

// Parameters shared by all members of a batch.
struct Params {
  double g, rho0, h0, cfl, dt_fixed, dt_max;
  int limiter;     // 0: off, 1: face-neighbour, 2: vertex-based (p = 1)
  int wetdry;
  int flux;  // 0: LLF, 1: Roe on edges wet on both sides
  int waves; // register budget of the p = 2 stage kernel (waves per SIMD), 0: default
  int persistent;  // 0: one workgroup per chunk; N: N resident workgroups per CU
  int n_cu;        // compute units of the device
  // measured alternatives, read from the environment when a solver is
  // created: DGSWE_RHS2_MFMA=1 puts the p = 2 momentum at the area points on
  // the matrix cores; DGSWE_PAIR_SPLIT=0 makes dgswe_step_pair run a stage
  // as (p = 2 post-processing) then (both orders' stage work) instead of
  // (p = 1 stage with the p = 2 post-processing) then (p = 2 right-hand side)
  int rhs2_mfma;
  int pair_split;
};

// Workgroups of a stage launch over n work items: one per item, or (with
// persistent workgroups) N per compute unit, a multiple of the 8 XCDs so
// that every item a workgroup takes maps to its own XCD.
inline unsigned stage_grid(const Params &p, int n) {
  if (p.persistent <= 0 || p.n_cu <= 0) return (unsigned)n;
  long long g = (long long)p.persistent * p.n_cu;
  g = (g + 7) / 8 * 8;
  return (unsigned)(g < n ? g : n);
}

// Buffers of one solver touched by the step.  The state lives in three
// rotating buffers (structure of arrays, so a wavefront reads and writes 64
// consecutive elements per array): zeta modes [3][ne] FP64, then momentum
// modes [6][ne] in FP64 or, in the mixed path, FP32.  Each holds a stage
// result BEFORE its limiter and wet/dry post-processing, which the next
// stage applies on the fly.
struct DevState {
  void *buf[3];
  void *wpp;       // post-processed w^n of the current step (RK base), same layout
  double *nodal;   // wind stress (x, y) pairs [nn], then pressure [nn], at the nodes
  double *partial; // [3][nblk] diagnostics partial sums
  double *vb;      // vertex-based limiter: per node range slot (lo, hi) of
                   // the element means of zeta, Qx, Qy (3 double2 per slot)
  Ctrl *ctrl;      // [nmem]
};

// Host-side preprocessing result (internal element order).
struct Prep {
  int nn = 0, ne = 0, ned = 0, nbnd = 0;
  std::vector<int> perm;     // internal element -> caller element
  std::vector<int> iperm;    // caller element -> internal element
  std::vector<double> gx1, gy1, gx2, gy2, area, inr2, hbv;  // hbv [3][ne]
  std::vector<int> el_edge, el_nb, el_node;                  // [3][ne]
  std::vector<int> ed_ep, ed_em, ed_info;
  std::vector<double> ed_nx, ed_ny, ed_hlen;
  std::vector<double> node_x, node_y;
  // chunks of C consecutive elements with their halos (fused stage kernel)
  int C = 0, nch = 0, nl_max = 0, nm_max = 0, ed_max = 0, n2_max = 0;
  std::vector<int> ch_off, h1_off, h1, h2_off, h2, le_off, le_gid, lo_off;
  std::vector<double> le_nx, le_ny, le_hl;                // per local edge
  // p = 2 extras (see DevMesh): mean bathymetry, global ids of each local edge's sides
  std::vector<double> hmean;
  std::vector<int2> le_g;                                  // per local edge: global (e+, e-)
  std::vector<uint32_t> le_ids;                            // packed ids (see DevMesh)
  std::vector<uint16_t> el_ledge;                          // [3][ne] local edge code per local edge
  // packed records (see DevMesh)
  std::vector<double2> eg1, eg2, eai, lhb01, le_a, le_b;
  std::vector<float4> egf, le_f;
  std::vector<int4> enode;
  std::vector<int> lgid;
  std::vector<double> lhb2;
  std::vector<unsigned long long> lnb;
};

// The per-chunk records of the stage kernel from a (merged) mesh and the
// member of each chunk.
void chunk_records(const Prep &P, const std::vector<int> &chunk_member, std::vector<int> &rec);

// Split the (Hilbert-ordered) elements into chunks of C and build, per chunk:
// the ring-1 halo (neighbours outside the chunk), the ring-2 halo
// (neighbours of ring 1 outside chunk and ring 1), the chunk-local edge list
// and local neighbour / edge indices, and the packed records of the stage
// kernel.  Local element index space of a chunk: [0, Cc) chunk elements,
// then ring 1, then ring 2.  Requires C <= 256 (12-bit local ids, 10-bit
// local edge codes).
void build_chunks(Prep &P, int C);

// The p = 2 per-element mean bathymetry (hmean) and the global ids of the
// two sides of each local edge (le_g).
void p2_records(Prep &P);

// Returns 0 on success, else a DGSWE status code with a message in `err`.
int prepare_mesh(int nn, const double *xy, const double *hb, int ne, const int *tri, int nbnd,
                 const int *bnd, const int *btype, Prep &out, std::string &err);

// Kernel launchers (dgswe_kernels.hip).  Each returns hipGetLastError().
// Holland forcing at the stage time for the nodes of every member with a
// moving vortex (nfblk = the total number of forcing blocks).
hipError_t launch_forcing(const DevMesh &m, const DevState &s, const Params &p, int nfblk, int slot, double c,
                          hipStream_t st);
// One RK stage of every member: post-process `win` (where the member's
// control block asks for it), edge fluxes, area integrals, gather, RK
// combination `sc`; writes the unlimited result to `wout`.  The first stage
// (first != 0) also writes the post-processed input to `wpp`; later stages
// with sc.a != 0 read it back as the RK base `wbase`.  `precision` is
// DGSWE_FP64 or DGSWE_MIXED (state buffer layout and kernels).
hipError_t launch_stage(const DevMesh &m, const DevState &s, const Params &p, const void *win,
                        const void *wbase, void *wout, void *wpp, int slot, int first, const StageCoef &sc,
                        int want_dt, int block, int precision, hipStream_t st);
// thread-block sizes the stage kernel is built for
constexpr int kStageBlocks[] = {256};
// Elements [e0, e0 + count) of a state as FP64 [9][count] (post-processed if
// pp), e.g. to read a member back.
// The vertex bounds of the limiter (limiter = 2) from the unlimited state win.
hipError_t launch_vbounds(const DevMesh &m, const DevState &s, const void *win, int precision, hipStream_t st);
// perm != nullptr: element e0 + i goes to column perm[e0 + i] (the caller's
// order) instead of i.
hipError_t launch_post_only(const DevMesh &m, const DevState &s, const Params &p, const void *win, int pp, int e0, int count,
                            double *wout, const int *perm, int precision, hipStream_t st);
// Reset member `mb`'s control block to time t (both parities; pp_in: the
// stored state still needs post-processing) and put the CFL candidates of
// its elements [e0, e0 + count) in `w` into dtmin[slot].
hipError_t launch_init_state(const DevMesh &m, const DevState &s, const Params &p, const void *w, int mb, int e0,
                             int count, double t, int slot, int pp_in, int precision, int order, hipStream_t st);
// mass, volume and wet count of elements [e0, e0 + count) of a state (its
// zeta block is read) into out4[0..2]; partial: 3 diag_blocks(count)
// doubles of per-block partial sums
hipError_t launch_diag(const DevMesh &m, const Params &p, const void *w, int e0, int count, double *partial,
                       double *out4, hipStream_t st);
// the diagnostics of one member as 8 doubles (t, dt_last, mass, volume,
// steps, n_wet, n_dry, status) from its control block (time of parity
// slot) and the sums launch_diag left in sums3
hipError_t launch_diag_pack(const Ctrl *ctl, int slot, int count, const double *sums3, double *out8,
                            hipStream_t st);
// p = 2: post-processing of a stage input (raw state, structure of arrays)
// into element records (the first stage also checks the time step and resets
// the next CFL minimum), then the RK stage from those records (and, in the
// second stage, the first stage's records as the RK base).
hipError_t launch_pp2(const DevMesh &m, const DevState &s, const Params &p, const void *win, void *rec, int slot,
                      int stage, int precision, hipStream_t st);
hipError_t launch_rhs2(const DevMesh &m, const DevState &s, const Params &p, const void *rec, const void *rbase,
                       void *wout, int slot, int first, const StageCoef &sc, int want_dt, int precision,
                       hipStream_t st);
// One RK stage of a p = 1 batch (buffers as launch_stage) and a p = 2
// batch (records of its stage input made by launch_pp2, RK base records,
// raw output) in one launch; sc is the stage of both.
hipError_t launch_stage12(const DevMesh &m1, const DevState &s1, const Params &p1, const void *win1,
                          const void *wbase1, void *wout1, void *wpp1, int slot1, int want_dt1, const DevMesh &m2,
                          const DevState &s2, const Params &p2, const void *rec2, const void *base2, void *wout2,
                          int slot2, int want_dt2, int first, const StageCoef &sc, int precision, hipStream_t st);
// The p = 1 stage of a p = 1 batch together with the post-processing of a
// p = 2 batch's stage input into records (k_pp2's work) in one launch.
hipError_t launch_stage1pp2(const DevMesh &m1, const DevState &s1, const Params &p1, const void *win1,
                            const void *wbase1, void *wout1, void *wpp1, int slot1, int want_dt1, const DevMesh &m2,
                            const DevState &s2, const Params &p2, const void *win2, void *rec2, int slot2, int first,
                            const StageCoef &sc, int precision, hipStream_t st);
// p = 2 read-back: elements [e0, e0 + count) as FP64 [18][count] (perm as
// for launch_post_only)
hipError_t launch_post_only2(const DevMesh &m, const Params &p, const void *win, int pp, int e0, int count,
                             double *wout, const int *perm, int precision, hipStream_t st);
size_t stage_lds_bytes(const DevMesh &m, int precision);
// LDS one stage-kernel workgroup may use (two workgroups share a CU's 160 KB)
constexpr size_t kStageLdsMax = 80 * 1024;
// LDS of a gfx950 compute unit, and the workgroups of the p = 1 stage kernel
// its registers allow per CU (164 VGPRs in FP64: 3 waves per SIMD; 124 in
// mixed precision: 4); kLdsSlack covers the kernel's static LDS and the
// allocation granularity
constexpr size_t kLdsPerCu = 160 * 1024;
constexpr int kStageWgPerCuFp64 = 3, kStageWgPerCuMixed = 4;
constexpr size_t kLdsSlack = 1024;
// bytes of one state buffer: (3 zeta modes FP64 + 6 momentum modes) per
// element at p = 1, (6 + 12) at p = 2
size_t state_bytes(size_t ne, int precision, int order);
bool stage_block_ok(int block);
int diag_blocks(int ne);

}  // namespace dgswe
