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

// Device control block: one per solver, read by every kernel of a step.
// Step n (counted from dgswe_set_state) reads t[n & 1] and dtmin[n & 1];
// its last kernel writes t[(n + 1) & 1] and the CFL candidates of step n + 1
// into dtmin[(n + 1) & 1], so no kernel writes a value another block of the
// same kernel reads.
struct Ctrl {
  double t[2];                   // model time at the start of a step, per parity
  double dt_last;                // dt of the last completed step
  unsigned long long dtmin[2];   // bit pattern of the raw CFL minimum, per parity
  long long steps;               // completed steps
  int status;                    // first error detected on the device (0 = none)
  int pad;
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
  const double *manning;                // Manning n of element e at manning[e * manning_step]
  const float *manningf;                // the same in FP32 (mixed path)
  int manning_step;                     // 1: per element, 0: one uniform value
  // nodes
  const double *node_x, *node_y;
  // chunks of the stage kernel (see build_chunks)
  int C, nch, nl_max, nm_max, ed_max, n2_max;
  const int *h1_off, *h2_off, *h2;       // per-chunk ring-1 counts, ring-2 element ids
  const int *le_off, *lo_off;            // per-chunk offsets of local edges / local elements
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
};

struct Params {
  double g, rho0, h0, cfl, dt_fixed, dt_max;
  int limiter, wetdry;
  double manning_n;
  int n_tide;
  double tide_amp[kMaxTide], tide_omega[kMaxTide], tide_phase[kMaxTide], tide_offset;
  int holland;
  double x0, y0, vx, vy, dp, pn, rmax, B, rho_air, coriolis_f, wind_factor;
};

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
  Ctrl *ctrl;
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
  std::vector<int> h1_off, h1, h2_off, h2, le_off, le_gid, lo_off;
  std::vector<double> le_nx, le_ny, le_hl;                // per local edge
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

// Split the (Hilbert-ordered) elements into chunks of C and build, per chunk:
// the ring-1 halo (neighbours outside the chunk), the ring-2 halo
// (neighbours of ring 1 outside chunk and ring 1), the chunk-local edge list
// and local neighbour / edge indices, and the packed records of the stage
// kernel.  Local element index space of a chunk: [0, Cc) chunk elements,
// then ring 1, then ring 2.  Requires C <= 256 (12-bit local ids, 10-bit
// local edge codes).
void build_chunks(Prep &P, int C);

// Returns 0 on success, else a DGSWE status code with a message in `err`.
int prepare_mesh(int nn, const double *xy, const double *hb, int ne, const int *tri, int nbnd,
                 const int *bnd, const int *btype, Prep &out, std::string &err);

// Kernel launchers (dgswe_kernels.hip).  Each returns hipGetLastError().
hipError_t launch_forcing(const DevMesh &m, const DevState &s, const Params &p, int slot, int stage,
                          hipStream_t st);
// One RK stage: post-process `win` (if pp_in), edge fluxes, area integrals,
// gather, RK combination; writes the unlimited result to `wout`.  The first
// stage (stage 0) also writes the post-processed input to `wpp`; the second
// stage reads it back as the RK base `wbase`.
// `precision` is DGSWE_FP64 or DGSWE_MIXED (state buffer layout and kernels).
hipError_t launch_stage(const DevMesh &m, const DevState &s, const Params &p, const void *win,
                        const void *wbase, void *wout, void *wpp, int slot, int stage, int pp_in,
                        int want_dt, int block, int precision, hipStream_t st);
// thread-block sizes the stage kernel is built for
constexpr int kStageBlocks[] = {256};
// A whole state as FP64 [9][ne] (post-processed if pp), e.g. to read it back.
hipError_t launch_post_only(const DevMesh &m, const Params &p, const void *win, int pp, double *wout,
                            int precision, hipStream_t st);
// Reset the control block to time t and put the CFL candidates of `w`
// into dtmin[0].
hipError_t launch_init_state(const DevMesh &m, const DevState &s, const Params &p, const void *w,
                             double t, int precision, hipStream_t st);
// mass, volume and wet count of a state (its zeta block is read)
hipError_t launch_diag(const DevMesh &m, const DevState &s, const Params &p, const void *w,
                       double *out4, hipStream_t st);
size_t stage_lds_bytes(const DevMesh &m, int precision);
size_t state_bytes(size_t ne, int precision);
bool stage_block_ok(int block);
int diag_blocks(int ne);

}  // namespace dgswe
