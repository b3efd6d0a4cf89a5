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
struct Ctrl {
  double t;                      // model time at the start of the current step
  double dt_last;                // dt of the last completed step
  unsigned long long dtmin[2];   // bit pattern of the raw CFL minimum, per step parity
  long long steps;               // completed steps
  int status;                    // first error detected on the device (0 = none)
  int pad;
};

// Element-major structure-of-arrays mesh on the device (internal order).
struct DevMesh {
  int ne, nn, ned;
  // elements
  const double *gx1, *gy1, *gx2, *gy2;  // physical gradients of phi_10, phi_01
  const double *area;                   // A_e
  const double *inr2;                   // 2 x inradius
  const double *hbv;                    // [3][ne] bathymetry at the element's vertices
  const int *el_edge;                   // [3][ne] edge id << 1 | side (0 = e+, 1 = e-)
  const int *el_nb;                     // [3][ne] neighbour across local edge, -1 none
  const int *el_node;                   // [3][ne] node ids
  const double *manning;                // [ne] or nullptr
  // edges (sorted by e+)
  const int *ed_ep, *ed_em;             // elements; em = -1 on the boundary
  const int *ed_info;                   // lp | lm << 2 | type << 4
  const double *ed_nx, *ed_ny, *ed_hlen;  // unit normal from e+, half length
  // nodes
  const double *node_x, *node_y;
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

// Buffers of one solver touched by the step.
struct DevState {
  double *w0;      // [9][ne] state w^n (after post-processing)
  double *w1;      // [9][ne] first-stage state (after post-processing)
  double *wt;      // [9][ne] unlimited RK combination of the current stage
  unsigned char *wet;  // [ne] wet flag of the current stage input
  double *edge;    // [6][ned] edge flux moments
  unsigned char *emode;  // [ned] which sides receive the edge flux
  double *nodal;   // [3][nn] wind stress x, y and pressure at the nodes
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
};

// Returns 0 on success, else a DGSWE status code with a message in `err`.
int prepare_mesh(int nn, const double *xy, const double *hb, int ne, const int *tri, int nbnd,
                 const int *bnd, const int *btype, Prep &out, std::string &err);

// Kernel launchers (dgswe_kernels.hip).  Each returns hipGetLastError().
hipError_t launch_forcing(const DevMesh &m, const DevState &s, const Params &p, int slot, int stage,
                          hipStream_t st);
hipError_t launch_edge(const DevMesh &m, const DevState &s, const Params &p, const double *w,
                       int slot, int stage, hipStream_t st);
hipError_t launch_element(const DevMesh &m, const DevState &s, const Params &p, const double *w,
                          const double *wbase, int slot, int stage, hipStream_t st);
hipError_t launch_post(const DevMesh &m, const DevState &s, const Params &p, double *wout,
                       int slot, int stage, int want_dt, hipStream_t st);
hipError_t launch_post_only(const DevMesh &m, const DevState &s, const Params &p, double *wout,
                            hipStream_t st);
hipError_t launch_init_state(const DevMesh &m, const DevState &s, const Params &p, int slot,
                             double t, hipStream_t st);
hipError_t launch_diag(const DevMesh &m, const DevState &s, const Params &p, double *out4,
                       hipStream_t st);
int diag_blocks(int ne);

}  // namespace dgswe
