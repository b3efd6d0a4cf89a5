// Host-side preprocessing of a triangle mesh for the gfx950 step:
// validation, locality reordering of elements along a Hilbert curve, the
// edge table (each edge once, oriented from its lower-numbered element),
// per-element geometry and the element -> edge / neighbour / node tables.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>

#include "dgswe_internal.h"
#include "../../include/dgswe.h"

namespace dgswe {
namespace {

// Index of cell (x, y) along a Hilbert curve filling a 2^order x 2^order grid.
// Each level picks the quadrant (visiting order 0: lower-left, 1: upper-left,
// 2: upper-right, 3: lower-right) and reflects/transposes the coordinates so
// that the sub-curve inside the quadrant starts and ends at the right corners.
uint64_t hilbert_index(int order, uint32_t x, uint32_t y) {
  uint64_t d = 0;
  for (int lvl = order - 1; lvl >= 0; --lvl) {
    const uint32_t half = 1u << lvl;
    const uint32_t rx = (x & half) ? 1u : 0u;
    const uint32_t ry = (y & half) ? 1u : 0u;
    d += (uint64_t)half * half * ((3u * rx) ^ ry);
    const uint32_t mask = (half << 1) - 1u;
    x &= mask >> 1;
    y &= mask >> 1;
    if (ry == 0) {
      if (rx == 1) {
        x = (half - 1u) - x;
        y = (half - 1u) - y;
      }
      std::swap(x, y);
    }
  }
  return d;
}

struct HalfEdge {
  uint64_t key;
  int e, l;
};

}  // namespace

int prepare_mesh(int nn, const double *xy, const double *hb, int ne, const int *tri, int nbnd,
                 const int *bnd, const int *btype, Prep &P, std::string &err) {
  if (nn <= 0 || ne <= 0 || nbnd < 0 || !xy || !hb || !tri || (nbnd > 0 && (!bnd || !btype))) {
    err = "invalid mesh arguments";
    return DGSWE_E_INVALID;
  }
  for (int i = 0; i < nbnd; ++i) {
    if (btype[i] == DGSWE_BC_RIVER) {
      err = "river boundaries are not supported";
      return DGSWE_E_INVALID;
    }
    if (btype[i] != DGSWE_BC_LAND && btype[i] != DGSWE_BC_OCEAN) {
      err = "unknown boundary type";
      return DGSWE_E_MESH;
    }
  }
  for (int i = 0; i < nn; ++i)
    if (!std::isfinite(xy[2 * i]) || !std::isfinite(xy[2 * i + 1]) || !std::isfinite(hb[i])) {
      err = "node " + std::to_string(i) + " has a non-finite coordinate or bathymetry";
      return DGSWE_E_MESH;
    }
  for (int64_t i = 0; i < 3LL * ne; ++i)
    if (tri[i] < 0 || tri[i] >= nn) {
      err = "triangle node index out of range";
      return DGSWE_E_MESH;
    }
  for (int e = 0; e < ne; ++e) {
    const int *v = tri + 3 * e;
    double ax = xy[2 * v[1]] - xy[2 * v[0]], ay = xy[2 * v[1] + 1] - xy[2 * v[0] + 1];
    double bx = xy[2 * v[2]] - xy[2 * v[0]], by = xy[2 * v[2] + 1] - xy[2 * v[0] + 1];
    if (!(ax * by - bx * ay > 0.0)) {
      err = "triangle " + std::to_string(e) + " is not counter-clockwise with positive area";
      return DGSWE_E_MESH;
    }
  }
  P.nn = nn;
  P.ne = ne;

  // --- Hilbert order of the element centroids
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  for (int i = 0; i < nn; ++i) {
    xmin = std::min(xmin, xy[2 * i]); xmax = std::max(xmax, xy[2 * i]);
    ymin = std::min(ymin, xy[2 * i + 1]); ymax = std::max(ymax, xy[2 * i + 1]);
  }
  const int order = 20;
  const double span = std::max(xmax - xmin, ymax - ymin);
  const double scale = span > 0 ? ((double)((1u << order) - 1u)) / span : 0.0;
  std::vector<uint64_t> key(ne);
  for (int e = 0; e < ne; ++e) {
    const int *v = tri + 3 * e;
    double cx = (xy[2 * v[0]] + xy[2 * v[1]] + xy[2 * v[2]]) / 3.0;
    double cy = (xy[2 * v[0] + 1] + xy[2 * v[1] + 1] + xy[2 * v[2] + 1]) / 3.0;
    key[e] = hilbert_index(order, (uint32_t)((cx - xmin) * scale), (uint32_t)((cy - ymin) * scale));
  }
  P.perm.resize(ne);
  std::iota(P.perm.begin(), P.perm.end(), 0);
  std::stable_sort(P.perm.begin(), P.perm.end(), [&](int a, int b) { return key[a] < key[b]; });
  P.iperm.resize(ne);
  for (int i = 0; i < ne; ++i) P.iperm[P.perm[i]] = i;

  // --- edges from half-edges sorted by their node pair
  std::vector<HalfEdge> he(3 * (size_t)ne);
  for (int i = 0; i < ne; ++i) {
    const int *v = tri + 3 * (size_t)P.perm[i];
    for (int l = 0; l < 3; ++l) {
      uint64_t a = (uint64_t)v[(l + 1) % 3], b = (uint64_t)v[(l + 2) % 3];
      he[3 * (size_t)i + l] = {std::min(a, b) * (uint64_t)nn + std::max(a, b), i, l};
    }
  }
  std::sort(he.begin(), he.end(), [](const HalfEdge &a, const HalfEdge &b) {
    return a.key != b.key ? a.key < b.key : a.e < b.e;
  });
  std::vector<std::pair<uint64_t, int>> bkeys(nbnd);
  for (int i = 0; i < nbnd; ++i) {
    int a = bnd[2 * i], b = bnd[2 * i + 1];
    if (a < 0 || a >= nn || b < 0 || b >= nn || a == b) {
      err = "boundary edge node index out of range";
      return DGSWE_E_MESH;
    }
    bkeys[i] = {(uint64_t)std::min(a, b) * (uint64_t)nn + (uint64_t)std::max(a, b), btype[i]};
  }
  std::sort(bkeys.begin(), bkeys.end());
  for (int i = 1; i < nbnd; ++i)
    if (bkeys[i].first == bkeys[i - 1].first) {
      err = "boundary edge listed twice";
      return DGSWE_E_MESH;
    }
  struct Edge { int ep, lp, em, lm, type; };
  std::vector<Edge> edges;
  edges.reserve(3 * (size_t)ne / 2 + 64);
  int nb_found = 0;
  for (size_t i = 0; i < he.size();) {
    size_t j = i + 1;
    while (j < he.size() && he[j].key == he[i].key) ++j;
    if (j - i > 2) {
      err = "edge shared by more than two triangles";
      return DGSWE_E_MESH;
    }
    Edge E{he[i].e, he[i].l, -1, -1, 0};
    if (j - i == 2) {
      E.em = he[i + 1].e;
      E.lm = he[i + 1].l;
    } else {
      auto it = std::lower_bound(bkeys.begin(), bkeys.end(), std::make_pair(he[i].key, -1));
      if (it == bkeys.end() || it->first != he[i].key) {
        err = "boundary edge without a type";
        return DGSWE_E_MESH;
      }
      E.type = it->second;
      ++nb_found;
    }
    edges.push_back(E);
    i = j;
  }
  if (nb_found != nbnd) {
    err = "a listed boundary edge is not on the mesh boundary";
    return DGSWE_E_MESH;
  }
  std::sort(edges.begin(), edges.end(), [](const Edge &a, const Edge &b) {
    return a.ep != b.ep ? a.ep < b.ep : a.lp < b.lp;
  });
  const int ned = (int)edges.size();
  P.ned = ned;
  P.nbnd = nbnd;

  // --- per-element geometry (internal order)
  P.gx1.resize(ne); P.gy1.resize(ne); P.gx2.resize(ne); P.gy2.resize(ne);
  P.area.resize(ne); P.inr2.resize(ne); P.hbv.resize(3 * (size_t)ne);
  P.el_edge.assign(3 * (size_t)ne, -1); P.el_nb.assign(3 * (size_t)ne, -1);
  P.el_node.resize(3 * (size_t)ne);
  for (int i = 0; i < ne; ++i) {
    const int *v = tri + 3 * (size_t)P.perm[i];
    double X[3], Y[3];
    for (int k = 0; k < 3; ++k) {
      X[k] = xy[2 * v[k]];
      Y[k] = xy[2 * v[k] + 1];
      P.hbv[(size_t)k * ne + i] = hb[v[k]];
      P.el_node[(size_t)k * ne + i] = v[k];
    }
    double A = 0.5 * ((X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]));
    // barycentric gradients grad lambda_k = (y_{k+1} - y_{k+2}, x_{k+2} - x_{k+1}) / 2A
    double lx[3], ly[3];
    for (int k = 0; k < 3; ++k) {
      int a = (k + 1) % 3, b = (k + 2) % 3;
      lx[k] = (Y[a] - Y[b]) / (2.0 * A);
      ly[k] = (X[b] - X[a]) / (2.0 * A);
    }
    // phi_10 = lambda_1 - lambda_0, phi_01 = 2 lambda_2 - lambda_0 - lambda_1
    P.gx1[i] = lx[1] - lx[0];
    P.gy1[i] = ly[1] - ly[0];
    P.gx2[i] = 2.0 * lx[2] - lx[0] - lx[1];
    P.gy2[i] = 2.0 * ly[2] - ly[0] - ly[1];
    P.area[i] = A;
    double per = std::hypot(X[1] - X[2], Y[1] - Y[2]) + std::hypot(X[2] - X[0], Y[2] - Y[0]) +
                 std::hypot(X[0] - X[1], Y[0] - Y[1]);
    P.inr2[i] = 4.0 * A / per;
  }
  P.ed_ep.resize(ned); P.ed_em.resize(ned); P.ed_info.resize(ned);
  P.ed_nx.resize(ned); P.ed_ny.resize(ned); P.ed_hlen.resize(ned);
  for (int d = 0; d < ned; ++d) {
    const Edge &E = edges[d];
    P.ed_ep[d] = E.ep;
    P.ed_em[d] = E.em;
    P.ed_info[d] = E.lp | ((E.lm < 0 ? 0 : E.lm) << 2) | (E.type << 4);
    const int *v = tri + 3 * (size_t)P.perm[E.ep];
    int na = v[(E.lp + 1) % 3], nb = v[(E.lp + 2) % 3];
    double dx = xy[2 * nb] - xy[2 * na], dy = xy[2 * nb + 1] - xy[2 * na + 1];
    double len = std::hypot(dx, dy);
    P.ed_nx[d] = dy / len;
    P.ed_ny[d] = -dx / len;
    P.ed_hlen[d] = 0.5 * len;
    P.el_edge[(size_t)E.lp * ne + E.ep] = d << 1;
    if (E.em >= 0) {
      P.el_edge[(size_t)E.lm * ne + E.em] = (d << 1) | 1;
      P.el_nb[(size_t)E.lp * ne + E.ep] = E.em;
      P.el_nb[(size_t)E.lm * ne + E.em] = E.ep;
    }
  }
  P.node_x.resize(nn);
  P.node_y.resize(nn);
  for (int i = 0; i < nn; ++i) {
    P.node_x[i] = xy[2 * i];
    P.node_y[i] = xy[2 * i + 1];
  }
  return DGSWE_OK;
}

namespace {
double bits_as_double(uint32_t v) {
  const uint64_t u = v;
  double d;
  std::memcpy(&d, &u, sizeof d);
  return d;
}
float bits_as_float(uint32_t v) {
  float f;
  std::memcpy(&f, &v, sizeof f);
  return f;
}
}  // namespace

void build_chunks(Prep &P, int C) {
  const int ne = P.ne;
  const size_t nes = (size_t)ne;
  P.C = C;
  P.nch = (ne + C - 1) / C;
  P.ch_off.assign(P.nch + 1, 0);
  P.h1_off.assign(P.nch + 1, 0);
  P.h2_off.assign(P.nch + 1, 0);
  P.le_off.assign(P.nch + 1, 0);
  P.lo_off.assign(P.nch + 1, 0);
  P.h1.clear(); P.h2.clear(); P.le_gid.clear(); P.le_ids.clear();
  P.le_nx.clear(); P.le_ny.clear(); P.le_hl.clear();
  P.lhb01.clear(); P.lhb2.clear(); P.lnb.clear(); P.lgid.clear();
  P.el_ledge.assign(3 * nes, 0);
  P.nl_max = P.nm_max = P.ed_max = P.n2_max = 0;
  std::vector<int> loc(nes, -1);       // global element -> local index in the current chunk
  std::vector<int> eloc(P.ned, -1);    // global edge -> local edge index in the current chunk
  std::vector<int> h1, h2, edges;
  for (int c = 0; c < P.nch; ++c) {
    const int c0 = c * C, cc = std::min(C, ne - c0);
    for (int i = 0; i < cc; ++i) loc[c0 + i] = i;
    h1.clear();
    for (int i = 0; i < cc; ++i)
      for (int l = 0; l < 3; ++l) {
        int f = P.el_nb[(size_t)l * nes + c0 + i];
        if (f >= 0 && loc[f] < 0) { loc[f] = -2; h1.push_back(f); }
      }
    std::sort(h1.begin(), h1.end());
    for (size_t k = 0; k < h1.size(); ++k) loc[h1[k]] = cc + (int)k;
    const int nl = cc + (int)h1.size();
    h2.clear();
    for (int f : h1)
      for (int l = 0; l < 3; ++l) {
        int g = P.el_nb[(size_t)l * nes + f];
        if (g >= 0 && loc[g] == -1) { loc[g] = -3; h2.push_back(g); }
      }
    std::sort(h2.begin(), h2.end());
    for (size_t k = 0; k < h2.size(); ++k) loc[h2[k]] = nl + (int)k;
    const int nm = nl + (int)h2.size();
    // local elements (chunk + ring 1): vertex bathymetry and local neighbours
    P.lo_off[c] = (int)P.lnb.size();
    for (int i = 0; i < nl; ++i) {
      const int g = i < cc ? c0 + i : h1[i - cc];
      P.lgid.push_back(g);
      P.lhb01.push_back(make_double2(P.hbv[g], P.hbv[nes + g]));
      P.lhb2.push_back(P.hbv[2 * nes + g]);
      unsigned long long nbw = 0;
      for (int l = 0; l < 3; ++l) {
        const int f = P.el_nb[(size_t)l * nes + g];
        const unsigned long long v = f < 0 ? 0xFFFFull : (unsigned long long)loc[f];
        nbw |= v << (16 * l);
      }
      P.lnb.push_back(nbw);
    }
    // chunk-local edges: every edge of a chunk element, once
    edges.clear();
    for (int i = 0; i < cc; ++i)
      for (int l = 0; l < 3; ++l) {
        int d = P.el_edge[(size_t)l * nes + c0 + i] >> 1;
        if (eloc[d] < 0) { eloc[d] = 0; edges.push_back(d); }
      }
    std::sort(edges.begin(), edges.end());
    P.le_off[c] = (int)P.le_gid.size();
    for (size_t k = 0; k < edges.size(); ++k) {
      int d = edges[k];
      eloc[d] = (int)k;
      P.le_gid.push_back(d);
      const uint32_t ip = (uint32_t)loc[P.ed_ep[d]];
      const uint32_t im = P.ed_em[d] < 0 ? 0u : (uint32_t)loc[P.ed_em[d]];
      P.le_ids.push_back(ip | (im << 12) | ((uint32_t)P.ed_info[d] << 24));
      P.le_nx.push_back(P.ed_nx[d]);
      P.le_ny.push_back(P.ed_ny[d]);
      P.le_hl.push_back(P.ed_hlen[d]);
    }
    for (int i = 0; i < cc; ++i)
      for (int l = 0; l < 3; ++l) {
        int code = P.el_edge[(size_t)l * nes + c0 + i];
        P.el_ledge[(size_t)l * nes + c0 + i] = (uint16_t)((eloc[code >> 1] << 1) | (code & 1));
      }
    P.ch_off[c] = c0;
    P.h1_off[c] = (int)P.h1.size();
    P.h1.insert(P.h1.end(), h1.begin(), h1.end());
    P.h2_off[c] = (int)P.h2.size();
    P.h2.insert(P.h2.end(), h2.begin(), h2.end());
    P.nl_max = std::max(P.nl_max, nl);
    P.nm_max = std::max(P.nm_max, nm);
    P.ed_max = std::max(P.ed_max, (int)edges.size());
    P.n2_max = std::max(P.n2_max, (int)h2.size());
    // reset the scratch maps
    for (int i = 0; i < cc; ++i) loc[c0 + i] = -1;
    for (int f : h1) loc[f] = -1;
    for (int g : h2) loc[g] = -1;
    for (int d : edges) eloc[d] = -1;
  }
  P.ch_off[P.nch] = ne;
  P.h1_off[P.nch] = (int)P.h1.size();
  P.h2_off[P.nch] = (int)P.h2.size();
  P.le_off[P.nch] = (int)P.le_gid.size();
  P.lo_off[P.nch] = (int)P.lnb.size();
  // one sentinel entry (element 0) past the end of the ring-2 list: the
  // stage kernel reads a clamped ring-2 position unconditionally, also for a
  // chunk without ring 2, and stores only the entries that exist
  P.h2.push_back(0);
  // packed records of the stage kernel
  const size_t nle = P.le_gid.size();
  P.le_a.resize(nle); P.le_b.resize(nle); P.le_f.resize(nle);
  for (size_t r = 0; r < nle; ++r) {
    P.le_a[r] = make_double2(P.le_nx[r], P.le_ny[r]);
    P.le_b[r] = make_double2(P.le_hl[r], bits_as_double(P.le_ids[r]));
    P.le_f[r] = make_float4((float)P.le_nx[r], (float)P.le_ny[r], (float)P.le_hl[r], bits_as_float(P.le_ids[r]));
  }
  P.eg1.resize(nes); P.eg2.resize(nes); P.egf.resize(nes); P.eai.resize(nes); P.enode.resize(nes);
  for (size_t e = 0; e < nes; ++e) {
    P.eg1[e] = make_double2(P.gx1[e], P.gy1[e]);
    P.eg2[e] = make_double2(P.gx2[e], P.gy2[e]);
    P.egf[e] = make_float4((float)P.gx1[e], (float)P.gy1[e], (float)P.gx2[e], (float)P.gy2[e]);
    P.eai[e] = make_double2(P.area[e], P.inr2[e]);
    const int codes = (int)P.el_ledge[e] | ((int)P.el_ledge[nes + e] << 10) | ((int)P.el_ledge[2 * nes + e] << 20);
    P.enode[e] = make_int4(P.el_node[e], P.el_node[nes + e], P.el_node[2 * nes + e], codes);
  }
}

}  // namespace dgswe

namespace dgswe {

void p2_records(Prep &P) {
  const size_t ne = (size_t)P.ne;
  P.hmean.resize(ne);
  for (size_t e = 0; e < ne; ++e) P.hmean[e] = (P.hbv[e] + P.hbv[ne + e] + P.hbv[2 * ne + e]) / 3.0;
  P.le_g.resize(P.le_gid.size());
  for (size_t r = 0; r < P.le_gid.size(); ++r) {
    const int d = P.le_gid[r];
    P.le_g[r] = make_int2(P.ed_ep[d], P.ed_em[d] < 0 ? P.ed_ep[d] : P.ed_em[d]);
  }
}

void chunk_records(const Prep &P, const std::vector<int> &chunk_member, std::vector<int> &rec) {
  rec.assign((size_t)P.nch * kChunkRec, 0);
  for (int c = 0; c < P.nch; ++c) {
    int *r = &rec[(size_t)c * kChunkRec];
    r[0] = P.ch_off[c];
    r[1] = P.ch_off[c + 1] - P.ch_off[c];
    r[2] = P.h1_off[c];
    r[3] = P.h1_off[c + 1] - P.h1_off[c];
    r[4] = P.h2_off[c];
    r[5] = P.h2_off[c + 1] - P.h2_off[c];
    r[6] = P.le_off[c];
    r[7] = P.le_off[c + 1] - P.le_off[c];
    r[8] = P.lo_off[c];
    r[9] = chunk_member[c];
    r[10] = (c == 0 || chunk_member[c - 1] != chunk_member[c]) ? 1 : 0;
    r[11] = P.ne + chunk_member[c];  // uniform Manning n of the member
    r[12] = 0;
  }
}

}  // namespace dgswe
