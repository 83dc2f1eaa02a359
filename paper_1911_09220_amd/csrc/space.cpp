// Mesh topology and the H1 finite element space (host).
//
// Builds the element restriction G of "Operator Decomposition" as an
// element->dof table in lexicographic local order.  Global numbering follows
// "Finite Element Spaces": vertex dofs, then edge dofs (each edge traversed
// in a fixed direction), then face dofs (each face in a fixed orientation),
// then element interiors.  The fixed direction of an edge runs from its
// smaller to its larger vertex id; the fixed frame of a face has its origin at
// the face's smallest vertex id, first axis towards the adjacent corner with
// the smaller id.  Every element maps its local edge/face nodes into that frame,
// which is the orientation permutation of "Finite Elements"
// (FiniteElementCollection).
//
// Edges and faces are matched by bucketing them by their smallest vertex and
// comparing within buckets (no hashing).  A face seen once is a boundary face;
// every dof on a boundary face is essential.
#include <algorithm>
#include <array>
#include <atomic>
#include <cstring>
#include <numeric>

#include "internal.hpp"

namespace pafem {

namespace {

// lexicographic corner c = cx + 2 cy + 4 cz -> slot in the usual hex vertex order
constexpr int kLexToSlot[8] = {0, 1, 3, 2, 4, 5, 7, 6};

struct ElemCorners {
  int64_t v[8];
};

inline ElemCorners corners_of(const Mesh& m, int64_t e) {
  ElemCorners c;
  for (int k = 0; k < 8; ++k) c.v[k] = m.hex[size_t(e) * 8 + kLexToSlot[k]];
  return c;
}

// 12 edges: (axis, low corner) pairs with bit `axis` of the corner clear
struct EdgeSlot {
  int axis, c0;
};
std::array<EdgeSlot, 12> edge_slots() {
  std::array<EdgeSlot, 12> out{};
  int k = 0;
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 8; ++c)
      if (!((c >> a) & 1)) out[k++] = {a, c};
  return out;
}

// 6 faces: axis a, side s; corners with bit a == s
struct FaceSlot {
  int axis, side, c[4];
};
std::array<FaceSlot, 6> face_slots() {
  std::array<FaceSlot, 6> out{};
  int k = 0;
  for (int a = 0; a < 3; ++a)
    for (int s = 0; s < 2; ++s) {
      FaceSlot f{a, s, {0, 0, 0, 0}};
      int n = 0;
      for (int c = 0; c < 8; ++c)
        if (((c >> a) & 1) == s) f.c[n++] = c;
      out[k++] = f;
    }
  return out;
}

// Match items (edges or faces) that carry the same sorted vertex key.  Items are
// bucketed by their first (smallest) key entry.  rep[i] = smallest item index
// with the same key; count[i] = multiplicity of the key.
template <int K>
void match_keys(const std::vector<std::array<int64_t, K>>& keys, int64_t nv,
                std::vector<int64_t>& rep, std::vector<int32_t>& mult) {
  const size_t n = keys.size();
  std::vector<int64_t> off(size_t(nv) + 1, 0);
  for (size_t i = 0; i < n; ++i) off[size_t(keys[i][0]) + 1]++;
  for (int64_t v = 0; v < nv; ++v) off[v + 1] += off[v];
  std::vector<int64_t> items(n);
  {
    std::vector<int64_t> fill(off.begin(), off.end() - 1);
    for (size_t i = 0; i < n; ++i) items[fill[size_t(keys[i][0])]++] = int64_t(i);
  }
  rep.assign(n, -1);
  mult.assign(n, 0);
  for (int64_t v = 0; v < nv; ++v) {
    for (int64_t a = off[v]; a < off[v + 1]; ++a) {
      const int64_t i = items[a];
      if (rep[i] >= 0) continue;
      rep[i] = i;
      int32_t m = 1;
      for (int64_t b = a + 1; b < off[v + 1]; ++b) {
        const int64_t j = items[b];
        if (rep[j] < 0 && keys[j] == keys[i]) {
          rep[j] = i;
          ++m;
        }
      }
      mult[i] = m;
    }
  }
  for (size_t i = 0; i < n; ++i) mult[i] = mult[size_t(rep[i])];
}

// spread the low 21 bits of v so that bit i lands at bit 3i
uint64_t spread3(uint64_t v) {
  v &= 0x1fffff;
  v = (v | (v << 32)) & 0x1f00000000ffffULL;
  v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
  v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
  v = (v | (v << 2)) & 0x1249249249249249ULL;
  return v;
}

// spread the low 31 bits of v so that bit i lands at bit 2i
uint64_t spread2(uint64_t v) {
  v &= 0x7fffffff;
  v = (v | (v << 16)) & 0x0000ffff0000ffffULL;
  v = (v | (v << 8)) & 0x00ff00ff00ff00ffULL;
  v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0fULL;
  v = (v | (v << 2)) & 0x3333333333333333ULL;
  v = (v | (v << 1)) & 0x5555555555555555ULL;
  return v;
}

// Device element order: Morton (Z-curve) order of element centroids.
std::vector<int32_t> morton_order(const Mesh& m) {
  const int64_t ne = m.ne;
  const int dim = m.dim, nvert = dim == 2 ? 4 : 8;
  const std::vector<int64_t>& conn = dim == 2 ? m.quad : m.hex;
  std::vector<double> c(static_cast<size_t>(ne) * 3, 0.0);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t e = 0; e < ne; ++e) {
    for (int k = 0; k < nvert; ++k)
      for (int a = 0; a < dim; ++a)
        c[size_t(e) * 3 + a] += m.xyz[size_t(conn[size_t(e) * nvert + k]) * dim + a];
    for (int a = 0; a < dim; ++a) {
      c[size_t(e) * 3 + a] /= nvert;
      lo[a] = std::min(lo[a], c[size_t(e) * 3 + a]);
      hi[a] = std::max(hi[a], c[size_t(e) * 3 + a]);
    }
  }
  std::vector<std::pair<uint64_t, int32_t>> key(static_cast<size_t>(ne));
  const int bits = dim == 2 ? 31 : 21;
  for (int64_t e = 0; e < ne; ++e) {
    uint64_t code = 0;
    for (int a = 0; a < dim; ++a) {
      const double span = hi[a] - lo[a];
      const double t = span > 0 ? (c[size_t(e) * 3 + a] - lo[a]) / span : 0.0;
      const uint64_t qv = uint64_t(std::min(std::max(t, 0.0), 1.0) * double((uint64_t(1) << bits) - 1));
      code |= (dim == 2 ? spread2(qv) : spread3(qv)) << a;
    }
    key[size_t(e)] = {code, int32_t(e)};
  }
  std::sort(key.begin(), key.end());
  std::vector<int32_t> order(static_cast<size_t>(ne));
  for (int64_t i = 0; i < ne; ++i) order[size_t(i)] = key[size_t(i)].second;
  return order;
}

// Device element order, optional renumbering, apply tiles, the essential list and
// the 1D tables: the same for every dimension once gmap and bmask are set.
void finish_space(Space* s, const Mesh& m, int flags) {
  const int p = s->p, dpe = s->dpe;
  const int64_t ne = s->ne, ndofs = s->ndofs;
  s->dev_order = mesh_element_order(m);
  if (flags & PAFEM_SPACE_RENUMBER) {
    // first touch while walking the elements in device order
    std::vector<int32_t> perm(size_t(ndofs), -1);
    int32_t nn = 0;
    for (int64_t k = 0; k < ne; ++k) {
      const int32_t* g = s->gmap.data() + size_t(s->dev_order[size_t(k)]) * dpe;
      for (int i = 0; i < dpe; ++i)
        if (perm[size_t(g[i])] < 0) perm[size_t(g[i])] = nn++;
    }
    for (auto& d : s->gmap) d = perm[size_t(d)];
    std::vector<uint8_t> bm(static_cast<size_t>(ndofs), 0);
    for (int64_t d = 0; d < ndofs; ++d) bm[size_t(perm[d])] = s->bmask[size_t(d)];
    s->bmask.swap(bm);
  }
  // apply tiles: tile_ne consecutive device elements share one list of unique dofs
  s->tile_ne = s->dim == 2 ? qdata_tile_2d(p + 2) : qdata_tile(p + 2);
  const int64_t ntiles = (ne + s->tile_ne - 1) / s->tile_ne;
  s->tile_off.assign(size_t(ntiles) + 1, 0);
  s->tile_slot.assign(size_t(ntiles) * s->tile_ne * dpe, 0);
  s->tile_dofs.reserve(size_t(ne) * dpe / 2);
  std::vector<int32_t> buf;
  for (int64_t t = 0; t < ntiles; ++t) {
    const int64_t e0 = t * s->tile_ne, e1 = std::min(ne, e0 + s->tile_ne);
    buf.clear();
    for (int64_t k = e0; k < e1; ++k) {
      const int32_t* g = s->gmap.data() + size_t(s->dev_order[size_t(k)]) * dpe;
      buf.insert(buf.end(), g, g + dpe);
    }
    std::sort(buf.begin(), buf.end());
    buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    for (int64_t k = e0; k < e1; ++k) {
      const int32_t* g = s->gmap.data() + size_t(s->dev_order[size_t(k)]) * dpe;
      uint16_t* sl = s->tile_slot.data() + size_t(k) * dpe;
      for (int i = 0; i < dpe; ++i)
        sl[i] = uint16_t(std::lower_bound(buf.begin(), buf.end(), g[i]) - buf.begin());
    }
    for (int32_t d : buf) s->tile_dofs.push_back(s->bmask[size_t(d)] ? ~d : d);
    s->tile_off[size_t(t) + 1] = int32_t(s->tile_dofs.size());
  }
  for (int64_t d = 0; d < ndofs; ++d)
    if (s->bmask[size_t(d)]) s->bdr.push_back(int32_t(d));
  s->tables = build_tables(p, s->ng);
}

// lexicographic corner c = cx + 2 cy -> slot in the counter-clockwise quad order
constexpr int kLexToSlot2[4] = {0, 1, 3, 2};

// Quadrilaterals: vertex dofs, edge dofs (each edge run from its smaller to its
// larger vertex id), interiors; every dof on an edge of one element only is essential.
Space* build_space_2d(const Mesh* mesh, int order, int flags) {
  const Mesh& m = *mesh;
  const int p = order, D1 = p + 1, dpe = D1 * D1;
  const int64_t ne = m.ne;
  auto* s = new Space();
  s->mesh = mesh;
  s->dim = 2;
  s->p = p;
  s->D1 = D1;
  s->dpe = dpe;
  s->ne = ne;
  s->ng = 2;
  s->ref_nodes.resize(D1);
  gauss_lobatto_01(D1, s->ref_nodes.data());
  auto corner = [&](int64_t e, int c) { return m.quad[size_t(e) * 4 + kLexToSlot2[c]]; };
  // 4 edges as (axis, low corner) with bit `axis` of the corner clear
  const int eaxis[4] = {0, 0, 1, 1}, ec0[4] = {0, 2, 0, 1};
  int edge_slot_of[2][4] = {{0, 0, 1, 0}, {2, 3, 0, 0}};
  std::vector<std::array<int64_t, 2>> ekeys(size_t(ne) * 4);
  for (int64_t e = 0; e < ne; ++e)
    for (int k = 0; k < 4; ++k) {
      const int64_t a = corner(e, ec0[k]), b = corner(e, ec0[k] | (1 << eaxis[k]));
      ekeys[size_t(e) * 4 + k] = {std::min(a, b), std::max(a, b)};
    }
  std::vector<int64_t> erep;
  std::vector<int32_t> emult;
  match_keys<2>(ekeys, m.nv, erep, emult);
  for (size_t i = 0; i < emult.size(); ++i)
    if (emult[i] > 2) {
      delete s;
      throw Error(PAFEM_EINVAL, "non-conforming mesh: edge shared by more than two elements "
                                "(element " + std::to_string(i / 4) + ")");
    }
  std::vector<int32_t> vdof(size_t(m.nv), -1);
  for (int64_t e = 0; e < ne; ++e)
    for (int k = 0; k < 4; ++k) vdof[size_t(m.quad[size_t(e) * 4 + k])] = 0;
  int64_t next = 0;
  for (int64_t v = 0; v < m.nv; ++v)
    if (vdof[size_t(v)] == 0) vdof[size_t(v)] = int32_t(next++);
  std::vector<int32_t> eid(erep.size(), -1);
  int64_t n_edges = 0;
  for (size_t i = 0; i < erep.size(); ++i)
    eid[i] = (erep[i] == int64_t(i)) ? int32_t(n_edges++) : eid[size_t(erep[i])];
  const int64_t ebase = next;
  const int64_t ibase = ebase + n_edges * (p - 1);
  const int64_t ndofs = ibase + ne * int64_t(p - 1) * (p - 1);
  if (ndofs >= (int64_t(1) << 31) - 1 || ne * int64_t(dpe) >= (int64_t(1) << 31) - 1) {
    delete s;
    throw Error(PAFEM_EINVAL, "problem too large for 32-bit dof indices");
  }
  s->ndofs = ndofs;
  s->gmap.assign(size_t(ne) * dpe, 0);
  s->bmask.assign(size_t(ndofs), 0);
  for (int64_t e = 0; e < ne; ++e) {
    int32_t* g = s->gmap.data() + size_t(e) * dpe;
    for (int i2 = 0; i2 < D1; ++i2)
      for (int i1 = 0; i1 < D1; ++i1) {
        const int idx[2] = {i1, i2};
        const bool b1 = (i1 == 0 || i1 == p), b2 = (i2 == 0 || i2 == p);
        int64_t dof;
        if (b1 && b2) {
          dof = vdof[size_t(corner(e, (i1 == p) | ((i2 == p) << 1)))];
        } else if (b1 || b2) {
          const int a = b1 ? 1 : 0, o = 1 - a;  // a: the axis along the edge
          const int c0 = (idx[o] == p) ? (1 << o) : 0;
          const int k = edge_slot_of[a][c0];
          const int64_t va = corner(e, c0), vb = corner(e, c0 | (1 << a));
          const int tc = (va < vb) ? idx[a] : p - idx[a];
          dof = ebase + int64_t(eid[size_t(e) * 4 + k]) * (p - 1) + (tc - 1);
        } else {
          dof = ibase + e * int64_t(p - 1) * (p - 1) + (i1 - 1) + int64_t(p - 1) * (i2 - 1);
        }
        g[i1 + D1 * i2] = int32_t(dof);
      }
    for (int k = 0; k < 4; ++k) {
      if (emult[size_t(e) * 4 + k] != 1) continue;
      const int a = eaxis[k], o = 1 - a;
      const int v = ((ec0[k] >> o) & 1) ? p : 0;
      for (int t = 0; t < D1; ++t) {
        const int i1 = a == 0 ? t : v, i2 = a == 0 ? v : t;
        s->bmask[size_t(g[i1 + D1 * i2])] = 1;
      }
    }
  }
  finish_space(s, m, flags);
  return s;
}

}  // namespace

uint64_t next_mesh_id() {
  static std::atomic<uint64_t> counter{0};
  return ++counter;
}

std::vector<int32_t> mesh_element_order(const Mesh& m) {
  return m.elem_order.empty() ? morton_order(m) : m.elem_order;
}

void refine_mesh(const Mesh& c, Mesh& f) {
  if (c.dim != 3) throw Error(PAFEM_EUNSUPPORTED, "refinement is built for hexahedra");
  const int64_t ne = c.ne, nv = c.nv;
  if (ne > (int64_t(1) << 27)) throw Error(PAFEM_ESHAPE, "refined mesh would exceed 2^30 elements");
  const auto es = edge_slots();
  const auto fs = face_slots();
  int edge_of[3][8] = {};  // (axis, low corner) -> edge slot
  for (int k = 0; k < 12; ++k) edge_of[es[size_t(k)].axis][es[size_t(k)].c0] = k;
  // shared edges and faces of the coarse mesh, by sorted vertex keys
  std::vector<std::array<int64_t, 2>> ek(size_t(ne) * 12);
  std::vector<std::array<int64_t, 4>> fk(size_t(ne) * 6);
  for (int64_t e = 0; e < ne; ++e) {
    const ElemCorners cc = corners_of(c, e);
    for (int k = 0; k < 12; ++k) {
      const int64_t a = cc.v[es[size_t(k)].c0], b = cc.v[es[size_t(k)].c0 | (1 << es[size_t(k)].axis)];
      ek[size_t(e) * 12 + size_t(k)] = {std::min(a, b), std::max(a, b)};
    }
    for (int k = 0; k < 6; ++k) {
      std::array<int64_t, 4> key{};
      for (int j = 0; j < 4; ++j) key[size_t(j)] = cc.v[fs[size_t(k)].c[j]];
      std::sort(key.begin(), key.end());
      fk[size_t(e) * 6 + size_t(k)] = key;
    }
  }
  std::vector<int64_t> erep, frep;
  std::vector<int32_t> mult;
  match_keys<2>(ek, nv, erep, mult);
  match_keys<4>(fk, nv, frep, mult);
  // new vertex ids: coarse vertices keep theirs, then edges, faces, cells (rep <= item)
  int64_t next = nv;
  std::vector<int64_t> eid(ek.size()), fid(fk.size());
  for (size_t i = 0; i < ek.size(); ++i) eid[i] = erep[i] == int64_t(i) ? next++ : eid[size_t(erep[i])];
  for (size_t i = 0; i < fk.size(); ++i) fid[i] = frep[i] == int64_t(i) ? next++ : fid[size_t(frep[i])];
  const int64_t cell0 = next, nvf = next + ne;

  f = Mesh();
  f.dim = 3;
  f.nv = nvf;
  f.ne = ne * 8;
  f.geom_order = c.geom_order;
  f.xyz.assign(size_t(nvf) * 3, 0.0);
  std::copy(c.xyz.begin(), c.xyz.begin() + nv * 3, f.xyz.begin());
  f.hex.resize(size_t(f.ne) * 8);
  std::vector<uint8_t> placed(size_t(nvf), 0);
  std::fill(placed.begin(), placed.begin() + nv, uint8_t(1));
  // the parent's map at reference point t: trilinear from the corners, or the
  // triquadratic map through the 27 nodes at {0, 1/2, 1}^3
  auto quad1d = [](int m, double t) {
    return m == 0 ? 2.0 * (t - 0.5) * (t - 1.0) : m == 1 ? 4.0 * t * (1.0 - t) : 2.0 * t * (t - 0.5);
  };
  auto parent_map = [&](int64_t e, const ElemCorners& cc, const double t[3], double x[3]) {
    x[0] = x[1] = x[2] = 0.0;
    if (c.geom_order == 2) {
      const double* gn = c.gnodes.data() + size_t(e) * 81;
      for (int m = 0; m < 27; ++m) {
        const double w = quad1d(m % 3, t[0]) * quad1d((m / 3) % 3, t[1]) * quad1d(m / 9, t[2]);
        for (int a = 0; a < 3; ++a) x[a] += w * gn[m * 3 + a];
      }
      return;
    }
    for (int k = 0; k < 8; ++k) {
      double w = 1.0;
      for (int a = 0; a < 3; ++a) w *= ((k >> a) & 1) ? t[a] : 1.0 - t[a];
      for (int a = 0; a < 3; ++a) x[a] += w * c.xyz[size_t(cc.v[k]) * 3 + size_t(a)];
    }
  };
  int64_t lat[27];  // fine vertex of each point of the parent's {0, 1/2, 1}^3 lattice
  for (int64_t e = 0; e < ne; ++e) {
    const ElemCorners cc = corners_of(c, e);
    for (int n = 0; n < 27; ++n) {
      const int ijk[3] = {n % 3, (n / 3) % 3, n / 9};
      int odd = 0, axis = 0, other = 0;
      for (int a = 0; a < 3; ++a) {
        if (ijk[a] == 1) {
          ++odd;
          axis = a;
        } else {
          other = a;
        }
      }
      int64_t id;
      if (odd == 0) {
        id = cc.v[(ijk[0] / 2) | ((ijk[1] / 2) << 1) | ((ijk[2] / 2) << 2)];
      } else if (odd == 1) {
        int c0 = 0;
        for (int a = 0; a < 3; ++a)
          if (a != axis) c0 |= (ijk[a] / 2) << a;
        id = eid[size_t(e) * 12 + size_t(edge_of[axis][c0])];
      } else if (odd == 2) {
        id = fid[size_t(e) * 6 + size_t(2 * other + ijk[other] / 2)];
      } else {
        id = cell0 + e;
      }
      lat[n] = id;
      if (!placed[size_t(id)]) {
        const double t[3] = {0.5 * ijk[0], 0.5 * ijk[1], 0.5 * ijk[2]};
        parent_map(e, cc, t, f.xyz.data() + size_t(id) * 3);
        placed[size_t(id)] = 1;
      }
    }
    for (int o = 0; o < 8; ++o) {
      const int off[3] = {o & 1, (o >> 1) & 1, (o >> 2) & 1};
      int64_t* h = f.hex.data() + size_t(e * 8 + o) * 8;
      for (int slot = 0; slot < 8; ++slot) {
        const int lc = kLexToSlot[slot];  // the slot order is its own inverse
        const int n = (off[0] + (lc & 1)) + 3 * (off[1] + ((lc >> 1) & 1)) + 9 * (off[2] + (lc >> 2));
        h[slot] = lat[n];
      }
    }
  }
  if (c.geom_order == 2) {
    f.gnodes.resize(size_t(f.ne) * 81);
    for (int64_t e = 0; e < ne; ++e) {
      const ElemCorners cc = corners_of(c, e);
      for (int o = 0; o < 8; ++o)
        for (int n = 0; n < 27; ++n) {
          const double t[3] = {0.5 * ((o & 1) + 0.5 * (n % 3)),
                               0.5 * (((o >> 1) & 1) + 0.5 * ((n / 3) % 3)),
                               0.5 * ((o >> 2) + 0.5 * (n / 9))};
          parent_map(e, cc, t, f.gnodes.data() + (size_t(e * 8 + o) * 27 + size_t(n)) * 3);
        }
    }
  }
  const std::vector<int32_t> corder = mesh_element_order(c);
  f.elem_order.resize(size_t(f.ne));
  for (int64_t k = 0; k < ne; ++k)
    for (int o = 0; o < 8; ++o) f.elem_order[size_t(k * 8 + o)] = corder[size_t(k)] * 8 + o;
  f.id = next_mesh_id();
  f.parent_id = c.id;
}

Space* build_space(const Mesh* mesh, int order, int flags) {
  if (order < 1 || order > kMaxOrder)
    throw Error(PAFEM_EUNSUPPORTED, "order must be in 1..8, got " + std::to_string(order));
  if (mesh->dim == 2) return build_space_2d(mesh, order, flags);
  const Mesh& m = *mesh;
  const int p = order, D1 = p + 1, dpe = D1 * D1 * D1;
  const int64_t ne = m.ne;
  auto* s = new Space();
  s->mesh = mesh;
  s->p = p;
  s->D1 = D1;
  s->dpe = dpe;
  s->ne = ne;
  s->ng = (m.geom_order == 2) ? 3 : 2;
  s->ref_nodes.resize(D1);
  gauss_lobatto_01(D1, s->ref_nodes.data());

  // ---- faces: always needed (boundary detection) -------------------------
  const auto fs = face_slots();
  std::vector<std::array<int64_t, 4>> fkeys(size_t(ne) * 6);
  for (int64_t e = 0; e < ne; ++e) {
    const ElemCorners c = corners_of(m, e);
    for (int f = 0; f < 6; ++f) {
      std::array<int64_t, 4> k = {c.v[fs[f].c[0]], c.v[fs[f].c[1]], c.v[fs[f].c[2]],
                                  c.v[fs[f].c[3]]};
      std::sort(k.begin(), k.end());
      fkeys[size_t(e) * 6 + f] = k;
    }
  }
  std::vector<int64_t> frep;
  std::vector<int32_t> fmult;
  match_keys<4>(fkeys, m.nv, frep, fmult);
  for (size_t i = 0; i < fmult.size(); ++i)
    if (fmult[i] > 2) {
      delete s;
      throw Error(PAFEM_EINVAL, "non-conforming mesh: face shared by more than two elements "
                                "(element " + std::to_string(i / 6) + ")");
    }
  fkeys.clear();
  fkeys.shrink_to_fit();

  // ---- numbering of vertices, edges, faces, interiors ---------------------
  std::vector<int32_t> vdof(size_t(m.nv), -1);
  for (int64_t e = 0; e < ne; ++e)
    for (int k = 0; k < 8; ++k) vdof[size_t(m.hex[size_t(e) * 8 + k])] = 0;
  int64_t next = 0;
  for (int64_t v = 0; v < m.nv; ++v)
    if (vdof[v] == 0) vdof[v] = int32_t(next++);

  const auto es = edge_slots();
  std::vector<int64_t> erep;
  std::vector<int32_t> eid, fid;
  int64_t n_edges = 0, n_faces = 0;
  if (p >= 2) {
    std::vector<std::array<int64_t, 2>> ekeys(size_t(ne) * 12);
    for (int64_t e = 0; e < ne; ++e) {
      const ElemCorners c = corners_of(m, e);
      for (int k = 0; k < 12; ++k) {
        int64_t a = c.v[es[k].c0], b = c.v[es[k].c0 | (1 << es[k].axis)];
        ekeys[size_t(e) * 12 + k] = {std::min(a, b), std::max(a, b)};
      }
    }
    std::vector<int32_t> emult;
    match_keys<2>(ekeys, m.nv, erep, emult);
    eid.assign(erep.size(), -1);
    for (size_t i = 0; i < erep.size(); ++i)
      eid[i] = (erep[i] == int64_t(i)) ? int32_t(n_edges++) : eid[size_t(erep[i])];
    fid.assign(frep.size(), -1);
    for (size_t i = 0; i < frep.size(); ++i)
      fid[i] = (frep[i] == int64_t(i)) ? int32_t(n_faces++) : fid[size_t(frep[i])];
  }
  const int64_t nvd = next;
  const int64_t ebase = nvd;
  const int64_t fbase = ebase + n_edges * (p - 1);
  const int64_t ibase = fbase + n_faces * int64_t(p - 1) * (p - 1);
  const int64_t ndofs = ibase + ne * int64_t(p - 1) * (p - 1) * (p - 1);
  if (ndofs >= (int64_t(1) << 31) - 1 || ne * int64_t(dpe) >= (int64_t(1) << 31) - 1) {
    delete s;
    throw Error(PAFEM_EINVAL, "problem too large for 32-bit dof indices");
  }
  s->ndofs = ndofs;

  // local (axis, low corner) -> edge slot index
  int edge_slot_of[3][8];
  for (int k = 0; k < 12; ++k) edge_slot_of[es[k].axis][es[k].c0] = k;

  s->gmap.assign(size_t(ne) * dpe, 0);
  s->bmask.assign(size_t(ndofs), 0);
  for (int64_t e = 0; e < ne; ++e) {
    const ElemCorners c = corners_of(m, e);
    int32_t* g = s->gmap.data() + size_t(e) * dpe;
    for (int i3 = 0; i3 < D1; ++i3)
      for (int i2 = 0; i2 < D1; ++i2)
        for (int i1 = 0; i1 < D1; ++i1) {
          const int idx[3] = {i1, i2, i3};
          int nb = 0;
          for (int a = 0; a < 3; ++a) nb += (idx[a] == 0 || idx[a] == p);
          int64_t dof = -1;
          if (nb == 3) {
            int cc = (i1 == p) | ((i2 == p) << 1) | ((i3 == p) << 2);
            dof = vdof[size_t(c.v[cc])];
          } else if (nb == 2) {
            int a = (idx[0] != 0 && idx[0] != p) ? 0 : (idx[1] != 0 && idx[1] != p) ? 1 : 2;
            int c0 = 0;
            for (int b = 0; b < 3; ++b)
              if (b != a && idx[b] == p) c0 |= (1 << b);
            const int k = edge_slot_of[a][c0];
            const int64_t va = c.v[c0], vb = c.v[c0 | (1 << a)];
            const int t = idx[a];
            const int tc = (va < vb) ? t : p - t;
            dof = ebase + int64_t(eid[size_t(e) * 12 + k]) * (p - 1) + (tc - 1);
          } else if (nb == 1) {
            int a = (idx[0] == 0 || idx[0] == p) ? 0 : (idx[1] == 0 || idx[1] == p) ? 1 : 2;
            const int side = (idx[a] == p);
            const int f = 2 * a + side;
            const int b0 = (a == 0) ? 1 : 0, b1 = (a == 2) ? 1 : 2;
            // origin: face corner with the smallest vertex id
            int O = fs[f].c[0];
            for (int q = 1; q < 4; ++q)
              if (c.v[fs[f].c[q]] < c.v[O]) O = fs[f].c[q];
            const int n0 = O ^ (1 << b0), n1 = O ^ (1 << b1);
            int au, av;
            if (c.v[n0] < c.v[n1]) {
              au = b0;
              av = b1;
            } else {
              au = b1;
              av = b0;
            }
            const int cu = ((O >> au) & 1) ? p - idx[au] : idx[au];
            const int cv = ((O >> av) & 1) ? p - idx[av] : idx[av];
            dof = fbase + int64_t(fid[size_t(e) * 6 + f]) * (p - 1) * (p - 1) + (cu - 1) +
                  int64_t(p - 1) * (cv - 1);
          } else {
            dof = ibase + e * int64_t(p - 1) * (p - 1) * (p - 1) + (i1 - 1) +
                  int64_t(p - 1) * ((i2 - 1) + int64_t(p - 1) * (i3 - 1));
          }
          g[i1 + D1 * (i2 + D1 * i3)] = int32_t(dof);
        }
    // essential dofs: all nodes of faces that belong to this element only
    for (int f = 0; f < 6; ++f) {
      if (fmult[size_t(e) * 6 + f] != 1) continue;
      const int a = fs[f].axis, v = fs[f].side ? p : 0;
      for (int i3 = 0; i3 < D1; ++i3)
        for (int i2 = 0; i2 < D1; ++i2)
          for (int i1 = 0; i1 < D1; ++i1) {
            const int idx[3] = {i1, i2, i3};
            if (idx[a] == v) s->bmask[size_t(g[i1 + D1 * (i2 + D1 * i3)])] = 1;
          }
    }
  }

  finish_space(s, m, flags);
  return s;
}

// Nedelec space.  Local dof (a, i0, i1, i2): the basis function of component a, open
// (Gauss-Legendre) index i_a in [0, p), closed (Gauss-Lobatto) indices i_b in [0, p]
// for b != a.  A dof with both closed indices on the element's boundary lies on an
// edge along a, one on a face, none in the interior.  Global numbering: edge dofs
// (p per edge, running from the edge's smaller to its larger vertex id), face dofs
// (2p(p-1) per face, in the face frame of the H1 space: first the dofs along its
// first axis, then along its second), interiors.  Orientation: the global basis
// function along local axis a is the local one when the smallest vertex id among
// the entity's corners with c_a = 1 exceeds the smallest among those with c_a = 0,
// else its negative; interior dofs are never negated.  Every dof on a boundary face
// is essential (tangential trace).
Space* build_nd_space(const Mesh* mesh, int order, int flags) {
  if (order < 1 || order > kMaxOrder)
    throw Error(PAFEM_EUNSUPPORTED, "order must be in 1..8, got " + std::to_string(order));
  if (mesh->dim != 3) throw Error(PAFEM_EUNSUPPORTED, "Nedelec spaces are built on hexahedra");
  const Mesh& m = *mesh;
  const int p = order, D1 = p + 1, dpe = nd_dofs_per_elem(p);
  const int64_t ne = m.ne;
  auto* s = new Space();
  s->mesh = mesh;
  s->family = kFamilyND;
  s->p = p;
  s->D1 = D1;
  s->dpe = dpe;
  s->ne = ne;
  s->ng = (m.geom_order == 2) ? 3 : 2;
  s->ref_nodes.resize(D1);
  gauss_lobatto_01(D1, s->ref_nodes.data());

  const auto fs = face_slots();
  const auto es = edge_slots();
  std::vector<std::array<int64_t, 4>> fkeys(size_t(ne) * 6);
  std::vector<std::array<int64_t, 2>> ekeys(size_t(ne) * 12);
  for (int64_t e = 0; e < ne; ++e) {
    const ElemCorners c = corners_of(m, e);
    for (int f = 0; f < 6; ++f) {
      std::array<int64_t, 4> k = {c.v[fs[f].c[0]], c.v[fs[f].c[1]], c.v[fs[f].c[2]],
                                  c.v[fs[f].c[3]]};
      std::sort(k.begin(), k.end());
      fkeys[size_t(e) * 6 + f] = k;
    }
    for (int k = 0; k < 12; ++k) {
      const int64_t a = c.v[es[k].c0], b = c.v[es[k].c0 | (1 << es[k].axis)];
      ekeys[size_t(e) * 12 + k] = {std::min(a, b), std::max(a, b)};
    }
  }
  std::vector<int64_t> frep, erep;
  std::vector<int32_t> fmult, emult;
  match_keys<4>(fkeys, m.nv, frep, fmult);
  match_keys<2>(ekeys, m.nv, erep, emult);
  fkeys.clear();
  fkeys.shrink_to_fit();
  ekeys.clear();
  ekeys.shrink_to_fit();
  for (size_t i = 0; i < fmult.size(); ++i)
    if (fmult[i] > 2) {
      delete s;
      throw Error(PAFEM_EINVAL, "non-conforming mesh: face shared by more than two elements "
                                "(element " + std::to_string(i / 6) + ")");
    }
  std::vector<int32_t> eid(erep.size(), -1), fid(frep.size(), -1);
  int64_t n_edges = 0, n_faces = 0;
  for (size_t i = 0; i < erep.size(); ++i)
    eid[i] = (erep[i] == int64_t(i)) ? int32_t(n_edges++) : eid[size_t(erep[i])];
  for (size_t i = 0; i < frep.size(); ++i)
    fid[i] = (frep[i] == int64_t(i)) ? int32_t(n_faces++) : fid[size_t(frep[i])];
  const int64_t per_face = 2 * int64_t(p) * (p - 1), per_int = 3 * int64_t(p) * (p - 1) * (p - 1);
  const int64_t fbase = n_edges * p;
  const int64_t ibase = fbase + n_faces * per_face;
  const int64_t ndofs = ibase + ne * per_int;
  if (ndofs >= (int64_t(1) << 31) - 1 || ne * int64_t(dpe) >= (int64_t(1) << 31) - 1) {
    delete s;
    throw Error(PAFEM_EINVAL, "problem too large for 32-bit dof indices");
  }
  s->ndofs = ndofs;
  int edge_slot_of[3][8];
  for (int k = 0; k < 12; ++k) edge_slot_of[es[k].axis][es[k].c0] = k;

  s->gmap.assign(size_t(ne) * dpe, 0);
  s->gsign.assign(size_t(ne) * dpe, 1);
  s->bmask.assign(size_t(ndofs), 0);
  for (int64_t e = 0; e < ne; ++e) {
    const ElemCorners c = corners_of(m, e);
    int32_t* g = s->gmap.data() + size_t(e) * dpe;
    int8_t* sg = s->gsign.data() + size_t(e) * dpe;
    int j = 0;
    for (int a = 0; a < 3; ++a) {
      const int n0 = a == 0 ? p : D1, n1 = a == 1 ? p : D1, n2 = a == 2 ? p : D1;
      for (int i2 = 0; i2 < n2; ++i2)
        for (int i1 = 0; i1 < n1; ++i1)
          for (int i0 = 0; i0 < n0; ++i0, ++j) {
            const int idx[3] = {i0, i1, i2};
            // doubled lattice: closed i -> 2i, open k -> 2k + 1
            int mm[3];
            for (int b = 0; b < 3; ++b) mm[b] = (b == a) ? 2 * idx[b] + 1 : 2 * idx[b];
            int nb = 0, nrm = -1;
            for (int b = 0; b < 3; ++b)
              if (b != a && (idx[b] == 0 || idx[b] == p)) {
                ++nb;
                nrm = b;
              }
            int64_t dof;
            int sgn = 1;
            if (nb == 2) {
              int c0 = 0;
              for (int b = 0; b < 3; ++b)
                if (b != a && idx[b] == p) c0 |= (1 << b);
              const int k = edge_slot_of[a][c0];
              const int64_t va = c.v[c0], vb = c.v[c0 | (1 << a)];
              const int kc = (va < vb) ? idx[a] : p - 1 - idx[a];
              sgn = (vb > va) ? 1 : -1;
              dof = int64_t(eid[size_t(e) * 12 + k]) * p + kc;
            } else if (nb == 1) {
              const int f = 2 * nrm + (idx[nrm] == p);
              const int b0 = (nrm == 0) ? 1 : 0, b1 = (nrm == 2) ? 1 : 2;
              int O = fs[f].c[0];
              for (int q = 1; q < 4; ++q)
                if (c.v[fs[f].c[q]] < c.v[O]) O = fs[f].c[q];
              const int nb0 = O ^ (1 << b0), nb1 = O ^ (1 << b1);
              const int au = (c.v[nb0] < c.v[nb1]) ? b0 : b1, av = (au == b0) ? b1 : b0;
              const int mu = ((O >> au) & 1) ? 2 * p - mm[au] : mm[au];
              const int mv = ((O >> av) & 1) ? 2 * p - mm[av] : mm[av];
              int64_t loc;
              if (a == au)
                loc = int64_t(mv / 2 - 1) * p + (mu - 1) / 2;
              else
                loc = int64_t(p) * (p - 1) + int64_t((mv - 1) / 2) * (p - 1) + (mu / 2 - 1);
              int64_t lo0 = INT64_MAX, lo1 = INT64_MAX;
              for (int q = 0; q < 4; ++q) {
                const int cc = fs[f].c[q];
                if ((cc >> a) & 1)
                  lo1 = std::min(lo1, c.v[cc]);
                else
                  lo0 = std::min(lo0, c.v[cc]);
              }
              sgn = (lo1 > lo0) ? 1 : -1;
              dof = fbase + int64_t(fid[size_t(e) * 6 + f]) * per_face + loc;
            } else {
              // interior: component a block, open index along a, closed interior indices
              int m0 = a == 0 ? p : p - 1, m1 = a == 1 ? p : p - 1;
              const int j0 = a == 0 ? i0 : i0 - 1, j1 = a == 1 ? i1 : i1 - 1,
                        j2 = a == 2 ? i2 : i2 - 1;
              dof = ibase + e * per_int + int64_t(a) * p * (p - 1) * (p - 1) + j0 +
                    int64_t(m0) * (j1 + int64_t(m1) * j2);
            }
            g[j] = int32_t(dof);
            sg[j] = int8_t(sgn);
          }
    }
    // essential dofs: the nodes on faces that belong to this element only
    for (int f = 0; f < 6; ++f) {
      if (fmult[size_t(e) * 6 + f] != 1) continue;
      const int nrm = fs[f].axis, v = fs[f].side ? p : 0;
      int jj = 0;
      for (int a = 0; a < 3; ++a) {
        const int n0 = a == 0 ? p : D1, n1 = a == 1 ? p : D1, n2 = a == 2 ? p : D1;
        for (int i2 = 0; i2 < n2; ++i2)
          for (int i1 = 0; i1 < n1; ++i1)
            for (int i0 = 0; i0 < n0; ++i0, ++jj) {
              const int idx[3] = {i0, i1, i2};
              if (a != nrm && idx[nrm] == v) s->bmask[size_t(g[jj])] = 1;
            }
      }
    }
  }
  finish_space(s, m, flags);
  s->tables_open = build_open_tables(p);
  return s;
}

// Discontinuous space: no shared dofs; the faces give the coupling.  Each interior
// face records its two device elements, local faces and the orientation that carries
// the "-" side's face indices to the "+" side's, found from the shared corner ids.
Space* build_l2_space(const Mesh* mesh, int order, int flags) {
  if (order < 1 || order > kMaxOrder)
    throw Error(PAFEM_EUNSUPPORTED, "order must be in 1..8, got " + std::to_string(order));
  if (mesh->dim != 3) throw Error(PAFEM_EUNSUPPORTED, "L2 spaces are built on hexahedra");
  const Mesh& m = *mesh;
  const int p = order, D1 = p + 1, dpe = D1 * D1 * D1;
  const int64_t ne = m.ne;
  if (ne * int64_t(dpe) >= (int64_t(1) << 31) - 1)
    throw Error(PAFEM_EINVAL, "problem too large for 32-bit dof indices");
  auto* s = new Space();
  s->mesh = mesh;
  s->family = kFamilyL2;
  s->p = p;
  s->D1 = D1;
  s->dpe = dpe;
  s->ne = ne;
  s->ng = (m.geom_order == 2) ? 3 : 2;
  s->ref_nodes.resize(D1);
  gauss_lobatto_01(D1, s->ref_nodes.data());
  s->ndofs = ne * dpe;
  s->gmap.resize(size_t(ne) * dpe);
  for (size_t i = 0; i < s->gmap.size(); ++i) s->gmap[i] = int32_t(i);
  s->bmask.assign(size_t(s->ndofs), 0);

  const auto fs = face_slots();
  std::vector<std::array<int64_t, 4>> fkeys(size_t(ne) * 6);
  for (int64_t e = 0; e < ne; ++e) {
    const ElemCorners c = corners_of(m, e);
    for (int f = 0; f < 6; ++f) {
      std::array<int64_t, 4> k = {c.v[fs[f].c[0]], c.v[fs[f].c[1]], c.v[fs[f].c[2]],
                                  c.v[fs[f].c[3]]};
      std::sort(k.begin(), k.end());
      fkeys[size_t(e) * 6 + f] = k;
    }
  }
  std::vector<int64_t> frep;
  std::vector<int32_t> fmult;
  match_keys<4>(fkeys, m.nv, frep, fmult);
  fkeys.clear();
  fkeys.shrink_to_fit();
  for (size_t i = 0; i < fmult.size(); ++i)
    if (fmult[i] > 2) {
      delete s;
      throw Error(PAFEM_EINVAL, "non-conforming mesh: face shared by more than two elements "
                                "(element " + std::to_string(i / 6) + ")");
    }
  finish_space(s, m, flags);
  std::vector<int32_t> dev_of(static_cast<size_t>(ne));
  for (int64_t k = 0; k < ne; ++k) dev_of[size_t(s->dev_order[size_t(k)])] = int32_t(k);
  // face-local coordinates (u, v) in {0,1}^2 of corner cc of face f: bits of the two
  // tangential axes in increasing order
  auto uv_of = [&](int f, int cc, int& u, int& v) {
    const int a = f / 2, b = (a == 0) ? 1 : 0, c2 = (a == 2) ? 1 : 2;
    u = (cc >> b) & 1;
    v = (cc >> c2) & 1;
  };
  struct FaceRec {
    int32_t key, em, ep, code;
  };
  std::vector<FaceRec> recs;
  std::vector<std::array<int32_t, 3>> brecs;
  for (size_t i = 0; i < frep.size(); ++i) {
    const int64_t e = int64_t(i) / 6;
    const int f = int(i % 6);
    if (fmult[i] == 1) {
      brecs.push_back({dev_of[size_t(e)], dev_of[size_t(e)], f});
      continue;
    }
    if (frep[i] == int64_t(i)) continue;  // the "-" side is the representative
    const int64_t em = frep[i] / 6, ep = e;
    const int fm = int(frep[i] % 6), fp = f;
    const ElemCorners cm = corners_of(m, em), cp = corners_of(m, ep);
    // corners of the "-" face at (s, t) = (0,0), (1,0), (0,1) -> "+" face (u, v)
    int U[3], V[3];
    const int st[3][2] = {{0, 0}, {1, 0}, {0, 1}};
    for (int k = 0; k < 3; ++k) {
      int cc = -1;
      for (int q = 0; q < 4; ++q) {
        int uu, vv;
        uv_of(fm, fs[fm].c[q], uu, vv);
        if (uu == st[k][0] && vv == st[k][1]) cc = fs[fm].c[q];
      }
      const int64_t vid = cm.v[cc];
      U[k] = V[k] = -1;
      for (int q = 0; q < 4; ++q)
        if (cp.v[fs[fp].c[q]] == vid) uv_of(fp, fs[fp].c[q], U[k], V[k]);
      if (U[k] < 0) {
        delete s;
        throw Error(PAFEM_EINVAL, "faces of elements " + std::to_string(em) + " and " +
                                      std::to_string(ep) + " do not share their corners");
      }
    }
    const int dsu = U[1] - U[0], dsv = V[1] - V[0], dtu = U[2] - U[0], dtv = V[2] - V[0];
    int orient;
    if (dsu != 0)  // s runs along u, t along v
      orient = (dsu < 0 ? 2 : 0) | (dtv < 0 ? 4 : 0);
    else           // s runs along v, t along u
      orient = 1 | (dtu < 0 ? 2 : 0) | (dsv < 0 ? 4 : 0);
    const int32_t a = dev_of[size_t(em)], b = dev_of[size_t(ep)];
    recs.push_back({std::min(a, b), a, b, fm | (fp << 3) | (orient << 6)});
  }
  std::sort(recs.begin(), recs.end(),
            [](const FaceRec& x, const FaceRec& y) { return x.key < y.key || (x.key == y.key && x.ep < y.ep); });
  s->faces.reserve(recs.size() * kFaceInts);
  for (const auto& r : recs) {
    s->faces.push_back(r.em);
    s->faces.push_back(r.ep);
    s->faces.push_back(r.code);
  }
  std::sort(brecs.begin(), brecs.end());
  s->bfaces.reserve(brecs.size() * 2);
  for (const auto& r : brecs) {
    s->bfaces.push_back(r[1]);
    s->bfaces.push_back(r[2]);
  }
  return s;
}

namespace {
// Nedelec dofs: the physical node of each dof (open index on the Gauss-Legendre
// points along its component's axis, closed indices on the Gauss-Lobatto points)
void nd_dof_coords(const Space& s, double* xyz) {
  const Mesh& m = *s.mesh;
  const int p = s.p, D1 = s.D1, ng = s.ng;
  std::vector<double> onodes(p), ow(p);
  gauss_legendre_01(p, onodes.data(), ow.data());
  std::vector<double> gn(ng), Bc(size_t(D1) * ng), Gc(size_t(D1) * ng), Bo(size_t(p) * ng),
      Go(size_t(p) * ng);
  for (int i = 0; i < ng; ++i) gn[i] = double(i) / (ng - 1);
  lagrange_tables(ng, gn.data(), D1, s.ref_nodes.data(), Bc.data(), Gc.data());
  lagrange_tables(ng, gn.data(), p, onodes.data(), Bo.data(), Go.data());
  const int nn = ng * ng * ng;
  std::vector<double> X(size_t(nn) * 3);
  for (int64_t e = 0; e < s.ne; ++e) {
    if (m.geom_order == 2) {
      std::memcpy(X.data(), m.gnodes.data() + size_t(e) * 27 * 3, sizeof(double) * 81);
    } else {
      const ElemCorners c = corners_of(m, e);
      for (int k = 0; k < 8; ++k)
        for (int a = 0; a < 3; ++a) X[k * 3 + a] = m.xyz[size_t(c.v[k]) * 3 + a];
    }
    const int32_t* g = s.gmap.data() + size_t(e) * s.dpe;
    int j = 0;
    for (int a = 0; a < 3; ++a) {
      const int n0 = a == 0 ? p : D1, n1 = a == 1 ? p : D1, n2 = a == 2 ? p : D1;
      const double* T0 = a == 0 ? Bo.data() : Bc.data();
      const double* T1 = a == 1 ? Bo.data() : Bc.data();
      const double* T2 = a == 2 ? Bo.data() : Bc.data();
      for (int i2 = 0; i2 < n2; ++i2)
        for (int i1 = 0; i1 < n1; ++i1)
          for (int i0 = 0; i0 < n0; ++i0, ++j) {
            double x[3] = {0, 0, 0};
            for (int k3 = 0; k3 < ng; ++k3)
              for (int k2 = 0; k2 < ng; ++k2)
                for (int k1 = 0; k1 < ng; ++k1) {
                  const double w = T0[i0 * ng + k1] * T1[i1 * ng + k2] * T2[i2 * ng + k3];
                  const int k = k1 + ng * (k2 + ng * k3);
                  for (int b = 0; b < 3; ++b) x[b] += w * X[k * 3 + b];
                }
            for (int b = 0; b < 3; ++b) xyz[size_t(g[j]) * 3 + b] = x[b];
          }
    }
  }
}
}  // namespace

void space_dof_coords(const Space& s, double* xyz) {
  if (s.family == kFamilyND) {
    nd_dof_coords(s, xyz);
    return;
  }
  const Mesh& m = *s.mesh;
  const int D1 = s.D1, ng = s.ng;
  if (s.dim == 2) {
    std::vector<double> gn = {0.0, 1.0}, Bg(size_t(D1) * 2), Gg(size_t(D1) * 2);
    lagrange_tables(2, gn.data(), D1, s.ref_nodes.data(), Bg.data(), Gg.data());
    for (int64_t e = 0; e < s.ne; ++e) {
      double X[4][2];
      for (int k = 0; k < 4; ++k)
        for (int a = 0; a < 2; ++a)
          X[k][a] = m.xyz[size_t(m.quad[size_t(e) * 4 + kLexToSlot2[k]]) * 2 + a];
      const int32_t* g = s.gmap.data() + size_t(e) * s.dpe;
      for (int i2 = 0; i2 < D1; ++i2)
        for (int i1 = 0; i1 < D1; ++i1) {
          double x[2] = {0, 0};
          for (int k2 = 0; k2 < 2; ++k2)
            for (int k1 = 0; k1 < 2; ++k1)
              for (int a = 0; a < 2; ++a) x[a] += Bg[i1 * 2 + k1] * Bg[i2 * 2 + k2] * X[k1 + 2 * k2][a];
          const int32_t d = g[i1 + D1 * i2];
          xyz[size_t(d) * 2] = x[0];
          xyz[size_t(d) * 2 + 1] = x[1];
        }
    }
    return;
  }
  // geometry basis (linear or quadratic Lagrange on equispaced nodes) at the
  // Gauss-Lobatto nodes
  std::vector<double> gn(ng), Bg(size_t(D1) * ng), Gg(size_t(D1) * ng);
  for (int i = 0; i < ng; ++i) gn[i] = double(i) / (ng - 1);
  lagrange_tables(ng, gn.data(), D1, s.ref_nodes.data(), Bg.data(), Gg.data());
  const int nn = ng * ng * ng;
  std::vector<double> X(size_t(nn) * 3);
  for (int64_t e = 0; e < s.ne; ++e) {
    if (m.geom_order == 2) {
      std::memcpy(X.data(), m.gnodes.data() + size_t(e) * 27 * 3, sizeof(double) * 81);
    } else {
      const ElemCorners c = corners_of(m, e);
      for (int k = 0; k < 8; ++k)
        for (int a = 0; a < 3; ++a) X[k * 3 + a] = m.xyz[size_t(c.v[k]) * 3 + a];
    }
    const int32_t* g = s.gmap.data() + size_t(e) * s.dpe;
    for (int i3 = 0; i3 < D1; ++i3)
      for (int i2 = 0; i2 < D1; ++i2)
        for (int i1 = 0; i1 < D1; ++i1) {
          double x[3] = {0, 0, 0};
          for (int k3 = 0; k3 < ng; ++k3)
            for (int k2 = 0; k2 < ng; ++k2)
              for (int k1 = 0; k1 < ng; ++k1) {
                const double w = Bg[i1 * ng + k1] * Bg[i2 * ng + k2] * Bg[i3 * ng + k3];
                const int k = k1 + ng * (k2 + ng * k3);
                for (int a = 0; a < 3; ++a) x[a] += w * X[k * 3 + a];
              }
          const int32_t d = g[i1 + D1 * (i2 + D1 * i3)];
          for (int a = 0; a < 3; ++a) xyz[size_t(d) * 3 + a] = x[a];
        }
  }
}

void space_device_layout(const Space& s, size_t* off, size_t* total) {
  const size_t nn = s.dim == 2 ? size_t(s.ng) * s.ng : size_t(s.ng) * s.ng * s.ng;
  size_t o = 0;
  const size_t sizes[kSpaceSegments] = {
      sizeof(int32_t) * size_t(s.ne) * s.dpe,      // 0 gmap (device order)
      sizeof(double) * size_t(s.ne) * nn * s.dim,  // 1 geometry nodes (device order)
      size_t(s.ndofs),                             // 2 boundary mask
      sizeof(int32_t) * size_t(s.ndofs + 1),       // 3 transposed offsets
      sizeof(int32_t) * size_t(s.ne) * s.dpe,      // 4 transposed entries
      sizeof(double) * s.tables.size(),            // 5 1D tables
      sizeof(int32_t) * 64,                        // 6 status words
      sizeof(int32_t) * size_t(s.ne),              // 7 caller element ids
      sizeof(int32_t) * s.tile_off.size(),         // 8 tile offsets
      sizeof(int32_t) * s.tile_dofs.size(),        // 9 tile dof lists
      sizeof(uint16_t) * s.tile_slot.size(),       // 10 tile slot maps
      sizeof(float) * s.tables.size(),             // 11 1D tables in FP32
      sizeof(uint32_t) * size_t(s.ne) * owner_words(s.dpe),  // 12 owner bits
      s.gsign.size(),                              // 13 Nedelec dof signs (device order)
      sizeof(double) * s.tables_open.size(),       // 14 Nedelec open-basis tables
      sizeof(int32_t) * s.faces.size(),            // 15 L2 interior faces
      sizeof(int32_t) * s.bfaces.size(),           // 16 L2 boundary faces
  };
  for (int i = 0; i < kSpaceSegments; ++i) {
    off[i] = o;
    o += align256(sizes[i]);
  }
  off[kSpaceSegments] = o;
  *total = o;
}

void space_pack(const Space& s, std::vector<int32_t>& gmap_enc, std::vector<double>& gnodes,
                std::vector<int32_t>& toff, std::vector<int32_t>& tidx,
                std::vector<uint32_t>& owner) {
  const Mesh& m = *s.mesh;
  const size_t n = size_t(s.ne) * s.dpe;
  gmap_enc.resize(n);
  for (int64_t k = 0; k < s.ne; ++k) {
    const int32_t* g = s.gmap.data() + size_t(s.dev_order[size_t(k)]) * s.dpe;
    for (int i = 0; i < s.dpe; ++i)
      gmap_enc[size_t(k) * s.dpe + i] = s.bmask[size_t(g[i])] ? ~g[i] : g[i];
  }
  if (s.dim == 2) {
    // [element][lexicographic corner][x, y]
    gnodes.resize(size_t(s.ne) * 8);
    for (int64_t k = 0; k < s.ne; ++k) {
      const int64_t e = s.dev_order[size_t(k)];
      for (int c = 0; c < 4; ++c)
        for (int a = 0; a < 2; ++a)
          gnodes[size_t(k) * 8 + c * 2 + a] = m.xyz[size_t(m.quad[size_t(e) * 4 + kLexToSlot2[c]]) * 2 + a];
    }
  }
  const int nn = s.ng * s.ng * s.ng;
  if (s.dim == 3) gnodes.resize(size_t(s.ne) * nn * 3);
  for (int64_t k = 0; k < s.ne && s.dim == 3; ++k) {
    const int64_t e = s.dev_order[size_t(k)];
    double* X = gnodes.data() + size_t(k) * nn * 3;
    if (m.geom_order == 2) {
      std::memcpy(X, m.gnodes.data() + size_t(e) * 81, sizeof(double) * 81);
    } else {
      const ElemCorners c = corners_of(m, e);
      for (int q = 0; q < 8; ++q)
        for (int a = 0; a < 3; ++a) X[q * 3 + a] = m.xyz[size_t(c.v[q]) * 3 + a];
    }
  }
  // transposed map: for each dof, its element-vector entries (device order) ascending
  toff.assign(size_t(s.ndofs) + 1, 0);
  auto dof_of = [&](size_t i) { const int32_t v = gmap_enc[i]; return v < 0 ? ~v : v; };
  for (size_t i = 0; i < n; ++i) toff[size_t(dof_of(i)) + 1]++;
  for (int64_t d = 0; d < s.ndofs; ++d) toff[size_t(d) + 1] += toff[size_t(d)];
  tidx.resize(n);
  std::vector<int32_t> fill(toff.begin(), toff.end() - 1);
  for (size_t i = 0; i < n; ++i) tidx[size_t(fill[size_t(dof_of(i))]++)] = int32_t(i);
  // owner bits: the first element-vector position of each dof
  const int W = owner_words(s.dpe);
  owner.assign(size_t(s.ne) * W, 0u);
  for (int64_t d = 0; d < s.ndofs; ++d) {
    const int64_t pos = tidx[size_t(toff[size_t(d)])];
    const int64_t k = pos / s.dpe, i = pos - k * s.dpe;
    owner[size_t(k) * W + size_t(i / 32)] |= 1u << (i % 32);
  }
}

}  // namespace pafem
