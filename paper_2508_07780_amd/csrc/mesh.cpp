// Host setup of the FEM box: Kuhn tetrahedra, node partitions with halos,
// per-partition element colouring and the deduplicated element geometry table.
//
// The paper discretises the inner cube with tetrahedra and the outer region with
// hexahedra (section "Numerical results", Fig. "meshes").  Here each hex cell of
// the FEM box is split into the 6 Kuhn tetrahedra (one per permutation of the
// axes), which keeps the mesh conforming; the kernels only see general tetrahedral
// connectivity plus a geometry table, so any conforming tetrahedral mesh whose
// nodes carry the same ownership rules would run unchanged.
//
// Owned (FEM-updated) nodes are the lattice nodes of layer >= 1; they are cut
// into blocks of FEM_PB^3 nodes.  A partition holds every tetrahedron that
// touches one of its owned nodes, so elements on a partition border are
// evaluated by each partition that needs them and no partial sums are exchanged.
// Elements are coloured so that two elements of one colour never share an owned
// node of the partition; the kernel scatters colour by colour without atomics,
// which makes every result bitwise reproducible.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <climits>
#include <map>
#include <set>
#include <unordered_map>
#include <vector>

#include "dd_common.hpp"

namespace dd {

namespace {

struct Lattice {
  int c[3];   // cells per axis
  int s[3];   // nodes per axis
  int64_t idx(int x, int y, int z) const { return x + (int64_t)s[0] * (y + (int64_t)s[1] * z); }
  int layer(int x, int y, int z) const {
    int l = std::min(x, c[0] - x);
    l = std::min(l, std::min(y, c[1] - y));
    return std::min(l, std::min(z, c[2] - z));
  }
};

const int kPerms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// Gradients of the 4 barycentric functions and the volume of a tetrahedron with
// vertices p[0..3] (FP64); returns false for a degenerate element.
bool tet_geometry(const double p[4][3], double grad[4][3], double* vol) {
  double J[3][3];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) J[r][k] = p[k + 1][r] - p[0][r];  // column k = edge k
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  if (!(std::fabs(det) > 0.0)) return false;
  // inverse: row k of J^{-1} is the gradient of barycentric coordinate k+1
  double inv[3][3];
  inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  for (int a = 0; a < 3; ++a) {
    grad[0][a] = -(inv[0][a] + inv[1][a] + inv[2][a]);
    for (int k = 0; k < 3; ++k) grad[k + 1][a] = inv[k][a];
  }
  *vol = std::fabs(det) / 6.0;
  return true;
}

}  // namespace

std::string build_mesh(const dd_problem_desc& d, HostMesh& m, const int pb[3], bool elements) {
  Lattice L;
  for (int a = 0; a < 3; ++a) {
    L.c[a] = d.fem_cells[a];
    L.s[a] = d.fem_cells[a] + 1;
  }
  m.n_fem = (int64_t)L.s[0] * L.s[1] * L.s[2];
  const int ow[3] = {L.c[0] - 1, L.c[1] - 1, L.c[2] - 1};  // owned nodes per axis
  m.n_own = (int64_t)ow[0] * ow[1] * ow[2];
  m.n_l0 = face_lex_count(L.s[0], L.s[1], L.s[2], 63u);
  int npb[3];
  for (int a = 0; a < 3; ++a) {
    if (pb[a] < 1 || pb[0] * pb[1] * pb[2] > FEM_OWN_MAX) return "bad FEM partition block";
    npb[a] = (ow[a] + pb[a] - 1) / pb[a];
  }
  m.n_part = npb[0] * npb[1] * npb[2];

  // internal numbering: partition-major, lexicographic inside the block
  std::vector<int> lat2int(m.n_fem, 0);  // owned: internal id; layer 0: -1 - layer0 index
  for (int z = 0; z < L.s[2]; ++z)
    for (int y = 0; y < L.s[1]; ++y)
      for (int x = 0; x < L.s[0]; ++x)
        if (L.layer(x, y, z) == 0)
          lat2int[L.idx(x, y, z)] = -1 - (int)face_lex_index(x, y, z, L.s[0], L.s[1], L.s[2], 63u);
  m.own_off.assign(m.n_part + 1, 0);
  m.own_grid.assign(m.n_own, -1);
  m.own_api.assign(m.n_own, 0);
  std::vector<std::array<int, 6>> prange(m.n_part);
  {
    int next = 0, p = 0;
    for (int pz = 0; pz < npb[2]; ++pz)
      for (int py = 0; py < npb[1]; ++py)
        for (int px = 0; px < npb[0]; ++px, ++p) {
          const int lo[3] = {1 + px * pb[0], 1 + py * pb[1], 1 + pz * pb[2]};
          const int hi[3] = {std::min(lo[0] + pb[0], L.c[0]), std::min(lo[1] + pb[1], L.c[1]),
                             std::min(lo[2] + pb[2], L.c[2])};
          prange[p] = {lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]};
          m.own_off[p] = next;
          for (int z = lo[2]; z < hi[2]; ++z)
            for (int y = lo[1]; y < hi[1]; ++y)
              for (int x = lo[0]; x < hi[0]; ++x) {
                const int64_t li = L.idx(x, y, z);
                lat2int[li] = next;
                m.own_api[next] = (int)li;
                if (L.layer(x, y, z) == 1) {
                  const int64_t gx = d.fem_lo[0] + x, gy = d.fem_lo[1] + y, gz = d.fem_lo[2] + z;
                  m.own_grid[next] = (int)(gx + (int64_t)d.n_outer[0] * (gy + (int64_t)d.n_outer[1] * gz));
                }
                ++next;
              }
        }
    m.own_off[m.n_part] = next;
  }

  // geometry table (deduplicated on the float32 image of the FP64 geometry)
  std::map<std::array<uint32_t, 13>, int> geom_ids;
  auto geom_id = [&](const int v[4][3]) -> int {
    double p[4][3], g[4][3], vol;
    for (int j = 0; j < 4; ++j)
      for (int a = 0; a < 3; ++a) p[j][a] = d.h * (double)(v[j][a] - v[0][a]);
    if (!tet_geometry(p, g, &vol)) return -1;
    std::array<uint32_t, 13> key;
    float f[13];
    for (int j = 0; j < 4; ++j)
      for (int a = 0; a < 3; ++a) f[3 * j + a] = (float)g[j][a];
    f[12] = (float)vol;
    for (int i = 0; i < 13; ++i) std::memcpy(&key[i], &f[i], 4);
    auto it = geom_ids.find(key);
    if (it != geom_ids.end()) return it->second;
    const int id = (int)geom_ids.size();
    geom_ids.emplace(key, id);
    for (int i = 0; i < 12; ++i) m.geom.push_back(f[i]);                       // grad phi_j
    for (int i = 0; i < 12; ++i) m.geom.push_back((float)((double)vol * g[i / 3][i % 3]));  // |K| grad phi_j
    m.geom.push_back(f[12]);                                                     // |K|
    for (int i = 25; i < GEOM_STRIDE; ++i) m.geom.push_back(0.f);
    return id;
  };

  // Every tetrahedron of the Kuhn split is a translate of one of six shapes (one per axis
  // permutation), so its geometry id, gradients and volume are computed once per shape.
  int shape_gid[6];
  double shape_g[6][4][3], shape_vol[6];
  int shape_v[6][4][3];
  for (int q = 0; q < 6; ++q) {
    for (int a = 0; a < 3; ++a) shape_v[q][0][a] = 0;
    for (int k = 1; k < 4; ++k) {
      for (int a = 0; a < 3; ++a) shape_v[q][k][a] = shape_v[q][k - 1][a];
      shape_v[q][k][kPerms[q][k - 1]] += 1;
    }
    shape_gid[q] = geom_id(shape_v[q]);
    if (shape_gid[q] < 0) return "degenerate tetrahedron";
    double p4[4][3];
    for (int j = 0; j < 4; ++j)
      for (int a = 0; a < 3; ++a) p4[j][a] = d.h * (double)shape_v[q][j][a];
    tet_geometry(p4, shape_g[q], &shape_vol[q]);
  }

  // Every owned node (layer >= 1) has all 8 cells around it in the box, so its element star is
  // a translate of one star of 24 tetrahedra: its lumped mass (the sum of |K| / 4) and its
  // assembled stencil of 3x3 blocks, 27 lattice offsets x (K_ij, B_ij), are those of that star,
  // accumulated in FP64 (cells z, y, x, then shape, as everywhere else).
  double star[27][10] = {};
  double star_mass = 0.0;
  for (int cz = -1; cz <= 0; ++cz)
    for (int cy = -1; cy <= 0; ++cy)
      for (int cx = -1; cx <= 0; ++cx)
        for (int q = 0; q < 6; ++q) {
          int v[4][3];
          int k = -1;
          for (int j = 0; j < 4; ++j) {
            v[j][0] = cx + shape_v[q][j][0];
            v[j][1] = cy + shape_v[q][j][1];
            v[j][2] = cz + shape_v[q][j][2];
            if (v[j][0] == 0 && v[j][1] == 0 && v[j][2] == 0) k = j;
          }
          if (k < 0) continue;
          const double(&g4)[4][3] = shape_g[q];
          const double vol = shape_vol[q];
          star_mass += vol / 4.0;
          for (int j = 0; j < 4; ++j) {
            const int slot = (v[j][0] + 1) + 3 * (v[j][1] + 1) + 9 * (v[j][2] + 1);
            double* t = star[slot];
            t[0] += vol * (g4[k][0] * g4[j][0] + g4[k][1] * g4[j][1] + g4[k][2] * g4[j][2]);
            for (int r = 0; r < 3; ++r)
              for (int c = 0; c < 3; ++c) t[1 + 3 * r + c] += vol * g4[k][r] * g4[j][c];
          }
        }
  m.mass.assign(m.n_own, star_mass);
  m.stencil_ok = m.n_own > 0;
  std::vector<float> ref32(270);
  for (int slot = 0; slot < 27; ++slot)
    for (int q = 0; q < 10; ++q) ref32[slot * 10 + q] = (float)star[slot][q];

  // local id of a halo node of the current partition, by lattice index (stamped per partition)
  std::vector<int> hloc_of(elements ? m.n_fem : 0, 0), hloc_stamp(elements ? m.n_fem : 0, -1);

  m.halo_off.assign(m.n_part + 1, 0);
  m.col_base.assign(m.n_part, 0);
  m.ncol.assign(m.n_part, 0);
  m.col_off.clear();
  m.elems.clear();
  m.halo.clear();
  m.part_dims.assign(4 * m.n_part, 0);
  m.box_codes.clear();
  for (int p = 0; p < m.n_part; ++p) {
    const auto& r = prange[p];
    const int o0 = m.own_off[p], no = m.own_off[p + 1] - o0;
    m.max_own = std::max(m.max_own, no);
    {
      // staging box of the assembled-stencil kernel: the owned block and a one-node rim
      const int ox = r[1] - r[0], oy = r[3] - r[2], oz = r[5] - r[4];
      m.part_dims[4 * p] = ox;
      m.part_dims[4 * p + 1] = oy;
      m.part_dims[4 * p + 2] = oz;
      m.part_dims[4 * p + 3] = (int)m.box_codes.size();
      for (int z = r[4] - 1; z <= r[5]; ++z)
        for (int y = r[2] - 1; y <= r[3]; ++y)
          for (int x = r[0] - 1; x <= r[1]; ++x) m.box_codes.push_back(lat2int[L.idx(x, y, z)]);
      m.max_box = std::max(m.max_box, (ox + 2) * (oy + 2) * (oz + 2));
    }
    m.halo_off[p] = (int)m.halo.size();
    if (!elements) continue;
    // element kernel data: every tetrahedron touching an owned node, its halo and colouring
    auto owned_here = [&](const int v[3]) {
      return v[0] >= r[0] && v[0] < r[1] && v[1] >= r[2] && v[1] < r[3] && v[2] >= r[4] && v[2] < r[5];
    };
    struct El { int v[4][3]; int gid; };
    std::vector<El> els;
    for (int cz = std::max(r[4] - 1, 0); cz <= std::min(r[5] - 1, L.c[2] - 1); ++cz)
      for (int cy = std::max(r[2] - 1, 0); cy <= std::min(r[3] - 1, L.c[1] - 1); ++cy)
        for (int cx = std::max(r[0] - 1, 0); cx <= std::min(r[1] - 1, L.c[0] - 1); ++cx)
          for (int q = 0; q < 6; ++q) {
            El e;
            for (int k = 0; k < 4; ++k) {
              e.v[k][0] = cx + shape_v[q][k][0];
              e.v[k][1] = cy + shape_v[q][k][1];
              e.v[k][2] = cz + shape_v[q][k][2];
            }
            bool touches = false;
            for (int k = 0; k < 4; ++k) touches |= owned_here(e.v[k]);
            if (!touches) continue;
            e.gid = shape_gid[q];
            els.push_back(e);
          }
    // halo: non-owned vertices, ordered by internal code (owned ids, then layer-0 codes)
    auto code_less = [](int a, int b) {
      if ((a >= 0) != (b >= 0)) return a >= 0;
      return a >= 0 ? a < b : a > b;
    };
    std::vector<int> hcodes;
    for (const auto& e : els)
      for (int k = 0; k < 4; ++k)
        if (!owned_here(e.v[k])) hcodes.push_back(lat2int[L.idx(e.v[k][0], e.v[k][1], e.v[k][2])]);
    std::sort(hcodes.begin(), hcodes.end(), code_less);
    hcodes.erase(std::unique(hcodes.begin(), hcodes.end()), hcodes.end());
    const int nl = no + (int)hcodes.size();
    if (nl > FEM_LOC_MAX || no > FEM_OWN_MAX) return "FEM partition exceeds local node limit";
    if ((int)els.size() > FEM_ELEM_MAX) return "FEM partition exceeds the element limit";
    m.max_loc = std::max(m.max_loc, nl);
    m.max_elem = std::max(m.max_elem, (int)els.size());
    for (const auto& e : els)
      for (int k = 0; k < 4; ++k)
        if (!owned_here(e.v[k])) {
          const int64_t li = L.idx(e.v[k][0], e.v[k][1], e.v[k][2]);
          if (hloc_stamp[li] != p) {
            hloc_stamp[li] = p;
            hloc_of[li] = no + (int)(std::lower_bound(hcodes.begin(), hcodes.end(), lat2int[li], code_less) -
                                     hcodes.begin());
          }
        }
    m.halo.insert(m.halo.end(), hcodes.begin(), hcodes.end());
    // local ids, greedy colouring on shared owned nodes
    struct Pk { int loc[4]; int gid; int color; };
    std::vector<Pk> pk(els.size());
    std::vector<uint64_t> used(no, 0);
    int ncol = 0;
    for (size_t i = 0; i < els.size(); ++i) {
      uint64_t forbid = 0;
      for (int k = 0; k < 4; ++k) {
        const int64_t li = L.idx(els[i].v[k][0], els[i].v[k][1], els[i].v[k][2]);
        const int loc = owned_here(els[i].v[k]) ? lat2int[li] - o0 : hloc_of[li];
        pk[i].loc[k] = loc;
        if (loc < no) forbid |= used[loc];
      }
      if (forbid == ~0ull) return "FEM colouring needs more than 64 colours";
      int c = 0;
      while (forbid & (1ull << c)) ++c;
      pk[i].color = c;
      pk[i].gid = els[i].gid;
      for (int k = 0; k < 4; ++k)
        if (pk[i].loc[k] < no) used[pk[i].loc[k]] |= (1ull << c);
      ncol = std::max(ncol, c + 1);
    }
    m.max_colors = std::max(m.max_colors, ncol);
    std::stable_sort(pk.begin(), pk.end(), [](const Pk& a, const Pk& b) { return a.color < b.color; });
    m.col_base[p] = (int)m.col_off.size();
    m.ncol[p] = ncol;
    const int e0 = (int)m.elems.size();
    {
      size_t i = 0;
      for (int c = 0; c <= ncol; ++c) {
        while (i < pk.size() && pk[i].color < c) ++i;
        m.col_off.push_back(e0 + (int)i);
      }
    }
    for (const auto& q : pk) {
      if (q.gid >= (1 << 20)) return "geometry table exceeds 2^20 entries";
      uint64_t w = 0;
      for (int k = 0; k < 4; ++k) w |= (uint64_t)(q.loc[k] & 0x7FF) << (11 * k);
      w |= (uint64_t)q.gid << 44;
      m.elems.push_back(w);
    }
  }
  m.halo_off[m.n_part] = (int)m.halo.size();
  m.n_geom = (int)geom_ids.size();
  // compress the shared stencil to its non-zero slots
  m.n_slots = 0;
  m.slot_off.clear();
  m.slot_k.clear();
  m.slot_b.clear();
  if (m.stencil_ok && !ref32.empty()) {
    for (int slot = 0; slot < 27; ++slot) {
      bool nz = false;
      for (int q = 0; q < 10; ++q) nz |= ref32[slot * 10 + q] != 0.f;
      if (!nz) continue;
      m.slot_off.push_back(slot % 3 - 1);
      m.slot_off.push_back((slot / 3) % 3 - 1);
      m.slot_off.push_back(slot / 9 - 1);
      m.slot_off.push_back(0);
      m.slot_k.push_back(ref32[slot * 10]);
      for (int q = 1; q < 10; ++q) m.slot_b.push_back(ref32[slot * 10 + q]);
      ++m.n_slots;
    }
  } else {
    m.stencil_ok = false;
  }
  return std::string();
}

}  // namespace dd

// ---------------------------------------------------------------------------------------
// Host-only diagnostic: applies the FEM operator with exactly the data the FEM kernel
// consumes (partition halos, colours, packed connectivity, geometry table), in FP64 and
// sequentially, checking every index against its bound and every colour for conflicts.
// ---------------------------------------------------------------------------------------
namespace {
int debug_apply(const dd_problem_desc* d, const dd::HostMesh& m, const double* eps, const double* E, int flags,
                double* out, int64_t* stats) {
  const bool adjoint = (flags & 1) != 0, stencil = (flags & 2) != 0;
  using namespace dd;
  const int s[3] = {d->fem_cells[0] + 1, d->fem_cells[1] + 1, d->fem_cells[2] + 1};
  const int64_t n_own = m.n_own, n_l0 = m.n_l0;
  std::vector<double> X(3 * n_own), em1(n_own), iface(3 * n_l0, 0.0);
  std::vector<char> l0_seen(n_l0, 0);
  for (int64_t id = 0; id < n_own; ++id) {
    const int api = m.own_api[id];
    if (api < 0 || api >= m.n_fem) return DD_ERR_UNSUPPORTED;
    for (int c = 0; c < 3; ++c) X[c * n_own + id] = E[(int64_t)api * 3 + c];
    em1[id] = eps[api] - 1.0;
  }
  for (int z = 0; z < s[2]; ++z)
    for (int y = 0; y < s[1]; ++y)
      for (int x = 0; x < s[0]; ++x) {
        const int64_t q = face_lex_index(x, y, z, s[0], s[1], s[2], 63u);
        if (q < 0) continue;
        if (q >= n_l0 || l0_seen[q]) return DD_ERR_UNSUPPORTED;
        l0_seen[q] = 1;
        const int64_t api = x + (int64_t)s[0] * (y + (int64_t)s[1] * z);
        for (int c = 0; c < 3; ++c) iface[c * n_l0 + q] = E[api * 3 + c];
      }
  for (int64_t i = 0; i < 3 * m.n_fem; ++i) out[i] = 0.0;
  int64_t n_elem = 0;
  if (stencil) {
    if (!m.stencil_ok) return DD_ERR_UNSUPPORTED;
    for (int p = 0; p < m.n_part; ++p) {
      const int ox = m.part_dims[4 * p], oy = m.part_dims[4 * p + 1], oz = m.part_dims[4 * p + 2];
      const int base = m.part_dims[4 * p + 3], BX = ox + 2, BY = oy + 2, nbox = BX * BY * (oz + 2);
      const int o0 = m.own_off[p];
      if (ox * oy * oz != m.own_off[p + 1] - o0 || nbox > m.max_box) return DD_ERR_UNSUPPORTED;
      std::vector<double> bx(4 * nbox);
      for (int l = 0; l < nbox; ++l) {
        const int code = m.box_codes[base + l];
        if (code >= n_own) return DD_ERR_UNSUPPORTED;
        for (int c = 0; c < 3; ++c) bx[4 * l + c] = code >= 0 ? X[c * n_own + code] : iface[c * n_l0 + (-1 - code)];
        bx[4 * l + 3] = code >= 0 ? em1[code] : 0.0;
        if (code < 0 && -1 - code >= n_l0) return DD_ERR_UNSUPPORTED;
      }
      for (int l = 0; l < ox * oy * oz; ++l) {
        const int ix = l % ox, iy = (l / ox) % oy, iz = l / (ox * oy);
        const int li = (ix + 1) + BX * ((iy + 1) + BY * (iz + 1));
        double r[3] = {0, 0, 0}, q[3] = {0, 0, 0};
        for (int s = 0; s < m.n_slots; ++s) {
          const int n = li + m.slot_off[4 * s] + BX * (m.slot_off[4 * s + 1] + BY * m.slot_off[4 * s + 2]);
          if (n < 0 || n >= nbox) return DD_ERR_UNSUPPORTED;
          const double* x = &bx[4 * n];
          const double w = adjoint ? 1.0 : x[3];
          for (int c = 0; c < 3; ++c) {
            r[c] += (double)m.slot_k[s] * x[c];
            for (int e = 0; e < 3; ++e) q[c] += (double)m.slot_b[9 * s + 3 * c + e] * w * x[e];
          }
        }
        const int api = m.own_api[o0 + l];
        for (int c = 0; c < 3; ++c) out[(int64_t)api * 3 + c] = r[c] + (adjoint ? em1[o0 + l] : 1.0) * q[c];
      }
    }
  }
  for (int p = 0; p < m.n_part && !stencil; ++p) {
    const int o0 = m.own_off[p], no = m.own_off[p + 1] - o0;
    const int h0 = m.halo_off[p], nh = m.halo_off[p + 1] - h0;
    const int nl = no + nh;
    if (nl > FEM_LOC_MAX || no > FEM_OWN_MAX || o0 + no > n_own) return DD_ERR_UNSUPPORTED;
    std::vector<double> sX(3 * nl), sM(nl, 0.0), acc(6 * no, 0.0);
    for (int l = 0; l < nl; ++l) {
      if (l < no) {
        for (int c = 0; c < 3; ++c) sX[c * nl + l] = X[c * n_own + o0 + l];
        sM[l] = em1[o0 + l];
      } else {
        const int hc = m.halo[h0 + l - no];
        if (hc >= 0) {
          if (hc >= n_own) return DD_ERR_UNSUPPORTED;
          for (int c = 0; c < 3; ++c) sX[c * nl + l] = X[c * n_own + hc];
          sM[l] = em1[hc];
        } else {
          const int64_t q = -1 - (int64_t)hc;
          if (q >= n_l0) return DD_ERR_UNSUPPORTED;
          for (int c = 0; c < 3; ++c) sX[c * nl + l] = iface[c * n_l0 + q];
        }
      }
    }
    const int cb = m.col_base[p];
    for (int c = 0; c < m.ncol[p]; ++c) {
      std::vector<char> touched(no, 0);
      for (int e = m.col_off[cb + c]; e < m.col_off[cb + c + 1]; ++e) {
        ++n_elem;
        const uint64_t w = m.elems[e];
        int v[4];
        for (int k = 0; k < 4; ++k) {
          v[k] = (int)((w >> (11 * k)) & 0x7FFu);
          if (v[k] >= nl) return DD_ERR_UNSUPPORTED;
        }
        const uint64_t gid = w >> 44;
        if ((int64_t)gid >= m.n_geom) return DD_ERR_UNSUPPORTED;
        const float* g = &m.geom[GEOM_STRIDE * gid];
        double G[3][3] = {{0}}, dv = 0.0;
        for (int j = 0; j < 4; ++j) {
          const double mj = adjoint ? 1.0 : sM[v[j]];
          for (int q = 0; q < 3; ++q)
            for (int a = 0; a < 3; ++a) G[q][a] += sX[q * nl + v[j]] * g[3 * j + a];
          for (int a = 0; a < 3; ++a) dv += mj * sX[a * nl + v[j]] * g[3 * j + a];
        }
        const double vol = g[24];
        for (int k = 0; k < 4; ++k) {
          if (v[k] >= no) continue;
          if (touched[v[k]]) return DD_ERR_UNSUPPORTED;  // two elements of one colour share an owned node
          touched[v[k]] = 1;
          for (int q = 0; q < 3; ++q) {
            const double kc = vol * (g[3 * k] * G[q][0] + g[3 * k + 1] * G[q][1] + g[3 * k + 2] * G[q][2]);
            const double dc = vol * g[3 * k + q] * dv;
            acc[q * no + v[k]] += kc;
            acc[(3 + q) * no + v[k]] += dc;
          }
        }
      }
    }
    for (int l = 0; l < no; ++l) {
      const int api = m.own_api[o0 + l];
      for (int q = 0; q < 3; ++q)
        out[(int64_t)api * 3 + q] =
            acc[q * no + l] + (adjoint ? em1[o0 + l] : 1.0) * acc[(3 + q) * no + l];
    }
  }
  if (stats) {
    stats[0] = m.n_part;
    stats[1] = m.max_colors;
    stats[2] = m.max_loc;
    stats[3] = m.n_geom;
    stats[4] = n_elem;
    stats[5] = m.n_own;
    stats[6] = m.n_l0;
    stats[7] = m.stencil_ok ? m.n_slots : 0;
  }
  return DD_OK;
}
}  // namespace

extern "C" int dd_debug_fem_apply(const dd_problem_desc* d, const double* eps, const double* E, int flags,
                                  double* out, int64_t* stats) {
  if (!d || !eps || !E || !out) return DD_ERR_INVALID_ARG;
  dd::HostMesh m;
  const int pb[3] = {dd::FEM_PB, dd::FEM_PB, dd::FEM_PB};
  if (!dd::build_mesh(*d, m, pb, (flags & 2) == 0).empty()) return DD_ERR_UNSUPPORTED;
  return debug_apply(d, m, eps, E, flags, out, stats);
}

extern "C" int dd_debug_fem_apply_mesh(const dd_problem_desc* d, int64_t n_extra, const double* extra_xyz,
                                       int64_t n_tets, const int32_t* tets, const double* eps, const double* E,
                                       int flags, double* out, int64_t* stats) {
  if (!d || !eps || !E || !out || (flags & 2)) return DD_ERR_INVALID_ARG;
  dd::HostMesh m;
  const int pb[3] = {dd::FEM_PB, dd::FEM_PB, dd::FEM_PB};
  if (!dd::build_mesh_general(*d, n_extra, extra_xyz, n_tets, tets, m, pb).empty()) return DD_ERR_UNSUPPORTED;
  return debug_apply(d, m, eps, E, flags, out, stats);
}

namespace dd {

// General tetrahedral mesh of the FEM box: the box's lattice nodes (lexicographic) and n_extra
// extra nodes strictly inside it, and n_tets tetrahedra in those node indices.  Owned nodes
// (lattice layer >= 1, every extra node) are grouped by lattice blocks of 8^3 (an extra node
// joins the block of the cell it lies in); a block that does not fit the element kernel's
// limits is cut at the median of its nodes, recursively.  Everything else is built as for the
// Kuhn split's element path.
std::string build_mesh_general(const dd_problem_desc& d, int64_t n_extra, const double* xyz, int64_t n_tets,
                               const int32_t* tv, HostMesh& m, const int pb[3]) {
  Lattice L;
  for (int a = 0; a < 3; ++a) {
    L.c[a] = d.fem_cells[a];
    L.s[a] = d.fem_cells[a] + 1;
  }
  const int64_t n_lat = (int64_t)L.s[0] * L.s[1] * L.s[2];
  const int64_t n_fem = n_lat + n_extra;
  if (n_extra < 0 || n_tets < 1 || (n_extra > 0 && !xyz) || !tv) return "null or empty mesh";
  if (n_fem >= (1ll << 31)) return "mesh too large";
  // node coordinates relative to the box's lower corner, in units of h
  std::vector<std::array<double, 3>> P(n_fem);
  for (int z = 0; z < L.s[2]; ++z)
    for (int y = 0; y < L.s[1]; ++y)
      for (int x = 0; x < L.s[0]; ++x) P[L.idx(x, y, z)] = {(double)x, (double)y, (double)z};
  for (int64_t e = 0; e < n_extra; ++e)
    for (int a = 0; a < 3; ++a) {
      const double u = (xyz[3 * e + a] - d.origin[a]) / d.h - d.fem_lo[a];
      if (!(u > 0.0 && u < L.c[a])) return "an extra node lies outside the FEM box's interior";
      P[n_lat + e][a] = u;
    }
  auto layer_of = [&](int64_t i) -> int {
    if (i >= n_lat) return 2;   // extra nodes are free
    const int x = (int)(i % L.s[0]), y = (int)((i / L.s[0]) % L.s[1]), z = (int)(i / ((int64_t)L.s[0] * L.s[1]));
    return L.layer(x, y, z);
  };
  // geometry (FP64, lengths in h scaled back to physical units), volumes, node -> tets
  std::vector<int> deg(n_fem + 1, 0);
  std::vector<double> tvol(n_tets);
  double vol_sum = 0.0;
  for (int64_t t = 0; t < n_tets; ++t) {
    double p[4][3], g[4][3], vol;
    for (int k = 0; k < 4; ++k) {
      const int64_t v = tv[4 * t + k];
      if (v < 0 || v >= n_fem) return "a tetrahedron references a node that does not exist";
      ++deg[v];
    }
    for (int k = 0; k < 4; ++k)
      for (int a = 0; a < 3; ++a) p[k][a] = d.h * (P[tv[4 * t + k]][a] - P[tv[4 * t]][a]);
    if (!tet_geometry(p, g, &vol)) return "degenerate tetrahedron";
    tvol[t] = vol;
    vol_sum += vol;
  }
  const double box = d.h * d.h * d.h * (double)L.c[0] * L.c[1] * L.c[2];
  if (std::fabs(vol_sum - box) > 1e-9 * box) return "the tetrahedra do not fill the FEM box";
  std::vector<int> adj_off(n_fem + 1, 0), adj(4 * n_tets);
  for (int64_t i = 0; i < n_fem; ++i) adj_off[i + 1] = adj_off[i] + deg[i];
  {
    std::vector<int> fill(adj_off.begin(), adj_off.end() - 1);
    for (int64_t t = 0; t < n_tets; ++t)
      for (int k = 0; k < 4; ++k) adj[fill[tv[4 * t + k]]++] = (int)t;
  }
  for (int64_t i = 0; i < n_fem; ++i)
    if (layer_of(i) >= 1 && deg[i] == 0) return "a FEM-owned node lies on no tetrahedron";

  // the geometry table, deduplicated on the float32 image of the FP64 geometry
  std::map<std::array<uint32_t, 13>, int> geom_ids;
  m.geom.clear();
  std::vector<int> tgid(n_tets);
  for (int64_t t = 0; t < n_tets; ++t) {
    double p[4][3], g[4][3], vol;
    for (int k = 0; k < 4; ++k)
      for (int a = 0; a < 3; ++a) p[k][a] = d.h * (P[tv[4 * t + k]][a] - P[tv[4 * t]][a]);
    tet_geometry(p, g, &vol);
    std::array<uint32_t, 13> key;
    float f[13];
    for (int j = 0; j < 4; ++j)
      for (int a = 0; a < 3; ++a) f[3 * j + a] = (float)g[j][a];
    f[12] = (float)vol;
    for (int i = 0; i < 13; ++i) std::memcpy(&key[i], &f[i], 4);
    auto it = geom_ids.find(key);
    if (it == geom_ids.end()) {
      const int id = (int)geom_ids.size();
      if (id >= (1 << 20)) return "geometry table exceeds 2^20 entries";
      it = geom_ids.emplace(key, id).first;
      for (int i = 0; i < 12; ++i) m.geom.push_back(f[i]);
      for (int i = 0; i < 12; ++i) m.geom.push_back((float)(vol * g[i / 3][i % 3]));
      m.geom.push_back(f[12]);
      for (int i = 25; i < GEOM_STRIDE; ++i) m.geom.push_back(0.f);
    }
    tgid[t] = it->second;
  }
  m.n_geom = (int)geom_ids.size();
  m.n_fem = n_fem;
  m.n_l0 = face_lex_count(L.s[0], L.s[1], L.s[2], 63u);
  m.stencil_ok = false;
  m.n_slots = 0;

  // partitions: owned nodes by lattice blocks of pb cells (an extra node joins the block of the
  // cell it lies in, by its cell's lower corner); a block that exceeds the element kernel's
  // limits (owned, local nodes, elements, colours) is cut in two at the median of its nodes
  // along its longest extent, recursively, lower half first
  std::vector<std::vector<int64_t>> members;
  {
    const int ow[3] = {L.c[0] - 1, L.c[1] - 1, L.c[2] - 1};
    int npb[3];
    for (int a = 0; a < 3; ++a) npb[a] = (ow[a] + pb[a] - 1) / pb[a];
    auto block_of = [&](const std::array<double, 3>& q) {
      int b[3];
      for (int a = 0; a < 3; ++a) {
        int c = (int)std::floor(q[a]);
        c = std::min(std::max(c, 1), L.c[a] - 1);
        b[a] = (c - 1) / pb[a];
      }
      return b[0] + npb[0] * (b[1] + npb[1] * b[2]);
    };
    std::vector<std::vector<int64_t>> blocks(npb[0] * npb[1] * npb[2]);
    for (int64_t i = 0; i < n_fem; ++i)
      if (layer_of(i) >= 1) blocks[block_of(P[i])].push_back(i);   // lattice first, then extra: index order
    std::vector<int> mark(n_fem, -1), tstamp(n_tets, -1), lpos(n_fem, 0);
    int call = 0;
    // does a partition of these owned nodes fit (the same counts and greedy colouring as below)?
    auto fits_part = [&](const std::vector<int64_t>& own) {
      const int id = call++;
      for (size_t k = 0; k < own.size(); ++k) mark[own[k]] = id;
      std::vector<int> els;
      for (int64_t i : own)
        for (int a = adj_off[i]; a < adj_off[i + 1]; ++a)
          if (tstamp[adj[a]] != id) {
            tstamp[adj[a]] = id;
            els.push_back(adj[a]);
          }
      if ((int)own.size() > FEM_OWN_MAX || (int)els.size() > FEM_ELEM_MAX) return false;
      std::sort(els.begin(), els.end());
      std::vector<int64_t> halo;
      for (int t : els)
        for (int k = 0; k < 4; ++k)
          if (mark[tv[4 * t + k]] != id) halo.push_back(tv[4 * t + k]);
      std::sort(halo.begin(), halo.end());
      halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
      if ((int)(own.size() + halo.size()) > FEM_LOC_MAX) return false;
      for (size_t k = 0; k < own.size(); ++k) lpos[own[k]] = (int)k;   // valid where mark == id
      std::vector<uint64_t> used(own.size(), 0);
      for (int t : els) {
        uint64_t forbid = 0;
        for (int k = 0; k < 4; ++k) {
          const int64_t v = tv[4 * t + k];
          if (mark[v] == id) forbid |= used[lpos[v]];
        }
        if (forbid == ~0ull) return false;
        int c = 0;
        while (forbid & (1ull << c)) ++c;
        for (int k = 0; k < 4; ++k) {
          const int64_t v = tv[4 * t + k];
          if (mark[v] == id) used[lpos[v]] |= (1ull << c);
        }
      }
      return true;
    };
    std::vector<std::vector<int64_t>> stack;
    for (auto& b : blocks) {
      if (b.empty()) continue;
      stack.push_back(std::move(b));
      while (!stack.empty()) {
        std::vector<int64_t> v = std::move(stack.back());
        stack.pop_back();
        if (fits_part(v)) {
          members.push_back(std::move(v));
          continue;
        }
        if (v.size() < 2) return "the mesh is too dense for the FEM kernel's partitions";
        int ax = 0;
        double ext = -1.0;
        for (int a = 0; a < 3; ++a) {
          double lo = 1e300, hi = -1e300;
          for (int64_t i : v) {
            lo = std::min(lo, P[i][a]);
            hi = std::max(hi, P[i][a]);
          }
          if (hi - lo > ext) {
            ext = hi - lo;
            ax = a;
          }
        }
        std::vector<int64_t> w = v;
        std::stable_sort(w.begin(), w.end(), [&](int64_t a, int64_t b) { return P[a][ax] < P[b][ax]; });
        const size_t half = w.size() / 2;
        std::vector<int64_t> lo(w.begin(), w.begin() + half), hi(w.begin() + half, w.end());
        std::sort(lo.begin(), lo.end());
        std::sort(hi.begin(), hi.end());
        stack.push_back(std::move(hi));   // the lower half is taken first
        stack.push_back(std::move(lo));
      }
    }
  }
  {
    const int n_part = (int)members.size();
    // internal numbering: partition-major
    std::vector<int> code(n_fem);
    for (int z = 0; z < L.s[2]; ++z)
      for (int y = 0; y < L.s[1]; ++y)
        for (int x = 0; x < L.s[0]; ++x)
          if (L.layer(x, y, z) == 0)
            code[L.idx(x, y, z)] = -1 - (int)face_lex_index(x, y, z, L.s[0], L.s[1], L.s[2], 63u);
    HostMesh q;
    q.n_fem = n_fem;
    q.n_l0 = m.n_l0;
    q.n_part = n_part;
    q.own_off.assign(n_part + 1, 0);
    int next = 0;
    for (int p = 0; p < n_part; ++p) {
      q.own_off[p] = next;
      for (int64_t i : members[p]) code[i] = next++;
    }
    q.own_off[n_part] = next;
    q.n_own = next;
    q.own_grid.assign(next, -1);
    q.own_api.assign(next, 0);
    q.mass.assign(next, 0.0);
    for (int p = 0; p < n_part; ++p)
      for (int64_t i : members[p]) {
        const int id = code[i];
        q.own_api[id] = (int)i;
        if (i < n_lat && layer_of(i) == 1) {
          const int x = (int)(i % L.s[0]), y = (int)((i / L.s[0]) % L.s[1]), z = (int)(i / ((int64_t)L.s[0] * L.s[1]));
          const int64_t gx = d.fem_lo[0] + x, gy = d.fem_lo[1] + y, gz = d.fem_lo[2] + z;
          q.own_grid[id] = (int)(gx + (int64_t)d.n_outer[0] * (gy + (int64_t)d.n_outer[1] * gz));
        }
        double ms = 0.0;   // lumped mass: |K| / 4 over the incident tetrahedra, in index order
        for (int a = adj_off[i]; a < adj_off[i + 1]; ++a) ms += tvol[adj[a]] / 4.0;
        q.mass[id] = ms;
      }
    q.halo_off.assign(n_part + 1, 0);
    q.col_base.assign(n_part, 0);
    q.ncol.assign(n_part, 0);
    std::vector<int> stamp(n_tets, -1), loc_of(n_fem, 0), loc_stamp(n_fem, -1);
    bool fits = true;
    for (int p = 0; p < n_part && fits; ++p) {
      const int o0 = q.own_off[p], no = q.own_off[p + 1] - o0;
      std::vector<int> els;
      for (int64_t i : members[p])
        for (int a = adj_off[i]; a < adj_off[i + 1]; ++a)
          if (stamp[adj[a]] != p) {
            stamp[adj[a]] = p;
            els.push_back(adj[a]);
          }
      std::sort(els.begin(), els.end());
      auto owned_here = [&](int64_t v) { return layer_of(v) >= 1 && code[v] >= o0 && code[v] < o0 + no; };
      auto code_less = [](int a, int b) {
        if ((a >= 0) != (b >= 0)) return a >= 0;
        return a >= 0 ? a < b : a > b;
      };
      std::vector<int> hcodes;
      for (int t : els)
        for (int k = 0; k < 4; ++k)
          if (!owned_here(tv[4 * t + k])) hcodes.push_back(code[tv[4 * t + k]]);
      std::sort(hcodes.begin(), hcodes.end(), code_less);
      hcodes.erase(std::unique(hcodes.begin(), hcodes.end()), hcodes.end());
      const int nl = no + (int)hcodes.size();
      if (nl > FEM_LOC_MAX || no > FEM_OWN_MAX || (int)els.size() > FEM_ELEM_MAX) {
        fits = false;
        break;
      }
      q.max_loc = std::max(q.max_loc, nl);
      q.max_own = std::max(q.max_own, no);
      q.max_elem = std::max(q.max_elem, (int)els.size());
      for (int t : els)
        for (int k = 0; k < 4; ++k) {
          const int64_t v = tv[4 * t + k];
          if (owned_here(v)) continue;
          if (loc_stamp[v] != p) {
            loc_stamp[v] = p;
            loc_of[v] = no + (int)(std::lower_bound(hcodes.begin(), hcodes.end(), code[v], code_less) - hcodes.begin());
          }
        }
      q.halo_off[p] = (int)q.halo.size();
      q.halo.insert(q.halo.end(), hcodes.begin(), hcodes.end());
      struct Pk { int loc[4]; int gid; int color; };
      std::vector<Pk> pk(els.size());
      std::vector<uint64_t> used(no, 0);
      int ncol = 0;
      for (size_t e = 0; e < els.size(); ++e) {
        const int t = els[e];
        uint64_t forbid = 0;
        for (int k = 0; k < 4; ++k) {
          const int64_t v = tv[4 * t + k];
          const int loc = owned_here(v) ? code[v] - o0 : loc_of[v];
          pk[e].loc[k] = loc;
          if (loc < no) forbid |= used[loc];
        }
        if (forbid == ~0ull) {
          fits = false;
          break;
        }
        int c = 0;
        while (forbid & (1ull << c)) ++c;
        pk[e].color = c;
        pk[e].gid = tgid[t];
        for (int k = 0; k < 4; ++k)
          if (pk[e].loc[k] < no) used[pk[e].loc[k]] |= (1ull << c);
        ncol = std::max(ncol, c + 1);
      }
      if (!fits) break;
      q.max_colors = std::max(q.max_colors, ncol);
      std::stable_sort(pk.begin(), pk.end(), [](const Pk& a, const Pk& b) { return a.color < b.color; });
      q.col_base[p] = (int)q.col_off.size();
      q.ncol[p] = ncol;
      const int e0 = (int)q.elems.size();
      size_t i = 0;
      for (int c = 0; c <= ncol; ++c) {
        while (i < pk.size() && pk[i].color < c) ++i;
        q.col_off.push_back(e0 + (int)i);
      }
      for (const auto& r : pk) {
        uint64_t w = 0;
        for (int k = 0; k < 4; ++k) w |= (uint64_t)(r.loc[k] & 0x7FF) << (11 * k);
        w |= (uint64_t)r.gid << 44;
        q.elems.push_back(w);
      }
    }
    if (!fits) return "the mesh is too dense for the FEM kernel's partitions";
    q.halo_off[n_part] = (int)q.halo.size();
    q.geom.swap(m.geom);
    q.n_geom = m.n_geom;
    q.stencil_ok = false;
    m = std::move(q);
    return std::string();
  }
}

}  // namespace dd

// ---------------------------------------------------------------------------------------
// Local refinement of a FEM mesh (box "ACGA", steps 2 and 3, eq. meshref), host only.
//
// Marking: h_K is an element's diameter (its longest edge) and eps, sigma are nodal; element K
// is marked when at one of its vertices v both h_K |eps(v)| >= beta_eps M_eps and
// h_K |sigma(v)| >= beta_sig M_sig hold, M the largest such product over all elements and
// their vertices.
//
// Refining: longest-edge bisection with propagation.  Element K is bisected at its longest
// edge e (ties within 1e-9: the smaller (low, high) pair of node ids), together with every
// element around e, at e's midpoint; any element around e whose own longest edge is another
// one is bisected first, the same way (recursively, in increasing element id), so that every
// element is split at its longest edge and the shapes do not degenerate.  An edge is bisected
// only when every element around it has all four vertices FEM-owned (lattice layer >= 1), so
// the overlap layers keep their lattice elements; a marked element whose propagation reaches
// another edge is left as it is.  Marked elements are taken in element order; the k-th
// bisection's midpoint becomes node n + k; an element split at (a, b), a < b, becomes its half
// with b replaced by the midpoint and its half with a replaced by it, in that order in the
// element list (children take ids after all existing ones).  Interpolation: each midpoint, in
// bisection order, takes the mean of its edge's endpoints (so the refined mesh carries the
// same piecewise-linear function), in FP64, rounded once to float32.
// ---------------------------------------------------------------------------------------
struct dd_refinement {
  int64_t n_old = 0;                           // FEM nodes of the input mesh
  int64_t n_tets_in = 0, n_marked = 0;
  std::vector<uint8_t> marks;                  // per input element
  std::vector<std::array<int64_t, 2>> split;   // bisected edges, in order
  std::vector<double> xyz;                     // extra nodes of the refined mesh (old, then new)
  std::vector<int32_t> tets;                   // refined elements
};

namespace {
// Kuhn tetrahedron q of cell (i, j, k): its four vertices as lattice coordinates.
void kuhn_tet(int i, int j, int k, int q, int v[4][3]) {
  static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  v[0][0] = i; v[0][1] = j; v[0][2] = k;
  for (int s = 1; s < 4; ++s) {
    for (int a = 0; a < 3; ++a) v[s][a] = v[s - 1][a];
    ++v[s][perm[q][s - 1]];
  }
}

using Edge = std::pair<int64_t, int64_t>;
inline Edge edge_of(int64_t a, int64_t b) { return a < b ? Edge(a, b) : Edge(b, a); }
constexpr double TIE = 1e-9;

struct Refiner {
  std::vector<std::array<double, 3>> P;        // node positions in units of h from the box corner
  std::vector<int> layer;                      // lattice layer; midpoints and extra nodes: free
  std::vector<std::array<int64_t, 4>> verts;   // element id -> vertices (leaves: the current mesh)
  std::vector<std::array<int64_t, 2>> kids;    // {-1, -1} for a leaf
  // Elements around each edge.  The input elements' edges are indexed once: grouped by their
  // low vertex (off / ent), each group sorted by (high vertex, element).  Elements created by
  // bisection are appended to `added` under their edges.  A lookup returns the leaves among
  // them: an element stops containing its edges when it is bisected, and its children take
  // new, larger ids, so the input entries followed by the added ones are in increasing id.
  int64_t n_in = 0;
  std::vector<int64_t> off;
  std::vector<std::pair<int32_t, int32_t>> ent;
  std::unordered_map<uint64_t, std::vector<int64_t>> added;
  static uint64_t key(const Edge& e) { return ((uint64_t)e.first << 32) | (uint64_t)e.second; }
  void index_input() {
    n_in = (int64_t)verts.size();
    off.assign(P.size() + 1, 0);
    for (int64_t t = 0; t < n_in; ++t)
      for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b) ++off[edge_of(verts[t][a], verts[t][b]).first + 1];
    for (size_t i = 1; i < off.size(); ++i) off[i] += off[i - 1];
    ent.resize((size_t)off.back());
    std::vector<int64_t> pos(off.begin(), off.end() - 1);
    for (int64_t t = 0; t < n_in; ++t)
      for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b) {
          const Edge e = edge_of(verts[t][a], verts[t][b]);
          ent[(size_t)pos[e.first]++] = {(int32_t)e.second, (int32_t)t};
        }
    for (size_t i = 0; i + 1 < off.size(); ++i) std::sort(ent.begin() + off[i], ent.begin() + off[i + 1]);
  }
  bool leaf(int64_t t) const { return kids[t][0] < 0; }
  std::vector<int64_t> around(const Edge& e) const {
    std::vector<int64_t> res;
    const auto b = ent.begin() + off[e.first], en = ent.begin() + off[e.first + 1];
    for (auto it = std::lower_bound(b, en, std::make_pair((int32_t)e.second, INT32_MIN));
         it != en && it->first == (int32_t)e.second; ++it)
      if (leaf(it->second)) res.push_back(it->second);
    const auto o = added.find(key(e));
    if (o != added.end())
      for (int64_t t : o->second)
        if (leaf(t)) res.push_back(t);
    return res;
  }
  std::vector<Edge> split;

  double len2(const Edge& e) const {
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double d = P[e.first][a] - P[e.second][a];
      s += d * d;
    }
    return s;
  }
  Edge longest(int64_t t) const {
    const auto& v = verts[t];
    Edge es[6];
    double l2[6], top = 0.0;
    int n = 0;
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b) {
        es[n] = edge_of(v[a], v[b]);
        l2[n] = len2(es[n]);
        top = std::max(top, l2[n]);
        ++n;
      }
    Edge best(INT64_MAX, INT64_MAX);
    for (int i = 0; i < 6; ++i)
      if (l2[i] >= (1.0 - TIE) * top && es[i] < best) best = es[i];
    return best;
  }
  void add(int64_t t) {
    const auto& v = verts[t];
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b) added[key(edge_of(v[a], v[b]))].push_back(t);
  }
  bool eligible(const Edge& e) const {
    const std::vector<int64_t> ts = around(e);
    if (ts.empty()) return false;
    for (int64_t t : ts)
      for (int64_t v : verts[t])
        if (layer[v] < 1) return false;
    return true;
  }
  void bisect(const Edge& e) {
    const int64_t m = (int64_t)P.size();
    std::array<double, 3> q;
    for (int a = 0; a < 3; ++a) q[a] = 0.5 * (P[e.first][a] + P[e.second][a]);
    P.push_back(q);
    layer.push_back(1 << 30);
    split.push_back(e);
    for (int64_t t : around(e)) {   // increasing id; each becomes a non-leaf below
      const auto v = verts[t];
      std::array<int64_t, 4> h0 = v, h1 = v;
      for (int a = 0; a < 4; ++a) {
        if (h0[a] == e.second) h0[a] = m;
        if (h1[a] == e.first) h1[a] = m;
      }
      const int64_t c0 = (int64_t)verts.size();
      verts.push_back(h0);
      kids.push_back({-1, -1});
      add(c0);
      verts.push_back(h1);
      kids.push_back({-1, -1});
      add(c0 + 1);
      kids[t] = {c0, c0 + 1};
    }
  }
  bool refine_element(int64_t t) {
    while (kids[t][0] < 0) {
      const Edge e = longest(t);
      if (!eligible(e)) return false;
      std::vector<int64_t> others;
      for (int64_t u : around(e))
        if (longest(u) != e) others.push_back(u);   // increasing id
      if (others.empty()) {
        bisect(e);
        return true;
      }
      for (int64_t u : others)
        if (kids[u][0] < 0 && !refine_element(u)) return false;
    }
    return true;
  }
  void emit(int64_t t, std::vector<int32_t>& out) const {
    if (kids[t][0] >= 0) {
      emit(kids[t][0], out);
      emit(kids[t][1], out);
    } else {
      for (int64_t v : verts[t]) out.push_back((int32_t)v);
    }
  }
};
}  // namespace

extern "C" int dd_meshref_create(const dd_problem_desc* d, int64_t n_extra, const double* extra_xyz, int64_t n_tets,
                                 const int32_t* tets, const float* eps, const float* sig, double beta_eps,
                                 double beta_sig, dd_refinement** out) {
  if (!out) return DD_ERR_INVALID_ARG;
  *out = nullptr;
  if (!d || !eps || !sig || !(beta_eps >= 0.0 && beta_eps <= 1.0) || !(beta_sig >= 0.0 && beta_sig <= 1.0) ||
      n_extra < 0 || n_tets < 0 || (n_extra > 0 && !extra_xyz) || (n_tets > 0 && !tets) || (n_tets == 0 && n_extra))
    return DD_ERR_INVALID_ARG;
  const int c[3] = {d->fem_cells[0], d->fem_cells[1], d->fem_cells[2]};
  if (c[0] < 2 || c[1] < 2 || c[2] < 2 || !(d->h > 0.0)) return DD_ERR_INVALID_ARG;
  const int s0 = c[0] + 1, s1 = c[1] + 1, s2 = c[2] + 1;
  const int64_t n_lat = (int64_t)s0 * s1 * s2;
  const int64_t n_old = n_lat + n_extra;
  if (n_old >= (1ll << 31)) return DD_ERR_INVALID_ARG;
  Refiner R;
  R.P.resize(n_old);
  R.layer.resize(n_old);
  for (int z = 0; z < s2; ++z)
    for (int y = 0; y < s1; ++y)
      for (int x = 0; x < s0; ++x) {
        const int64_t i = x + (int64_t)s0 * (y + (int64_t)s1 * z);
        R.P[i] = {(double)x, (double)y, (double)z};
        R.layer[i] = std::min({x, c[0] - x, y, c[1] - y, z, c[2] - z});
      }
  for (int64_t e = 0; e < n_extra; ++e) {
    for (int a = 0; a < 3; ++a) {
      const double u = (extra_xyz[3 * e + a] - d->origin[a]) / d->h - d->fem_lo[a];
      if (!(u > 0.0 && u < c[a])) return DD_ERR_INVALID_ARG;
      R.P[n_lat + e][a] = u;
    }
    R.layer[n_lat + e] = 1 << 30;
  }
  if (n_tets == 0) {
    for (int k = 0; k < c[2]; ++k)
      for (int j = 0; j < c[1]; ++j)
        for (int i = 0; i < c[0]; ++i)
          for (int q = 0; q < 6; ++q) {
            int v[4][3];
            kuhn_tet(i, j, k, q, v);
            std::array<int64_t, 4> id;
            for (int s = 0; s < 4; ++s) id[s] = v[s][0] + (int64_t)s0 * (v[s][1] + (int64_t)s1 * v[s][2]);
            R.verts.push_back(id);
          }
  } else {
    for (int64_t t = 0; t < n_tets; ++t) {
      std::array<int64_t, 4> id;
      for (int s = 0; s < 4; ++s) {
        id[s] = tets[4 * t + s];
        if (id[s] < 0 || id[s] >= n_old) return DD_ERR_INVALID_ARG;
      }
      R.verts.push_back(id);
    }
  }
  const int64_t nt = (int64_t)R.verts.size();
  if (nt >= (1ll << 31)) return DD_ERR_INVALID_ARG;   // element ids are indexed as 32-bit values
  R.kids.assign(nt, {-1, -1});
  // step 2: marks
  std::vector<double> hk(nt);
  double me = 0.0, ms = 0.0;
  for (int64_t t = 0; t < nt; ++t) {
    double top = 0.0;
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b) top = std::max(top, R.len2(edge_of(R.verts[t][a], R.verts[t][b])));
    hk[t] = std::sqrt(top);
    for (int64_t v : R.verts[t]) {
      me = std::max(me, hk[t] * std::fabs((double)eps[v]));
      ms = std::max(ms, hk[t] * std::fabs((double)sig[v]));
    }
  }
  auto* r = new dd_refinement();
  r->n_old = n_old;
  r->n_tets_in = nt;
  r->marks.assign(nt, 0);
  const double te = beta_eps * me, ts = beta_sig * ms;
  for (int64_t t = 0; t < nt; ++t)
    for (int64_t v : R.verts[t])
      if (hk[t] * std::fabs((double)eps[v]) >= te && hk[t] * std::fabs((double)sig[v]) >= ts) {
        r->marks[t] = 1;
        ++r->n_marked;
        break;
      }
  // step 3: bisection
  R.index_input();
  for (int64_t t = 0; t < nt; ++t)
    if (r->marks[t] && R.kids[t][0] < 0) R.refine_element(t);
  for (int64_t t = 0; t < nt; ++t) R.emit(t, r->tets);
  r->split.reserve(R.split.size());
  for (const Edge& e : R.split) r->split.push_back({e.first, e.second});
  r->xyz.assign(extra_xyz, extra_xyz + 3 * n_extra);
  for (size_t k = 0; k < R.split.size(); ++k) {
    const auto& q = R.P[n_old + k];
    for (int a = 0; a < 3; ++a) r->xyz.push_back(d->origin[a] + d->h * (d->fem_lo[a] + q[a]));
  }
  *out = r;
  return DD_OK;
}

extern "C" int dd_meshref_sizes(const dd_refinement* r, int64_t* n_marked, int64_t* n_bisected, int64_t* n_extra,
                                int64_t* n_tets) {
  if (!r) return DD_ERR_INVALID_ARG;
  if (n_marked) *n_marked = r->n_marked;
  if (n_bisected) *n_bisected = (int64_t)r->split.size();
  if (n_extra) *n_extra = (int64_t)r->xyz.size() / 3;
  if (n_tets) *n_tets = (int64_t)r->tets.size() / 4;
  return DD_OK;
}

extern "C" int dd_meshref_result(const dd_refinement* r, uint8_t* marks, double* extra_xyz, int32_t* tets) {
  if (!r || (!extra_xyz && !r->xyz.empty()) || !tets) return DD_ERR_INVALID_ARG;
  if (marks) std::memcpy(marks, r->marks.data(), r->marks.size());
  if (!r->xyz.empty()) std::memcpy(extra_xyz, r->xyz.data(), r->xyz.size() * sizeof(double));
  std::memcpy(tets, r->tets.data(), r->tets.size() * sizeof(int32_t));
  return DD_OK;
}

extern "C" int dd_meshref_interpolate(const dd_refinement* r, const float* in, float* out) {
  if (!r || !in || !out) return DD_ERR_INVALID_ARG;
  std::vector<double> v(in, in + r->n_old);
  v.reserve(r->n_old + r->split.size());
  for (const auto& e : r->split) v.push_back(0.5 * (v[e[0]] + v[e[1]]));
  for (size_t i = 0; i < v.size(); ++i) out[i] = (float)v[i];
  return DD_OK;
}

extern "C" int dd_meshref_destroy(dd_refinement* r) {
  delete r;
  return DD_OK;
}
