// Host setup: meshes, the dof map of C_{N,k}, boundary dofs, reference tables and
// the cell tiling used by the device kernels.
#include <algorithm>
#include <array>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "internal.hpp"
#include "reftab.hpp"

namespace dogip {

// ---------------------------------------------------------------- meshes

static double cell_det(int dim, const double* X) {
  // X: (dim+1) vertices of dim coordinates; R columns X_r - X_0
  if (dim == 2) {
    double a = X[2] - X[0], b = X[4] - X[0], c = X[3] - X[1], d = X[5] - X[1];
    return a * d - b * c;
  }
  double r[3][3];
  for (int x = 0; x < 3; ++x)
    for (int c = 0; c < 3; ++c) r[x][c] = X[(c + 1) * 3 + x] - X[x];
  return r[0][0] * (r[1][1] * r[2][2] - r[1][2] * r[2][1]) - r[0][1] * (r[1][0] * r[2][2] - r[1][2] * r[2][0]) +
         r[0][2] * (r[1][0] * r[2][1] - r[1][1] * r[2][0]);
}

std::shared_ptr<Mesh> make_mesh(int dim, int64_t nv, const double* xyz, int64_t nc, const int32_t* cells) {
  DOGIP_CHECK(dim == 2 || dim == 3, DOGIP_E_RANGE, "dim must be 2 or 3");
  DOGIP_CHECK(nv > 0 && nc > 0, DOGIP_E_INVALID, "empty mesh");
  DOGIP_CHECK(xyz && cells, DOGIP_E_NULL, "null coordinate or cell array");
  DOGIP_CHECK(nv < (int64_t(1) << 31), DOGIP_E_RANGE, "too many vertices");
  auto m = std::make_shared<Mesh>();
  m->dim = dim;
  m->nv = nv;
  m->nc = nc;
  m->xyz.assign(xyz, xyz + nv * dim);
  m->cells.assign(cells, cells + nc * (dim + 1));
  std::vector<uint8_t> used(nv, 0);
  double X[12];
  for (int64_t c = 0; c < nc; ++c) {
    double hmax = 0;
    for (int j = 0; j <= dim; ++j) {
      int32_t v = m->cells[c * (dim + 1) + j];
      DOGIP_CHECK(v >= 0 && v < nv, DOGIP_E_INVALID, "cell " + std::to_string(c) + " has an out-of-range vertex");
      used[v] = 1;
      for (int x = 0; x < dim; ++x) X[j * dim + x] = m->xyz[int64_t(v) * dim + x];
    }
    for (int a = 0; a <= dim; ++a)
      for (int b = a + 1; b <= dim; ++b) {
        double s = 0;
        for (int x = 0; x < dim; ++x) s += (X[a * dim + x] - X[b * dim + x]) * (X[a * dim + x] - X[b * dim + x]);
        hmax = std::max(hmax, std::sqrt(s));
      }
    double det = cell_det(dim, X);
    DOGIP_CHECK(std::isfinite(det) && std::fabs(det) > 1e-14 * std::pow(hmax, dim), DOGIP_E_INVALID,
                "cell " + std::to_string(c) + " is degenerate (det R_T = 0)");
  }
  for (int64_t v = 0; v < nv; ++v)
    DOGIP_CHECK(used[v], DOGIP_E_INVALID, "vertex " + std::to_string(v) + " belongs to no cell");
  return m;
}

std::shared_ptr<Mesh> make_unit_mesh(int dim, int n) {
  DOGIP_CHECK(dim == 2 || dim == 3, DOGIP_E_RANGE, "dim must be 2 or 3");
  DOGIP_CHECK(n >= 1 && n <= (dim == 2 ? 16384 : 1024), DOGIP_E_RANGE, "n out of range");
  const int64_t m = n + 1;
  const int64_t nv = dim == 2 ? m * m : m * m * m;
  std::vector<double> xyz(nv * dim);
  for (int64_t v = 0; v < nv; ++v) {
    int64_t i = v % m, j = (v / m) % m, l = v / (m * m);
    xyz[v * dim + 0] = double(i) / n;
    xyz[v * dim + 1] = double(j) / n;
    if (dim == 3) xyz[v * dim + 2] = double(l) / n;
  }
  std::vector<int32_t> cells;
  if (dim == 2) {
    cells.resize(int64_t(2) * n * n * 3);
    int64_t c = 0;
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) {
        int32_t v00 = int32_t(i + m * j), v10 = v00 + 1, v01 = int32_t(v00 + m), v11 = v01 + 1;
        int32_t t[6] = {v00, v10, v11, v00, v11, v01};
        std::memcpy(&cells[c * 3], t, sizeof t);
        c += 2;
      }
  } else {
    cells.resize(int64_t(6) * n * n * n * 4);
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int64_t c = 0;
    for (int64_t l = 0; l < n; ++l)
      for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
          for (int p = 0; p < 6; ++p) {
            int64_t o[3] = {i, j, l};
            cells[c * 4 + 0] = int32_t(o[0] + m * (o[1] + m * o[2]));
            for (int s = 0; s < 3; ++s) {
              o[perms[p][s]] += 1;
              cells[c * 4 + 1 + s] = int32_t(o[0] + m * (o[1] + m * o[2]));
            }
            ++c;
          }
  }
  auto out = make_mesh(dim, nv, xyz.data(), int64_t(cells.size()) / (dim + 1), cells.data());
  out->unit_n = n;
  return out;
}

// ---------------------------------------------------------------- reference tables

void reference_tables(int dim, int k, int kind, std::vector<double>& bhat, std::vector<double>& what, int64_t& nnz,
                      int64_t& nnz_pm1) {
  const int vt = dim_p(dim, k), q = w_order(k, kind), wt = dim_p(dim, q), nb = kind == KIND_SE ? dim : 1;
  bhat.assign(size_t(nb) * wt * vt, 0.0);
  what.assign(wt, 0.0);
  nnz = nnz_pm1 = 0;
  for (int r = 0; r < nb; ++r)
    for (int i = 0; i < wt; ++i)
      for (int l = 0; l < vt; ++l) {
        ref::Q v = ref::bhat_entry(dim, k, kind, r, i, l);
        bhat[(size_t(r) * wt + i) * vt + l] = ref::to_double(v);
        if (!ref::is_zero(v)) ++nnz;
        if (v.d == 1 && (v.n == 1 || v.n == -1)) ++nnz_pm1;
      }
  for (int i = 0; i < wt; ++i) what[i] = ref::to_double(ref::what_entry(dim, q, i));
}

// ---------------------------------------------------------------- space-filling order

static uint64_t spread3(uint64_t x) {  // 21 bits -> every third bit
  x &= 0x1fffff;
  x = (x | x << 32) & 0x1f00000000ffffULL;
  x = (x | x << 16) & 0x1f0000ff0000ffULL;
  x = (x | x << 8) & 0x100f00f00f00f00fULL;
  x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
  x = (x | x << 2) & 0x1249249249249249ULL;
  return x;
}
static uint64_t spread2(uint64_t x) {  // 32 bits -> every second bit
  x &= 0xffffffffULL;
  x = (x | x << 16) & 0x0000ffff0000ffffULL;
  x = (x | x << 8) & 0x00ff00ff00ff00ffULL;
  x = (x | x << 4) & 0x0f0f0f0f0f0f0f0fULL;
  x = (x | x << 2) & 0x3333333333333333ULL;
  x = (x | x << 1) & 0x5555555555555555ULL;
  return x;
}

// Order of n points (coordinates [n][d]) along the Morton curve of their bounding
// box; ties keep the input order.
static std::vector<int64_t> morton_order(const double* xyz, int64_t n, int d) {
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = 0; i < n; ++i)
    for (int x = 0; x < d; ++x) {
      lo[x] = std::min(lo[x], xyz[i * d + x]);
      hi[x] = std::max(hi[x], xyz[i * d + x]);
    }
  const double bits = d == 3 ? 2097151.0 : 4294967295.0;
  std::vector<std::pair<uint64_t, int64_t>> key(n);
  parallel_for(n, [&](int64_t i) {
    uint64_t code = 0;
    for (int x = 0; x < d; ++x) {
      const double t = hi[x] > lo[x] ? (xyz[i * d + x] - lo[x]) / (hi[x] - lo[x]) : 0.0;
      const uint64_t qv = uint64_t(std::min(std::max(t, 0.0), 1.0) * bits);
      code |= (d == 3 ? spread3(qv) : spread2(qv)) << x;
    }
    key[i] = {code, i};
  });
  // LSD radix sort on 16-bit digits: each pass is a stable counting sort, so equal codes
  // keep ascending index order (the order of sorting the (code, index) pairs).  A pass
  // splits the keys into contiguous ranges, one per thread: per-range digit counts, then
  // each range scatters from its own offsets (range r's keys of a digit follow those of
  // ranges < r), which keeps the pass stable
  const int64_t nr = std::max<int64_t>(
      1, std::min<int64_t>({n / 65536, 16, int64_t(std::max(1u, std::thread::hardware_concurrency()))}));
  const int64_t chunk = (n + nr - 1) / nr;
  std::vector<std::pair<uint64_t, int64_t>> tmp(n);
  std::vector<int64_t> cnt(size_t(nr) * 65536);
  for (int shift = 0; shift < 64; shift += 16) {
    std::fill(cnt.begin(), cnt.end(), 0);
    parallel_tasks(nr, [&](int64_t r) {
      int64_t* c = &cnt[size_t(r) * 65536];
      for (int64_t i = r * chunk; i < std::min(n, (r + 1) * chunk); ++i) c[(key[i].first >> shift) & 0xffff]++;
    });
    // offsets in (digit, range) order; a single digit value throughout leaves the order as is
    bool trivial = false;
    int64_t run = 0;
    for (int b = 0; b < 65536; ++b) {
      int64_t tot = 0;
      for (int64_t r = 0; r < nr; ++r) {
        const int64_t c = cnt[size_t(r) * 65536 + b];
        cnt[size_t(r) * 65536 + b] = run + tot;
        tot += c;
      }
      if (tot == n) trivial = true;
      run += tot;
    }
    if (trivial) continue;
    parallel_tasks(nr, [&](int64_t r) {
      int64_t* c = &cnt[size_t(r) * 65536];
      for (int64_t i = r * chunk; i < std::min(n, (r + 1) * chunk); ++i) tmp[c[(key[i].first >> shift) & 0xffff]++] = key[i];
    });
    key.swap(tmp);
  }
  std::vector<int64_t> order(n);
  parallel_for(n, [&](int64_t i) { order[i] = key[i].second; });
  return order;
}

// ---------------------------------------------------------------- dof map

namespace {

struct EntityIds {
  std::vector<int32_t> cell_ent;  // [nc][n_local] entity id
  std::vector<int32_t> count;     // cells per entity
  int64_t n = 0;
};

// Number the distinct vertex tuples (sorted) taken from each cell: local tuples
// are given by lists of local vertex indices.
template <int NV>
EntityIds number_entities(const Mesh& m, const std::vector<std::array<int, NV>>& loc) {
  const int d1 = m.dim + 1, nl = int(loc.size());
  struct Key {
    std::array<int32_t, NV> v;
    int64_t slot;
  };
  std::vector<Key> keys(size_t(m.nc) * nl);
  parallel_for(m.nc, [&](int64_t c) {
    for (int e = 0; e < nl; ++e) {
      Key& k = keys[size_t(c) * nl + e];
      for (int t = 0; t < NV; ++t) k.v[t] = m.cells[c * d1 + loc[e][t]];
      std::sort(k.v.begin(), k.v.end());
      k.slot = c * nl + e;
    }
  });
  // lexicographic order of the tuples: a counting sort by the smallest vertex id, then
  // each bucket (the entities around one vertex, a few dozen) sorted on the full tuple
  {
    std::vector<int64_t> start(size_t(m.nv) + 1, 0);
    for (const Key& k : keys) start[size_t(k.v[0]) + 1]++;
    for (int64_t v = 0; v < m.nv; ++v) start[v + 1] += start[v];
    std::vector<Key> by(keys.size());
    std::vector<int64_t> at(start.begin(), start.end() - 1);
    for (const Key& k : keys) by[at[k.v[0]]++] = k;
    // (equal tuples get one id whatever their order, so the buckets sort independently)
    parallel_for(m.nv, [&](int64_t v) {
      std::sort(by.begin() + start[v], by.begin() + start[v + 1], [](const Key& a, const Key& b) { return a.v < b.v; });
    });
    keys.swap(by);
  }
  EntityIds ids;
  ids.cell_ent.assign(size_t(m.nc) * nl, -1);
  int64_t id = -1;
  for (size_t i = 0; i < keys.size(); ++i) {
    if (i == 0 || keys[i].v != keys[i - 1].v) {
      ++id;
      ids.count.push_back(0);
    }
    ids.cell_ent[keys[i].slot] = int32_t(id);
    ids.count[id]++;
  }
  ids.n = id + 1;
  return ids;
}

int tri_index(int i, int j, int n) { return i * (n + 1) - i * (i - 1) / 2 + j; }

// local edges (a, b), a < b, in the order (0,1), (0,2), ..., (d-1,d)
std::vector<std::array<int, 2>> local_edges(int d) {
  std::vector<std::array<int, 2>> e;
  for (int a = 0; a <= d; ++a)
    for (int b = a + 1; b <= d; ++b) e.push_back({a, b});
  return e;
}

int local_edge_of(const std::vector<std::array<int, 2>>& le, int a, int b) {
  if (a > b) std::swap(a, b);
  for (size_t e = 0; e < le.size(); ++e)
    if (le[e][0] == a && le[e][1] == b) return int(e);
  return -1;
}

}  // namespace

std::shared_ptr<const MeshEntities> mesh_entities(const Mesh& m) {
  std::lock_guard<std::mutex> lock(m.ent_mu);
  if (m.ent) return m.ent;
  auto out = std::make_shared<MeshEntities>();
  EntityIds E = number_entities<2>(m, local_edges(m.dim));
  out->cell_edge.swap(E.cell_ent);
  out->edge_cells.swap(E.count);
  out->ne = E.n;
  if (m.dim == 3) {
    // face opposite local vertex j
    std::vector<std::array<int, 3>> lf;
    for (int j = 0; j < 4; ++j) {
      std::array<int, 3> f{};
      int t = 0;
      for (int a = 0; a < 4; ++a)
        if (a != j) f[t++] = a;
      lf.push_back(f);
    }
    EntityIds F = number_entities<3>(m, lf);
    out->cell_face.swap(F.cell_ent);
    out->face_cells.swap(F.count);
    out->nf = F.n;
  }
  m.ent = out;
  return out;
}

// Lagrange nodes of order q on every cell of the mesh, numbered globally:
// vertices, then the q-1 nodes of each edge, the (q-1)(q-2)/2 of each face (3D),
// then the cell-interior nodes.  A node shared by several cells gets one number
// whatever the cells' local vertex orders (edge and face nodes are keyed by
// vertex ids and multiplicities).  With xyz, also the node coordinates and the
// flag of nodes on boundary facets.
LatticeDofs number_lattice(const Mesh& m, int q, bool xyz) {
  const int d = m.dim, d1 = d + 1;
  LatticeDofs out;
  out.nl = dim_p(d, q);
  const std::vector<std::array<int, 2>> ledges = local_edges(d);
  const int nle = int(ledges.size());
  const std::shared_ptr<const MeshEntities> ent = mesh_entities(m);
  const MeshEntities& M = *ent;
  const int64_t ne1 = q - 1, nf1 = d == 3 ? int64_t(q - 1) * (q - 2) / 2 : 0;
  const int64_t nint = d == 2 ? int64_t(q - 1) * (q - 2) / 2 : int64_t(q - 1) * (q - 2) * (q - 3) / 6;
  const int64_t base_e = m.nv, base_f = base_e + M.ne * ne1, base_c = base_f + (d == 3 ? M.nf * nf1 : 0);
  out.ndofs = base_c + m.nc * nint;
  DOGIP_CHECK(out.ndofs <= int64_t(TD_MASK), DOGIP_E_RANGE, "too many dofs for the tile encoding");

  // per local node: barycentric index, support (local vertices where it is positive,
  // ascending) with multiplicities, the local edge or opposite face, the interior ordinal
  struct Node {
    int b[4];
    int ns, sup[4], mult[4];
    int edge, opp, iord;
  };
  const int vt = out.nl;
  std::vector<Node> nd(vt);
  int cnt = 0;
  for (int l = 0; l < vt; ++l) {
    Node& n = nd[l];
    int b[4] = {0, 0, 0, 0};
    ref::bary_index(d, q, l, b);
    n.ns = 0;
    n.edge = n.opp = n.iord = -1;
    for (int j = 0; j < 4; ++j) n.b[j] = b[j];
    for (int j = 0; j <= d; ++j)
      if (b[j] > 0) {
        n.sup[n.ns] = j;
        n.mult[n.ns] = b[j];
        ++n.ns;
      }
    if (n.ns == 2) n.edge = local_edge_of(ledges, n.sup[0], n.sup[1]);
    if (n.ns == 3 && d == 3)
      for (int j = 0; j < 4; ++j)
        if (b[j] == 0) n.opp = j;
    if (n.ns == d1) n.iord = cnt++;
  }
  // 2D: the local edge opposite local vertex j
  int opp_edge[3] = {-1, -1, -1};
  if (d == 2)
    for (int j = 0; j < 3; ++j) opp_edge[j] = local_edge_of(ledges, (j + 1) % 3, (j + 2) % 3);

  out.cell_dofs.assign(size_t(m.nc) * vt, -1);
  // the dof of every cell node (cells in parallel; a pure function of the cell)
  parallel_for(m.nc, [&](int64_t c) {
    const int32_t* cv = &m.cells[c * d1];
    for (int l = 0; l < vt; ++l) {
      const Node& n = nd[l];
      int64_t dof;
      if (n.ns == 1) {
        dof = cv[n.sup[0]];
      } else if (n.ns == 2) {
        const int a = n.sup[0], b = n.sup[1];
        const int64_t eid = M.cell_edge[c * nle + n.edge];
        const int mb = cv[a] < cv[b] ? n.mult[1] : n.mult[0];  // multiplicity at the larger vertex id
        dof = base_e + eid * ne1 + (mb - 1);
      } else if (n.ns == 3 && d == 3) {
        const int64_t fid = M.cell_face[c * 4 + n.opp];
        // order the three (vertex, multiplicity) pairs by vertex id
        std::array<std::pair<int32_t, int>, 3> vm = {std::make_pair(cv[n.sup[0]], n.mult[0]),
                                                     std::make_pair(cv[n.sup[1]], n.mult[1]),
                                                     std::make_pair(cv[n.sup[2]], n.mult[2])};
        std::sort(vm.begin(), vm.end());
        dof = base_f + fid * nf1 + tri_index(vm[1].second - 1, vm[2].second - 1, q - 3);
      } else {
        dof = base_c + c * nint + n.iord;
      }
      out.cell_dofs[c * vt + l] = int32_t(dof);
    }
  });
  if (!xyz) return out;
  out.xyz.assign(size_t(out.ndofs) * d, 0.0);
  out.is_bnd.assign(out.ndofs, 0);
  // boundary flags: nodes on a facet held by one cell only
  for (int64_t c = 0; c < m.nc; ++c)
    for (int j = 0; j <= d; ++j) {
      const bool fb = d == 2 ? M.edge_cells[M.cell_edge[c * nle + opp_edge[j]]] == 1
                             : M.face_cells[M.cell_face[c * 4 + j]] == 1;
      if (!fb) continue;
      for (int l = 0; l < vt; ++l)
        if (nd[l].b[j] == 0) out.is_bnd[out.cell_dofs[c * vt + l]] = 1;
    }
  // coordinates, once per dof from its first cell node (an atomic minimum over the cells
  // in parallel), summed in ascending vertex-id order so they do not depend on the cell
  std::vector<std::atomic<int64_t>> first(size_t(out.ndofs));
  for (auto& f : first) f.store(INT64_MAX, std::memory_order_relaxed);
  parallel_for(m.nc, [&](int64_t c) {
    for (int l = 0; l < vt; ++l) {
      const int64_t v = c * vt + l;
      std::atomic<int64_t>& f = first[size_t(out.cell_dofs[v])];
      int64_t cur = f.load(std::memory_order_relaxed);
      while (v < cur && !f.compare_exchange_weak(cur, v, std::memory_order_relaxed)) {
      }
    }
  });
  parallel_for(out.ndofs, [&](int64_t dof) {
    const int64_t v = first[size_t(dof)].load(std::memory_order_relaxed);
    const int64_t c = v / vt;
    const Node& n = nd[size_t(v % vt)];
    const int32_t* cv = &m.cells[c * d1];
    std::array<std::pair<int32_t, int>, 4> vw;
    for (int t = 0; t < n.ns; ++t) vw[t] = {cv[n.sup[t]], n.mult[t]};
    std::sort(vw.begin(), vw.begin() + n.ns);
    for (int x = 0; x < d; ++x) {
      double acc = 0.0;
      for (int t = 0; t < n.ns; ++t) acc += (double(vw[t].second) / q) * m.xyz[int64_t(vw[t].first) * d + x];
      out.xyz[dof * d + x] = acc;
    }
  });
  return out;
}

std::shared_ptr<Space> make_space(std::shared_ptr<const Mesh> mesh, int k, int kind, int bc) {
  const Mesh& m = *mesh;
  const int d = m.dim;
  DOGIP_CHECK(kind == DOGIP_WP || kind == DOGIP_SE, DOGIP_E_RANGE, "kind must be DOGIP_WP or DOGIP_SE");
  DOGIP_CHECK(bc == DOGIP_BC_NONE || bc == DOGIP_BC_DIRICHLET0, DOGIP_E_RANGE, "unknown boundary condition");
  DOGIP_CHECK(k >= 1 && k <= (d == 2 ? 8 : 4), DOGIP_E_RANGE, "k must be in 1..8 (2D) or 1..4 (3D)");
  auto s = std::make_shared<Space>();
  s->mesh = mesh;
  s->dim = d;
  s->k = k;
  s->kind = kind;
  s->bc = bc;
  s->nc = m.nc;
  s->vt = dim_p(d, k);
  s->wt = dim_p(d, w_order(k, kind));
  s->nsym = kind == KIND_SE ? n_sym(d) : 1;
  s->nb = kind == KIND_SE ? d : 1;
  reference_tables(d, k, kind, s->bhat, s->what, s->nnz_bhat, s->nnz_pm1);
  {
    LatticeDofs L = number_lattice(m, k, true);
    s->ndofs = L.ndofs;
    s->cell_dofs.swap(L.cell_dofs);
    s->dof_xyz.swap(L.xyz);
    s->is_bnd.swap(L.is_bnd);
  }
  // final numbering: dofs in the Morton order of their coordinates, so that the dofs
  // of a compact group of cells occupy a compact index range
  {
    const std::vector<int64_t> order = morton_order(s->dof_xyz.data(), s->ndofs, d);
    std::vector<int32_t> inv(s->ndofs);
    parallel_for(s->ndofs, [&](int64_t i) { inv[order[i]] = int32_t(i); });
    parallel_for(int64_t(s->cell_dofs.size()), [&](int64_t i) { s->cell_dofs[size_t(i)] = inv[s->cell_dofs[size_t(i)]]; });
    std::vector<double> xyz(s->dof_xyz.size());
    std::vector<uint8_t> bnd(s->ndofs);
    parallel_for(s->ndofs, [&](int64_t i) {
      for (int x = 0; x < d; ++x) xyz[i * d + x] = s->dof_xyz[order[i] * d + x];
      bnd[i] = s->is_bnd[order[i]];
    });
    s->dof_xyz.swap(xyz);
    s->is_bnd.swap(bnd);
  }
  if (bc == DOGIP_BC_DIRICHLET0) {
    for (int64_t i = 0; i < s->ndofs; ++i)
      if (s->is_bnd[i]) s->boundary.push_back(int32_t(i));
  } else {
    std::fill(s->is_bnd.begin(), s->is_bnd.end(), 0);
  }
  return s;
}

// ---------------------------------------------------------------- tiling

std::shared_ptr<const std::vector<int32_t>> mesh_cell_order(const Mesh& m) {
  std::lock_guard<std::mutex> lock(m.ent_mu);
  if (m.cell_order) return m.cell_order;
  const int d = m.dim, d1 = d + 1;
  std::vector<double> cen(size_t(m.nc) * d, 0.0);
  for (int64_t c = 0; c < m.nc; ++c)
    for (int x = 0; x < d; ++x) {
      double cx = 0;
      for (int j = 0; j < d1; ++j) cx += m.xyz[int64_t(m.cells[c * d1 + j]) * d + x];
      cen[c * d + x] = cx / d1;
    }
  const std::vector<int64_t> order = morton_order(cen.data(), m.nc, d);
  auto out = std::make_shared<std::vector<int32_t>>(size_t(m.nc));
  for (int64_t c = 0; c < m.nc; ++c) (*out)[size_t(c)] = int32_t(order[c]);
  m.cell_order = out;
  return out;
}

TilePlan make_tiles(const Space& s, int te) {
  const Mesh& m = *s.mesh;
  const int vt = s.vt;
  TilePlan p;
  p.te = te;
  p.ntiles = (s.nc + te - 1) / te;
  p.nel_pad = p.ntiles * te;
  // Morton order of cell centroids (shared by every operator on the mesh)
  p.perm = *mesh_cell_order(m);

  p.nlc = (vt + 7) / 8;
  p.lidx.assign(size_t(p.nel_pad / 64) * p.nlc * 64 * 8, 0);
  p.tile_off.assign(p.ntiles + 1, 0);
  // pass 1 (tiles in parallel): distinct dofs of every tile, ascending
  std::vector<std::vector<int32_t>> lists(size_t(p.ntiles));
  parallel_for(p.ntiles, [&](int64_t t) {
    const int64_t e0 = t * te, e1 = std::min<int64_t>(s.nc, e0 + te);
    std::vector<int32_t>& l = lists[size_t(t)];
    l.reserve(size_t(e1 - e0) * vt);
    for (int64_t e = e0; e < e1; ++e) {
      const int32_t* cd = &s.cell_dofs[int64_t(p.perm[e]) * vt];
      l.insert(l.end(), cd, cd + vt);
    }
    std::sort(l.begin(), l.end());
    l.erase(std::unique(l.begin(), l.end()), l.end());
  });
  // how many tiles touch each dof, and the first of them (tile order)
  std::vector<int32_t> ntile_of(s.ndofs, 0), first_tile(s.ndofs, -1);
  for (int64_t t = 0; t < p.ntiles; ++t) {
    const auto& l = lists[size_t(t)];
    DOGIP_CHECK(l.size() <= 65535, DOGIP_E_RANGE, "tile touches too many dofs");
    for (int32_t dof : l) {
      ntile_of[dof]++;
      if (first_tile[dof] < 0) first_tile[dof] = int32_t(t);
    }
    p.tile_off[t + 1] = p.tile_off[t] + int64_t(l.size());
    p.max_tile_dofs = std::max<int64_t>(p.max_tile_dofs, int64_t(l.size()));
  }
  // shared (non-Dirichlet) dofs, numbered in ascending dof order
  std::vector<int32_t> sh_index(s.ndofs, -1);
  for (int64_t i = 0; i < s.ndofs; ++i)
    if (ntile_of[i] > 1 && !s.is_bnd[i]) {
      sh_index[i] = int32_t(p.shared.size());
      p.shared.push_back(int32_t(i));
    }
  // pass 2 (tiles in parallel): order each tile's list as [shared | exclusive | Dirichlet]
  // (ascending dof within each group); the shared group's partial sums go to
  // stage[stage_off[t] + j].  Local indices of the cells' nodes by binary search in the
  // ascending list.
  p.tile_dofs.resize(size_t(p.tile_off[p.ntiles]));
  std::vector<int64_t> nsh(size_t(p.ntiles), 0);
  parallel_for(p.ntiles, [&](int64_t t) {
    const auto& l = lists[size_t(t)];
    const int64_t o0 = p.tile_off[t];
    std::vector<uint16_t> at(l.size());
    int64_t w = 0;
    for (int grp = 0; grp < 3; ++grp)
      for (size_t j = 0; j < l.size(); ++j) {
        const int32_t dof = l[j];
        const int g = s.is_bnd[dof] ? 2 : (sh_index[dof] >= 0 ? 0 : 1);
        if (g != grp) continue;
        uint32_t v = uint32_t(dof);
        if (g == 2) v |= TD_BND;
        if (g == 0) v |= TD_SHARED;
        if (first_tile[dof] == t) v |= TD_OWNER;
        at[j] = uint16_t(w);
        p.tile_dofs[size_t(o0 + w++)] = v;
        if (g == 0) nsh[size_t(t)]++;
      }
    const int64_t e0 = t * te, e1 = std::min<int64_t>(s.nc, e0 + te);
    for (int64_t e = e0; e < e1; ++e) {
      const int32_t* cd = &s.cell_dofs[int64_t(p.perm[e]) * vt];
      for (int lo = 0; lo < vt; ++lo) {
        const size_t j = size_t(std::lower_bound(l.begin(), l.end(), cd[lo]) - l.begin());
        const size_t pos = ((size_t(e >> 6) * p.nlc + lo / 8) * 64 + (e & 63)) * 8 + (lo % 8);
        p.lidx[pos] = at[j];
      }
    }
  });
  p.stage_off.assign(p.ntiles + 1, 0);
  for (int64_t t = 0; t < p.ntiles; ++t) p.stage_off[t + 1] = p.stage_off[t] + nsh[size_t(t)];
  DOGIP_CHECK(p.stage_off[p.ntiles] < (int64_t(1) << 32), DOGIP_E_RANGE, "too many shared entries");
  // reduction lists: for each shared dof, its staging slots in ascending tile order
  std::vector<uint32_t> cnt(p.shared.size() + 1, 0);
  for (int64_t t = 0; t < p.ntiles; ++t)
    for (int64_t j = p.tile_off[t]; j < p.tile_off[t + 1]; ++j) {
      const uint32_t v = p.tile_dofs[size_t(j)];
      if (!(v & TD_SHARED)) break;  // shared entries come first
      cnt[size_t(sh_index[v & TD_MASK]) + 1]++;
    }
  for (size_t i = 1; i < cnt.size(); ++i) cnt[i] += cnt[i - 1];
  p.sh_rowptr = cnt;
  p.sh_slots.assign(p.stage_off[p.ntiles], 0);
  std::vector<uint32_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t t = 0; t < p.ntiles; ++t)
    for (int64_t j = p.tile_off[t]; j < p.tile_off[t + 1]; ++j) {
      const uint32_t v = p.tile_dofs[j];
      if (!(v & TD_SHARED)) break;  // shared entries come first
      const int32_t si = sh_index[v & TD_MASK];
      p.sh_slots[fill[si]++] = uint32_t(p.stage_off[t] + (j - p.tile_off[t]));
    }
  pair_lists(p.sh_rowptr, p.sh_slots, p.sh_pair, p.sh_more_off, p.sh_more);
  return p;
}

void pair_lists(const std::vector<uint32_t>& rowptr, const std::vector<uint32_t>& slots, std::vector<uint32_t>& pair,
                std::vector<uint32_t>& more_off, std::vector<uint32_t>& more) {
  const size_t n = rowptr.empty() ? 0 : rowptr.size() - 1;
  pair.assign(2 * n, 0);
  more_off.assign(n + 1, 0);
  more.clear();
  for (size_t i = 0; i < n; ++i) {
    const uint32_t a = rowptr[i], b = rowptr[i + 1];
    DOGIP_CHECK(b >= a + 2, DOGIP_E_INVALID, "a shared dof with fewer than two partial sums");
    DOGIP_CHECK(slots[a] < (1u << 31) && slots[a + 1] < (1u << 31), DOGIP_E_RANGE, "too many staged partial sums");
    pair[2 * i] = slots[a];
    pair[2 * i + 1] = slots[a + 1] | (b > a + 2 ? (1u << 31) : 0u);
    for (uint32_t j = a + 2; j < b; ++j) more.push_back(slots[j]);
    more_off[i + 1] = uint32_t(more.size());
  }
}

// ---------------------------------------------------------------- global projection form

GlobalPlan make_global_plan(const Space& s, const TilePlan& p) {
  const Mesh& m = *s.mesh;
  const int d = s.dim, q = 2 * s.k;
  DOGIP_CHECK(s.kind == DOGIP_WP, DOGIP_E_RANGE, "the global form is defined for the weighted projection");
  const LatticeDofs W = number_lattice(m, q, false);
  const int wt = W.nl;
  DOGIP_CHECK(wt == s.wt, DOGIP_E_INVALID, "W node count mismatch");
  std::vector<int> ent(wt);
  for (int i = 0; i < wt; ++i) ent[i] = ref::node_entity(d, q, i);
  GlobalPlan g;
  g.nw = W.ndofs;
  // owner: the first cell in tile order holding the W dof
  std::vector<int64_t> owner(g.nw, -1);
  for (int64_t e = 0; e < s.nc; ++e) {
    const int32_t* wd = &W.cell_dofs[int64_t(p.perm[e]) * wt];
    for (int i = 0; i < wt; ++i)
      if (owner[wd[i]] < 0) owner[wd[i]] = e;
  }
  for (int64_t j = 0; j < g.nw; ++j) DOGIP_CHECK(owner[j] >= 0, DOGIP_E_INVALID, "W dof held by no cell");
  // per-cell slot masks (all nodes of an owned slot belong to the cell, no other node does)
  const int nslot = gw_slots(d);
  g.mask.assign(p.nel_pad, 0u);
  for (int64_t e = 0; e < s.nc; ++e) {
    const int32_t* wd = &W.cell_dofs[int64_t(p.perm[e]) * wt];
    uint32_t mask = 0;
    for (int i = 0; i < wt; ++i)
      if (owner[wd[i]] == e) mask |= 1u << ent[i];
    for (int i = 0; i < wt; ++i)
      DOGIP_CHECK(((mask >> ent[i]) & 1u) == (owner[wd[i]] == e ? 1u : 0u), DOGIP_E_INVALID,
                  "W dof ownership does not follow sub-simplices");
    g.mask[e] = mask;
  }
  // nodes of each slot in lattice order
  std::vector<std::vector<int>> slot_nodes(nslot);
  for (int i = 0; i < wt; ++i) slot_nodes[ent[i]].push_back(i);
  // wave layout: slot by slot, node by node, owning lanes in lane order
  const int64_t nwave = p.nel_pad / 64;
  std::vector<int64_t> pos(g.nw, -1);
  g.woff.assign(nwave + 1, 0);
  int64_t count = 0;
  for (int64_t w = 0; w < nwave; ++w) {
    g.woff[w] = count;
    for (int sl = 0; sl < nslot; ++sl)
      for (int i : slot_nodes[sl])
        for (int lane = 0; lane < 64; ++lane) {
          const int64_t e = w * 64 + lane;
          if (e >= s.nc || !((g.mask[e] >> sl) & 1u)) continue;
          pos[W.cell_dofs[int64_t(p.perm[e]) * wt + i]] = count++;
        }
  }
  g.woff[nwave] = count;
  DOGIP_CHECK(count == g.nw, DOGIP_E_INVALID, "W dofs not all owned");
  // incidence lists by position: (internal cell, local node), ascending cell
  g.inc_ptr.assign(g.nw + 1, 0);
  for (int64_t e = 0; e < s.nc; ++e) {
    const int32_t* wd = &W.cell_dofs[int64_t(p.perm[e]) * wt];
    for (int i = 0; i < wt; ++i) g.inc_ptr[pos[wd[i]] + 1]++;
  }
  for (int64_t j = 0; j < g.nw; ++j) g.inc_ptr[j + 1] += g.inc_ptr[j];
  g.inc.assign(g.inc_ptr[g.nw], 0);
  std::vector<int64_t> fill(g.inc_ptr.begin(), g.inc_ptr.end() - 1);
  for (int64_t e = 0; e < s.nc; ++e) {
    const int32_t* wd = &W.cell_dofs[int64_t(p.perm[e]) * wt];
    for (int i = 0; i < wt; ++i) g.inc[fill[pos[wd[i]]]++] = e * wt + i;
  }
  return g;
}

}  // namespace dogip
