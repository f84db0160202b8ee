// C interface of libdogip: opaque handles, status codes, thread-local error text.
#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "batch.hpp"
#include "internal.hpp"
#include "reftab.hpp"

struct dogip_mesh_s {
  std::shared_ptr<dogip::Mesh> m;
};
struct dogip_space_s {
  std::shared_ptr<dogip::Space> s;
};
struct dogip_op_s {
  std::shared_ptr<dogip::Op> op;
};
struct dogip_batch_s {
  std::unique_ptr<dogip::Batch> b;
};

namespace {

thread_local std::string g_err;

template <class F>
int guard(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const dogip::Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return DOGIP_E_NOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return DOGIP_E_INVALID;
  } catch (...) {
    g_err = "unknown failure";
    return DOGIP_E_INVALID;
  }
}

hipStream_t S(dogip_stream s) { return static_cast<hipStream_t>(s); }

template <class H>
void need(H h) {
  DOGIP_CHECK(h != nullptr, DOGIP_E_NULL, "null handle");
}

// Compile-time table of (D, K, KIND) against the exact run-time tables.
template <int D, int K, int KIND>
int64_t table_mismatch() {
  static constexpr dogip::ref::BTable<D, K, KIND> t{};
  std::vector<double> b, w;
  int64_t nnz = 0, pm1 = 0, bad = 0;
  dogip::reference_tables(D, K, KIND, b, w, nnz, pm1);
  for (int r = 0; r < t.NB; ++r)
    for (int i = 0; i < t.WT; ++i)
      for (int l = 0; l < t.VT; ++l)
        if (t.v[r][i][l] != b[(size_t(r) * t.WT + i) * t.VT + l]) ++bad;
  return bad;
}

}  // namespace

extern "C" {

const char* dogip_last_error(void) { return g_err.c_str(); }

int dogip_version(void) { return 2; }

int dogip_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

int dogip_check_tables(int64_t* mismatches) {
  return guard([&] {
    DOGIP_CHECK(mismatches, DOGIP_E_NULL, "null output");
    using namespace dogip;
    int64_t bad = 0;
    bad += table_mismatch<2, 1, KIND_WP>() + table_mismatch<2, 2, KIND_WP>() + table_mismatch<2, 3, KIND_WP>() +
           table_mismatch<2, 4, KIND_WP>() + table_mismatch<2, 5, KIND_WP>();
    bad += table_mismatch<2, 1, KIND_SE>() + table_mismatch<2, 2, KIND_SE>() + table_mismatch<2, 3, KIND_SE>() +
           table_mismatch<2, 4, KIND_SE>() + table_mismatch<2, 5, KIND_SE>();
    bad += table_mismatch<3, 1, KIND_WP>() + table_mismatch<3, 2, KIND_WP>();
    bad += table_mismatch<3, 1, KIND_SE>() + table_mismatch<3, 2, KIND_SE>() + table_mismatch<3, 3, KIND_SE>();
    *mismatches = bad;
    return DOGIP_OK;
  });
}

// ---- mesh ----
int dogip_mesh_create(int dim, int64_t nv, const double* xyz, int64_t nc, const int32_t* cells, dogip_mesh* out) {
  return guard([&] {
    need(out);
    *out = nullptr;
    auto h = new dogip_mesh_s{dogip::make_mesh(dim, nv, xyz, nc, cells)};
    *out = h;
    return DOGIP_OK;
  });
}

int dogip_mesh_unit(int dim, int n, dogip_mesh* out) {
  return guard([&] {
    need(out);
    *out = nullptr;
    *out = new dogip_mesh_s{dogip::make_unit_mesh(dim, n)};
    return DOGIP_OK;
  });
}

int dogip_mesh_info(dogip_mesh m, int* dim, int64_t* nv, int64_t* nc) {
  return guard([&] {
    need(m);
    if (dim) *dim = m->m->dim;
    if (nv) *nv = m->m->nv;
    if (nc) *nc = m->m->nc;
    return DOGIP_OK;
  });
}

int dogip_mesh_copy(dogip_mesh m, double* xyz, int32_t* cells) {
  return guard([&] {
    need(m);
    if (xyz) std::memcpy(xyz, m->m->xyz.data(), m->m->xyz.size() * sizeof(double));
    if (cells) std::memcpy(cells, m->m->cells.data(), m->m->cells.size() * sizeof(int32_t));
    return DOGIP_OK;
  });
}

void dogip_mesh_destroy(dogip_mesh m) { delete m; }

// ---- space ----
int dogip_space_create(dogip_mesh m, int k, int kind, int bc, dogip_space* out) {
  return guard([&] {
    need(m);
    need(out);
    *out = nullptr;
    *out = new dogip_space_s{dogip::make_space(m->m, k, kind, bc)};
    return DOGIP_OK;
  });
}

int dogip_space_get_info(dogip_space s, dogip_space_info* info) {
  return guard([&] {
    need(s);
    need(info);
    const dogip::Space& p = *s->s;
    dogip_space_info i{};
    i.dim = p.dim;
    i.k = p.k;
    i.kind = p.kind;
    i.bc = p.bc;
    i.ncells = p.nc;
    i.ndofs = p.ndofs;
    i.nboundary = int64_t(p.boundary.size());
    i.vt = p.vt;
    i.wt = p.wt;
    i.nsym = p.nsym;
    i.nb = p.nb;
    i.nnz_bhat = p.nnz_bhat;
    i.nnz_pm1_bhat = p.nnz_pm1;
    *info = i;
    return DOGIP_OK;
  });
}

int dogip_space_dof_coords(dogip_space s, double* xyz) {
  return guard([&] {
    need(s);
    DOGIP_CHECK(xyz, DOGIP_E_NULL, "null output");
    std::memcpy(xyz, s->s->dof_xyz.data(), s->s->dof_xyz.size() * sizeof(double));
    return DOGIP_OK;
  });
}

int dogip_space_cell_dofs(dogip_space s, int32_t* cd) {
  return guard([&] {
    need(s);
    DOGIP_CHECK(cd, DOGIP_E_NULL, "null output");
    std::memcpy(cd, s->s->cell_dofs.data(), s->s->cell_dofs.size() * sizeof(int32_t));
    return DOGIP_OK;
  });
}

int dogip_space_boundary(dogip_space s, int32_t* bnd) {
  return guard([&] {
    need(s);
    DOGIP_CHECK(bnd || s->s->boundary.empty(), DOGIP_E_NULL, "null output");
    if (!s->s->boundary.empty()) std::memcpy(bnd, s->s->boundary.data(), s->s->boundary.size() * sizeof(int32_t));
    return DOGIP_OK;
  });
}

int dogip_space_bhat(dogip_space s, double* bhat, double* what) {
  return guard([&] {
    need(s);
    if (bhat) std::memcpy(bhat, s->s->bhat.data(), s->s->bhat.size() * sizeof(double));
    if (what) std::memcpy(what, s->s->what.data(), s->s->what.size() * sizeof(double));
    return DOGIP_OK;
  });
}

int dogip_space_bhat_factors(dogip_space s, double* b1, double* b2) {
  return guard([&] {
    need(s);
    const auto& sp = *s->s;
    DOGIP_CHECK(dogip::has_factored(sp.dim, sp.k, sp.kind), DOGIP_E_RANGE, "no factored B^ for this space");
    dogip::factored_tables(sp.dim, sp.k, b1, b2);
    return DOGIP_OK;
  });
}

void dogip_space_destroy(dogip_space s) { delete s; }

// ---- operator ----
int dogip_op_create(dogip_space s, int coef_kind, const double* coef, unsigned flags, int tile_waves, int variant,
                    dogip_stream stream, dogip_op* out) {
  return guard([&] {
    need(s);
    need(out);
    *out = nullptr;
    auto op = dogip::make_op(s->s, coef_kind, coef, flags, tile_waves, variant, S(stream));
    *out = new dogip_op_s{std::shared_ptr<dogip::Op>(std::move(op))};
    return DOGIP_OK;
  });
}

int dogip_quadrature(int dim, int n, double* pts, double* wts) {
  return guard([&] {
    need(pts);
    need(wts);
    std::vector<double> p, w;
    dogip::collapsed_rule(dim, n, p, w);
    std::copy(p.begin(), p.end(), pts);
    std::copy(w.begin(), w.end(), wts);
    return DOGIP_OK;
  });
}

int dogip_op_create_qp(dogip_space s, int n, const double* coef, unsigned flags, int tile_waves, dogip_stream stream,
                       dogip_op* out) {
  return guard([&] {
    need(s);
    need(out);
    *out = nullptr;
    auto op = dogip::make_op_qp(s->s, n, coef, flags, tile_waves, S(stream));
    *out = new dogip_op_s{std::shared_ptr<dogip::Op>(std::move(op))};
    return DOGIP_OK;
  });
}

int dogip_op_set_inclusions(dogip_op op, int nballs, const double* balls, double a_in, double a_out, int depth, int ng,
                            double* mean_points, dogip_stream stream) {
  return guard([&] {
    need(op);
    dogip::op_set_inclusions(*op->op, nballs, balls, a_in, a_out, depth, ng, mean_points, S(stream));
    return DOGIP_OK;
  });
}

int dogip_op_set_coef(dogip_op op, int coef_kind, const double* coef, dogip_stream stream) {
  return guard([&] {
    need(op);
    dogip::op_set_coef(*op->op, coef_kind, coef, S(stream));
    return DOGIP_OK;
  });
}

int dogip_op_set_tile_lanes(dogip_op op, int lanes64, int lanes32) {
  return guard([&] {
    need(op);
    dogip::op_set_tile_lanes(*op->op, lanes64, lanes32);
    return DOGIP_OK;
  });
}

int dogip_op_get_info(dogip_op op, dogip_op_info* info) {
  return guard([&] {
    need(op);
    need(info);
    *info = dogip::op_info(*op->op);
    return DOGIP_OK;
  });
}

int dogip_op_export_d(dogip_op op, double* d_out, dogip_stream stream) {
  return guard([&] {
    need(op);
    dogip::op_export_d(*op->op, d_out, S(stream));
    return DOGIP_OK;
  });
}

int dogip_apply(dogip_op op, const double* u, double* y, int prec, dogip_stream stream) {
  return guard([&] {
    need(op);
    dogip::op_apply(*op->op, u, y, prec, S(stream));
    return DOGIP_OK;
  });
}

int dogip_apply_noalloc(dogip_op op, const double* u, double* y, int prec, dogip_stream stream) {
  return guard([&] {
    need(op);
    dogip::op_apply_noalloc(*op->op, u, y, prec, S(stream));
    return DOGIP_OK;
  });
}

int dogip_diag(dogip_op op, double* diag, dogip_stream stream) {
  return guard([&] {
    need(op);
    dogip::op_diag(*op->op, diag, S(stream));
    return DOGIP_OK;
  });
}

int dogip_pcg(dogip_op op, const double* b, double* x, const dogip_solve_opts* opts, dogip_solve_stats* stats,
              dogip_stream stream) {
  dogip_solve_stats local{};
  dogip_solve_stats* st = stats ? stats : &local;
  const int rc = guard([&] {
    need(op);
    DOGIP_CHECK(opts, DOGIP_E_NULL, "null options");
    const int status = dogip::op_pcg(*op->op, b, x, *opts, *st, S(stream));
    if (status == DOGIP_E_NOT_CONVERGED) g_err = "CG did not reach the tolerance within maxit";
    if (status == DOGIP_E_BREAKDOWN) g_err = "CG breakdown: p^T A p <= 0";
    if (status == DOGIP_E_NONFINITE) g_err = "non-finite value in CG";
    return status;
  });
  st->status = rc;
  return rc;
}

int dogip_grad_logcoef(dogip_op op, const double* u, const double* lam, double* g, dogip_stream stream) {
  return guard([&] {
    need(op);
    dogip::op_grad(*op->op, u, lam, g, S(stream));
    return DOGIP_OK;
  });
}

int dogip_op_timer_enable(dogip_op op, int enable) {
  return guard([&] {
    need(op);
    dogip::op_timer_enable(*op->op, enable != 0);
    return DOGIP_OK;
  });
}

int dogip_op_timer_read(dogip_op op, double* tile_ms_sum, double* finish_ms_sum, int64_t* count) {
  return guard([&] {
    need(op);
    dogip::op_timer_read(*op->op, tile_ms_sum, finish_ms_sum, count);
    return DOGIP_OK;
  });
}

void dogip_op_destroy(dogip_op op) { delete op; }

// ---- batch ----
int dogip_batch_create(const dogip_op* ops, int nops, dogip_stream stream, dogip_batch* out) {
  return guard([&] {
    need(out);
    *out = nullptr;
    DOGIP_CHECK(ops && nops > 0, DOGIP_E_NULL, "empty operator list");
    std::vector<std::shared_ptr<dogip::Op>> v;
    for (int i = 0; i < nops; ++i) {
      need(ops[i]);
      v.push_back(ops[i]->op);
    }
    *out = new dogip_batch_s{dogip::make_batch(v, S(stream))};
    return DOGIP_OK;
  });
}

int dogip_batch_offsets(dogip_batch b, int64_t* offsets) {
  return guard([&] {
    need(b);
    DOGIP_CHECK(offsets, DOGIP_E_NULL, "null output");
    std::memcpy(offsets, b->b->offsets.data(), b->b->offsets.size() * sizeof(int64_t));
    return DOGIP_OK;
  });
}

int dogip_batch_apply(dogip_batch b, const double* u, double* y, int prec, dogip_stream stream) {
  return guard([&] {
    need(b);
    dogip::batch_apply(*b->b, u, y, prec, S(stream));
    return DOGIP_OK;
  });
}

int dogip_batch_pcg(dogip_batch b, const double* rhs, double* x, const dogip_solve_opts* opts,
                    dogip_solve_stats* stats, dogip_stream stream) {
  return guard([&] {
    need(b);
    DOGIP_CHECK(opts, DOGIP_E_NULL, "null options");
    const int status = dogip::batch_pcg(*b->b, rhs, x, *opts, stats, S(stream));
    if (status != DOGIP_OK) g_err = "at least one problem of the batch did not converge (see its stats)";
    return status;
  });
}

void dogip_batch_destroy(dogip_batch b) { delete b; }

}  // extern "C"
