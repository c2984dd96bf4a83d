// api.hip -- the C ABI of libfem (declared in include/fem.h): argument
// validation, plan ownership and dispatch to the kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "chunk.h"
#include "fem.h"
#include "kernels.h"
#include "plan.h"
#include "solver.h"

struct fem_plan {
    fem::DevPlan dev{};
    fem_plan_stats stats{};
    void *arena = nullptr;
    double *scratch64 = nullptr;
    float *scratch32 = nullptr;
    int64_t n_isolated_free = 0;
    fem::SolverWork work[3];  // [0] FP64 solver, [1] mixed precision, [2] matrix-free
};

fem::DevPlan fem::plan_device(const fem_plan *p) { return p->dev; }

namespace {

using fem::set_error;

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct ArenaLayout {
    size_t total = 0;
    size_t add(size_t bytes) {
        size_t off = total;
        total = align_up(total + std::max<size_t>(bytes, 1));
        return off;
    }
};

bool valid_dtype(int t) { return t == FEM_F64 || t == FEM_F32 || t == FEM_F32X2; }


int check_plan(const fem_plan *p) {
    if (!p) return set_error(FEM_EINVAL, "plan is NULL");
    return FEM_OK;
}

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

int alloc_work(fem_plan *plan, int slot, int dtype) {
    fem::SolverWork &w = plan->work[slot];
    if (w.arena) return FEM_OK;
    const fem::DevPlan &P = plan->dev;
    const int64_t n = P.n_nodes;
    const int64_t npk = (int64_t)fem::packed_count(P.nb) * P.n_elems;
    // the largest chunk grid (8 workgroups per CU) plus the fix-up grid
    const int64_t npart = 8 * (int64_t)fem::device_cu_count() + fem::fixup_grid(P.n_shared, fem::kFixDotsCap) + 8;
    ArenaLayout L;
    // FP64 packed operator, or FP32 hi/lo pair of it: the same bytes; the
    // matrix-free solver keeps the coordinates in the solver-local order there
    size_t oA = L.add(dtype == FEM_MFREE ? (size_t)P.dim * n * sizeof(double) : (size_t)npk * sizeof(double));
    size_t od = L.add(n * sizeof(double));
    size_t odi = L.add(n * sizeof(double));
    size_t or_ = L.add(n * sizeof(double));
    size_t op_ = L.add(n * sizeof(double));
    size_t oq = L.add(n * sizeof(double));
    size_t oxc = L.add(n * sizeof(float));
    size_t or64 = L.add(n * sizeof(double));
    size_t opart64 = L.add(std::max<int64_t>(P.n_partials, 1) * sizeof(double));
    size_t opartv = L.add(std::max<int64_t>(P.n_partials, 1) * sizeof(double));
    size_t odots = L.add((size_t)8 * npart * sizeof(double));
    size_t oxl = L.add(n * sizeof(double));
    size_t operm = L.add(n * sizeof(int32_t));
    size_t oupd = L.add((size_t)3 * 1024 * sizeof(double));
    size_t ost = L.add(sizeof(fem::IterState));
    size_t obad = L.add(sizeof(int));
    void *arena = nullptr;
    if (hipMalloc(&arena, L.total) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FEM_ENOMEM, "device allocation of the solver workspace failed");
    }
    char *b = static_cast<char *>(arena);
    w.arena = arena;
    w.bytes = L.total;
    w.kind = dtype;
    w.Apk = b + oA;
    w.d64 = reinterpret_cast<double *>(b + od);
    w.dinv = b + odi;
    w.r = b + or_;
    w.p = b + op_;
    w.q = b + oq;
    w.xc = b + oxc;
    w.r64 = reinterpret_cast<double *>(b + or64);
    w.part64 = reinterpret_cast<double *>(b + opart64);
    w.partv = b + opartv;
    w.dots = reinterpret_cast<double *>(b + odots);
    w.xl = b + oxl;
    w.perm = reinterpret_cast<int32_t *>(b + operm);
    w.upd = reinterpret_cast<double *>(b + oupd);
    w.st = reinterpret_cast<fem::IterState *>(b + ost);
    w.bad = reinterpret_cast<int *>(b + obad);
    return FEM_OK;
}

}  // namespace

extern "C" {

const char *fem_last_error(void) { return fem::last_error().c_str(); }

void fem_solve_opts_default(fem_solve_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->dtype = FEM_F64;
    o->nu = 0.0;
    o->rtol = 1e-8;
    o->max_iter = 100000;
    o->precond = FEM_PRECOND_JACOBI;
    o->inner_rtol = 0.1;
    o->max_outer = 200;
    o->check_every = 32;
    o->profile = 0;
    o->vectors = 0;
    o->block = 0;
}

namespace {

int plan_create(int dim, int nb, int64_t n_nodes, int64_t n_elems, const double *d_coords, const int32_t *d_conn,
                const int32_t *d_dirichlet, int64_t n_dirichlet, int chunk_elems, void *stream, fem_plan **out) {
    fem::last_error().clear();
    if (!out) return set_error(FEM_EINVAL, "out is NULL");
    *out = nullptr;
    if (dim != 2 && dim != 3) return set_error(FEM_EINVAL, "dim must be 2 or 3");
    if (n_nodes < 1 || n_nodes > INT32_MAX) return set_error(FEM_EINVAL, "n_nodes must be in [1, 2^31)");
    if (n_elems < 0 || n_elems > INT32_MAX) return set_error(FEM_EINVAL, "n_elems must be in [0, 2^31)");
    if (!d_coords) return set_error(FEM_EINVAL, "coords is NULL");
    if (n_elems > 0 && !d_conn) return set_error(FEM_EINVAL, "conn is NULL");
    if (n_dirichlet < 0 || (n_dirichlet > 0 && !d_dirichlet)) return set_error(FEM_EINVAL, "bad Dirichlet list");
    if (chunk_elems == 0) chunk_elems = fem::default_chunk_elems(nb);
    if (!fem::valid_chunk_elems(nb, chunk_elems))
        return set_error(FEM_EINVAL, nb == 3    ? "chunk_elems must be one of 64, 128, 256, 512, 1024, 1536, 2048"
                                     : nb == 4  ? "chunk_elems must be one of 64, 128, 256, 512, 1024, 1536"
                                     : nb == 6  ? "chunk_elems must be one of 64, 128, 256, 512, 1024"
                                                : "chunk_elems must be one of 64, 128, 256, 512");
    hipStream_t s = S(stream);
    std::vector<double> coords((size_t)dim * n_nodes);
    std::vector<int32_t> conn((size_t)nb * n_elems);
    std::vector<int32_t> dir((size_t)n_dirichlet);
    FEM_HIP_CHECK(hipMemcpyAsync(coords.data(), d_coords, coords.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    if (n_elems)
        FEM_HIP_CHECK(hipMemcpyAsync(conn.data(), d_conn, conn.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (n_dirichlet)
        FEM_HIP_CHECK(
            hipMemcpyAsync(dir.data(), d_dirichlet, dir.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    for (double c : coords)
        if (!std::isfinite(c)) return set_error(FEM_EINVAL, "non-finite coordinate");
    fem::HostPlan H;
    std::string err;
    try {
        if (fem::build_host_plan(dim, nb, n_nodes, n_elems, coords.data(), conn.data(), dir.data(), n_dirichlet,
                                 chunk_elems, H, err) != 0)
            return set_error(FEM_EINVAL, err);
    } catch (const std::bad_alloc &) {
        return set_error(FEM_ENOMEM, "host allocation failed while building the plan");
    }
    ArenaLayout L;
    const size_t o_coords = L.add(coords.size() * sizeof(double));
    const size_t o_conn = L.add(conn.size() * sizeof(int32_t));
    const size_t o_cno = L.add(H.chunk_node_off.size() * sizeof(int32_t));
    const size_t o_cin = L.add(H.chunk_info.size() * sizeof(int32_t));
    const size_t o_ln = L.add(H.loc_nodes.size() * sizeof(int32_t));
    const size_t o_le = L.add(H.loc_end.size() * sizeof(uint16_t));
    const size_t o_sl = L.add(H.slots.size() * sizeof(uint16_t));
    const size_t o_fn = L.add(H.fix_nodes.size() * sizeof(int32_t));
    const size_t o_fo = L.add(H.fix_off.size() * sizeof(int32_t));
    const size_t o_fp = L.add(H.fix_parts.size() * sizeof(int32_t));
    const size_t o_po = L.add(H.part_owner.size() * sizeof(int32_t));
    const size_t o_fr = L.add(H.fix_rec.size() * sizeof(int32_t));
    const size_t o_co = L.add(H.comp_off.size() * sizeof(int32_t));
    const size_t o_mask = L.add(H.mask.size());
    const size_t o_s64 = L.add(std::max<int64_t>(H.n_partials, 1) * sizeof(double));
    const size_t o_s32 = L.add(std::max<int64_t>(H.n_partials, 1) * sizeof(float));
    fem_plan *plan = new (std::nothrow) fem_plan();
    if (!plan) return set_error(FEM_ENOMEM, "host allocation failed");
    if (hipMalloc(&plan->arena, L.total) != hipSuccess) {
        (void)hipGetLastError();
        delete plan;
        return set_error(FEM_ENOMEM, "device allocation of the plan failed");
    }
    char *b = static_cast<char *>(plan->arena);
    auto up = [&](size_t off, const void *src, size_t bytes) -> int {
        if (bytes == 0) return 0;
        return hipMemcpyAsync(b + off, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess ? 0 : -1;
    };
    int bad = 0;
    bad |= up(o_coords, coords.data(), coords.size() * sizeof(double));
    bad |= up(o_conn, conn.data(), conn.size() * sizeof(int32_t));
    bad |= up(o_cno, H.chunk_node_off.data(), H.chunk_node_off.size() * sizeof(int32_t));
    bad |= up(o_cin, H.chunk_info.data(), H.chunk_info.size() * sizeof(int32_t));
    bad |= up(o_ln, H.loc_nodes.data(), H.loc_nodes.size() * sizeof(int32_t));
    bad |= up(o_le, H.loc_end.data(), H.loc_end.size() * sizeof(uint16_t));
    bad |= up(o_sl, H.slots.data(), H.slots.size() * sizeof(uint16_t));
    bad |= up(o_fn, H.fix_nodes.data(), H.fix_nodes.size() * sizeof(int32_t));
    bad |= up(o_fo, H.fix_off.data(), H.fix_off.size() * sizeof(int32_t));
    bad |= up(o_fp, H.fix_parts.data(), H.fix_parts.size() * sizeof(int32_t));
    bad |= up(o_po, H.part_owner.data(), H.part_owner.size() * sizeof(int32_t));
    bad |= up(o_fr, H.fix_rec.data(), H.fix_rec.size() * sizeof(int32_t));
    bad |= up(o_co, H.comp_off.data(), H.comp_off.size() * sizeof(int32_t));
    bad |= up(o_mask, H.mask.data(), H.mask.size());
    if (bad || hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(plan->arena);
        delete plan;
        return set_error(FEM_EHIP, "upload of the plan failed");
    }
    fem::DevPlan &D = plan->dev;
    D.dim = dim;
    D.nb = nb;
    D.E = chunk_elems;
    D.n_nodes = n_nodes;
    D.n_elems = n_elems;
    D.n_chunks = H.n_chunks;
    D.n_local = H.n_local;
    D.n_shared = H.n_shared;
    D.n_partials = H.n_partials;
    D.max_local = 0;
    for (size_t c = 0; c + 1 < H.chunk_node_off.size(); ++c)
        D.max_local = std::max(D.max_local, H.chunk_node_off[c + 1] - H.chunk_node_off[c]);
    D.coords = reinterpret_cast<const double *>(b + o_coords);
    D.conn = reinterpret_cast<const int32_t *>(b + o_conn);
    D.chunk_node_off = reinterpret_cast<const int32_t *>(b + o_cno);
    D.chunk_info = reinterpret_cast<const int32_t *>(b + o_cin);
    D.loc_nodes = reinterpret_cast<const int32_t *>(b + o_ln);
    D.loc_end = reinterpret_cast<const uint16_t *>(b + o_le);
    D.slots = reinterpret_cast<const uint16_t *>(b + o_sl);
    D.fix_nodes = reinterpret_cast<const int32_t *>(b + o_fn);
    D.fix_off = reinterpret_cast<const int32_t *>(b + o_fo);
    D.fix_parts = reinterpret_cast<const int32_t *>(b + o_fp);
    D.part_owner = reinterpret_cast<const int32_t *>(b + o_po);
    D.fix_rec = H.fix_rec.empty() ? nullptr : reinterpret_cast<const int32_t *>(b + o_fr);
    D.comp_off = reinterpret_cast<const int32_t *>(b + o_co);
    D.mask = reinterpret_cast<const uint8_t *>(b + o_mask);
    plan->scratch64 = reinterpret_cast<double *>(b + o_s64);
    plan->scratch32 = reinterpret_cast<float *>(b + o_s32);
    plan->n_isolated_free = H.n_isolated_free;
    fem_plan_stats &st = plan->stats;
    st.dim = dim;
    st.n_b = nb;
    st.n_nodes = n_nodes;
    st.n_elems = n_elems;
    st.n_dirichlet = H.n_dirichlet;
    st.chunk_elems = chunk_elems;
    st.n_chunks = H.n_chunks;
    st.n_local = H.n_local;
    st.n_shared = H.n_shared;
    st.n_partials = H.n_partials;
    st.index_bytes = (int64_t)(o_s64 - o_cno);
    *out = plan;
    return FEM_OK;
}

}  // namespace

int fem_plan_create(int dim, int64_t n_nodes, int64_t n_elems, const double *d_coords, const int32_t *d_conn,
                    const int32_t *d_dirichlet, int64_t n_dirichlet, int chunk_elems, void *stream,
                    fem_plan **out) {
    return plan_create(dim, dim + 1, n_nodes, n_elems, d_coords, d_conn, d_dirichlet, n_dirichlet, chunk_elems,
                       stream, out);
}

int fem_plan_create_p2(int dim, int64_t n_nodes, int64_t n_elems, const double *d_coords, const int32_t *d_conn,
                       const int32_t *d_dirichlet, int64_t n_dirichlet, int chunk_elems, void *stream,
                       fem_plan **out) {
    if (dim != 2 && dim != 3) {
        fem::last_error().clear();
        if (out) *out = nullptr;
        return set_error(FEM_EINVAL, "dim must be 2 or 3");
    }
    return plan_create(dim, dim == 2 ? 6 : 10, n_nodes, n_elems, d_coords, d_conn, d_dirichlet, n_dirichlet,
                       chunk_elems, stream, out);
}

int fem_plan_destroy(fem_plan *plan) {
    if (!plan) return FEM_OK;
    int rc = FEM_OK;
    for (auto &w : plan->work) {
        if (w.graph && hipGraphExecDestroy(w.graph) != hipSuccess) rc = FEM_EHIP;
        if (w.cap && hipStreamDestroy(w.cap) != hipSuccess) rc = FEM_EHIP;
        if (w.arena && hipFree(w.arena) != hipSuccess) rc = FEM_EHIP;
    }
    if (plan->arena && hipFree(plan->arena) != hipSuccess) rc = FEM_EHIP;
    delete plan;
    if (rc) set_error(rc, "hipFree failed");
    return rc;
}

int fem_plan_get_stats(const fem_plan *plan, fem_plan_stats *out) {
    if (int rc = check_plan(plan)) return rc;
    if (!out) return set_error(FEM_EINVAL, "out is NULL");
    *out = plan->stats;
    return FEM_OK;
}

int fem_build_local_matrices(const fem_plan *plan, int dtype, void *d_K_e, void *d_M_e, double *d_vol,
                             void *stream) {
    if (int rc = check_plan(plan)) return rc;
    if (!valid_dtype(dtype)) return set_error(FEM_EINVAL, "unknown dtype");
    if (plan->dev.n_elems == 0 || (!d_K_e && !d_M_e && !d_vol)) return FEM_OK;
    return fem::launch_local_matrices(plan->dev, dtype, d_K_e, d_M_e, d_vol, S(stream));
}

int fem_combine_local(const fem_plan *plan, int dtype_in, const void *d_K_e, const void *d_M_e, double nu,
                      int dtype_out, void *d_A_e, void *stream) {
    if (int rc = check_plan(plan)) return rc;
    if (!valid_dtype(dtype_in) || !valid_dtype(dtype_out)) return set_error(FEM_EINVAL, "unknown dtype");
    if (!d_K_e || !d_A_e) return set_error(FEM_EINVAL, "K_e and A_e must not be NULL");
    if (!std::isfinite(nu) || nu < 0.0) return set_error(FEM_EINVAL, "nu must be finite and >= 0");
    if (d_A_e == d_K_e || d_A_e == d_M_e) return set_error(FEM_EINVAL, "A_e must not alias K_e or M_e");
    if (plan->dev.n_elems == 0) return FEM_OK;
    return fem::launch_combine(plan->dev, dtype_in, d_K_e, nu != 0.0 ? d_M_e : nullptr, nu, dtype_out, d_A_e,
                               S(stream));
}

int fem_element_residual(const fem_plan *plan, int dtype, const void *d_K_e, const void *d_M_e, double nu,
                         const double *d_b, const double *d_x, double *d_r, int mask_dirichlet, void *stream) {
    if (int rc = check_plan(plan)) return rc;
    if (dtype == FEM_MFREE) {
        if (!d_x || !d_r) return set_error(FEM_EINVAL, "NULL argument");
        if (!std::isfinite(nu) || nu < 0.0) return set_error(FEM_EINVAL, "nu must be finite and >= 0");
        if (d_r == d_x || (d_b && d_r == d_b)) return set_error(FEM_EINVAL, "r must not alias x or b");
        return fem::launch_apply_mf(plan->dev, 1.0, nu, d_x, d_b, d_r, -1.0, mask_dirichlet ? 1 : 0, plan->scratch64,
                                    S(stream));
    }
    if (!valid_dtype(dtype)) return set_error(FEM_EINVAL, "unknown dtype");
    if ((!d_K_e && plan->dev.n_elems > 0) || !d_x || !d_r) return set_error(FEM_EINVAL, "NULL argument");
    if (d_M_e && (!std::isfinite(nu) || nu < 0.0)) return set_error(FEM_EINVAL, "nu must be finite and >= 0");
    if ((const void *)d_r == (const void *)d_x || (d_b && (const void *)d_r == (const void *)d_b))
        return set_error(FEM_EINVAL, "r must not alias x or b");
    return fem::launch_apply64(plan->dev, dtype, d_K_e, (d_M_e && nu != 0.0) ? d_M_e : nullptr, nu, d_x, d_b, d_r,
                               -1.0, mask_dirichlet ? 1 : 0, plan->scratch64, S(stream));
}

int fem_element_residual_f32(const fem_plan *plan, const float *d_A_e, const float *d_b, const float *d_x,
                             float *d_r, int mask_dirichlet, void *stream) {
    if (int rc = check_plan(plan)) return rc;
    if ((!d_A_e && plan->dev.n_elems > 0) || !d_x || !d_r) return set_error(FEM_EINVAL, "NULL argument");
    if (d_r == d_x || (d_b && d_r == d_b)) return set_error(FEM_EINVAL, "r must not alias x or b");
    return fem::launch_apply32(plan->dev, d_A_e, d_x, d_b, d_r, -1.0f, mask_dirichlet ? 1 : 0, plan->scratch32,
                               S(stream));
}

int fem_jacobi_diag(const fem_plan *plan, int dtype, const void *d_K_e, const void *d_M_e, double nu,
                    double *d_diag, void *stream) {
    if (int rc = check_plan(plan)) return rc;
    if (dtype == FEM_MFREE) {
        if (!d_diag) return set_error(FEM_EINVAL, "NULL argument");
        if (!std::isfinite(nu) || nu < 0.0) return set_error(FEM_EINVAL, "nu must be finite and >= 0");
        return fem::launch_diag_mf(plan->dev, nu, d_diag, plan->scratch64, S(stream));
    }
    if (!valid_dtype(dtype)) return set_error(FEM_EINVAL, "unknown dtype");
    if ((!d_K_e && plan->dev.n_elems > 0) || !d_diag) return set_error(FEM_EINVAL, "NULL argument");
    if (d_M_e && (!std::isfinite(nu) || nu < 0.0)) return set_error(FEM_EINVAL, "nu must be finite and >= 0");
    return fem::launch_diag64(plan->dev, dtype, d_K_e, (d_M_e && nu != 0.0) ? d_M_e : nullptr, nu, d_diag,
                              plan->scratch64, S(stream));
}

int fem_assemble_rhs(const fem_plan *plan, int dtype, const void *d_M_e, const double *d_f, double *d_b,
                     void *stream) {
    if (int rc = check_plan(plan)) return rc;
    if (dtype == FEM_MFREE) {
        if (!d_f || !d_b) return set_error(FEM_EINVAL, "NULL argument");
        if ((const void *)d_b == (const void *)d_f) return set_error(FEM_EINVAL, "b must not alias f");
        return fem::launch_apply_mf(plan->dev, 0.0, 1.0, d_f, nullptr, d_b, 1.0, 0, plan->scratch64, S(stream));
    }
    if (!valid_dtype(dtype)) return set_error(FEM_EINVAL, "unknown dtype");
    if ((!d_M_e && plan->dev.n_elems > 0) || !d_f || !d_b) return set_error(FEM_EINVAL, "NULL argument");
    if ((const void *)d_b == (const void *)d_f) return set_error(FEM_EINVAL, "b must not alias f");
    return fem::launch_apply64(plan->dev, dtype, d_M_e, nullptr, 0.0, d_f, nullptr, d_b, 1.0, 0, plan->scratch64,
                               S(stream));
}

int fem_pcg_solve(const fem_plan *plan_c, const fem_solve_opts *o, const void *d_K_e, const void *d_M_e,
                  const double *d_b, double *d_x, fem_solve_info *info, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (int rc = check_plan(plan_c)) return rc;
    fem_plan *plan = const_cast<fem_plan *>(plan_c);
    if (!o || !info) return set_error(FEM_EINVAL, "opts and info must not be NULL");
    std::memset(info, 0, sizeof(*info));
    const bool mf = o->dtype == FEM_MFREE;
    if (!valid_dtype(o->dtype) && !mf) return set_error(FEM_EINVAL, "unknown dtype");
    if (!std::isfinite(o->nu) || o->nu < 0.0) return set_error(FEM_EINVAL, "nu must be finite and >= 0");
    if (!(o->rtol > 0.0) || !(o->rtol < 1.0)) return set_error(FEM_EINVAL, "rtol must be in (0, 1)");
    if (o->max_iter < 1) return set_error(FEM_EINVAL, "max_iter must be >= 1");
    if (o->check_every < 1 || o->check_every > 4096) return set_error(FEM_EINVAL, "check_every must be in [1, 4096]");
    if (o->precond != FEM_PRECOND_NONE && o->precond != FEM_PRECOND_JACOBI)
        return set_error(FEM_EINVAL, "unknown preconditioner");
    if (o->dtype != FEM_F64 && !mf && (!(o->inner_rtol > 0.0) || !(o->inner_rtol < 1.0) || o->max_outer < 1))
        return set_error(FEM_EINVAL, "mixed precision needs inner_rtol in (0,1) and max_outer >= 1");
    if (o->profile < 0) return set_error(FEM_EINVAL, "profile must be >= 0");
    if (o->vectors != 0 && o->vectors != 1) return set_error(FEM_EINVAL, "vectors must be 0 (FP64) or 1 (FP32)");
    if (o->block != 0 && o->block != 256 && o->block != 512 && o->block != 1024)
        return set_error(FEM_EINVAL, "block must be 0, 256, 512 or 1024");
    if ((!d_K_e && plan->dev.n_elems > 0 && !mf) || !d_b || !d_x) return set_error(FEM_EINVAL, "NULL argument");
    if (o->nu != 0.0 && !d_M_e && !mf) return set_error(FEM_EINVAL, "nu > 0 needs M_e");
    if (mf && o->vectors != 0) return set_error(FEM_EINVAL, "the matrix-free solver keeps FP64 vectors");
    if (plan->dev.nb > 4 && (mf || o->vectors != 0))
        return set_error(FEM_EINVAL, "quadratic elements need stored matrices and FP64 vectors");
    if ((const void *)d_x == (const void *)d_b) return set_error(FEM_EINVAL, "x must not alias b");
    if (o->nu == 0.0 && plan->stats.n_dirichlet == 0)
        return set_error(FEM_ESINGULAR, "nu = 0 needs a Dirichlet part of positive measure");
    if (plan->n_isolated_free > 0)
        return set_error(FEM_ESINGULAR, "a node outside every element is not a Dirichlet node");
    const int slot = mf ? 2 : o->dtype == FEM_F64 ? 0 : 1;
    if (int rc = alloc_work(plan, slot, o->dtype)) return rc;
    hipStream_t s = S(stream);
    // matrix-free: two elements per thread by default (one thread per element
    // leaves too little work to cover the rebuild's LDS and ALU latency)
    const int E = plan->dev.E;
    const int block = o->block ? o->block
                      : mf     ? (E >= 2048 ? 1024 : E >= 1024 ? 512 : 256)
                               : fem::default_block(plan->dev.nb, E);
    int rc = fem::solve_pcg(plan->dev, plan->work[slot], o->dtype, o->vectors == 0, block, d_K_e, d_M_e, o->nu, d_b,
                            d_x, o->rtol,
                            o->max_iter, o->precond == FEM_PRECOND_JACOBI, o->inner_rtol, o->max_outer,
                            o->check_every, o->profile, info, s);
    if (hipStreamSynchronize(s) != hipSuccess && rc == FEM_OK) rc = set_error(FEM_EHIP, "stream synchronisation failed");
    info->status = rc;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc == FEM_ENOCONV) set_error(rc, "iteration limit reached before rtol");
    if (rc == FEM_EBREAKDOWN) set_error(rc, "CG breakdown (p^T A p <= 0 or non-finite scalar)");
    return rc;
}

void fem_iter_opts_default(fem_iter_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->method = FEM_CHEBYSHEV3;
    o->dtype = FEM_F64;
    o->cycle = 1;
}

int fem_iterate(const fem_plan *plan_c, const fem_iter_opts *o, const void *d_K_e, const void *d_M_e,
                const double *d_b, double *d_x, fem_iter_info *info, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (int rc = check_plan(plan_c)) return rc;
    if (!o || !info) return set_error(FEM_EINVAL, "opts and info must not be NULL");
    std::memset(info, 0, sizeof(*info));
    if (o->method < FEM_RICHARDSON || o->method > FEM_CHEBYSHEV3_LISTING)
        return set_error(FEM_EINVAL, "unknown iteration");
    if (plan_c->dev.nb > 4) return set_error(FEM_EINVAL, "the iterations run on linear elements");
    if (!valid_dtype(o->dtype)) return set_error(FEM_EINVAL, "unknown dtype");
    if (!std::isfinite(o->nu) || o->nu < 0.0) return set_error(FEM_EINVAL, "nu must be finite and >= 0");
    if (!std::isfinite(o->lam1) || !std::isfinite(o->lam2) || !(o->lam1 > 0.0) || !(o->lam2 > o->lam1))
        return set_error(FEM_EINVAL, "need finite bounds 0 < lam1 < lam2");
    if (o->iters < 0) return set_error(FEM_EINVAL, "iters must be >= 0");
    if (o->method == FEM_CHEBYSHEV2 && o->cycle < 1) return set_error(FEM_EINVAL, "cycle must be >= 1");
    if ((!d_K_e && plan_c->dev.n_elems > 0) || !d_b || !d_x) return set_error(FEM_EINVAL, "NULL argument");
    if (o->nu != 0.0 && !d_M_e) return set_error(FEM_EINVAL, "nu > 0 needs M_e");
    if ((const void *)d_x == (const void *)d_b) return set_error(FEM_EINVAL, "x must not alias b");
    hipStream_t s = S(stream);
    fem::IterResult res;
    int rc = fem::run_iteration(plan_c->dev, o->dtype, d_K_e, o->nu != 0.0 ? d_M_e : nullptr, o->nu, d_b, d_x,
                                o->method, o->lam1, o->lam2, o->method == FEM_CHEBYSHEV2 ? o->cycle : 1, o->iters,
                                res, s);
    if (hipStreamSynchronize(s) != hipSuccess && rc == FEM_OK) rc = set_error(FEM_EHIP, "stream synchronisation failed");
    info->status = rc;
    info->iters = res.iters;
    info->relres = res.relres;
    info->r0 = res.r0;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

void fem_fcg_opts_default(fem_fcg_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->dtype = FEM_F64;
    o->rtol = 1e-8;
    o->max_iter = 100000;
    o->stall_iters = 200;
    o->max_replace = 8;
    o->smooth = 4;
    o->omega = 2.0 / 3.0;
    o->graph = 1;
    o->check_every = 16;
    o->cycle_dtype = FEM_F64;
}

namespace {

// Validation shared by fem_fcg_solve and fem_fcg_precondition.
int check_fcg(const fem_plan *plan, const fem_fcg_opts *o, fem_unet *net, const void *d_K_e, const void *d_M_e) {
    if (net && plan->dev.nb != 3) return set_error(FEM_EINVAL, "flexible CG with the network runs on linear triangles");
    if (plan->dev.nb != 3 && plan->dev.nb != 4)
        return set_error(FEM_EINVAL, "flexible CG runs on linear triangles or tetrahedra");
    if (!valid_dtype(o->dtype)) return set_error(FEM_EINVAL, "unknown dtype");
    if (!std::isfinite(o->nu) || o->nu < 0.0) return set_error(FEM_EINVAL, "nu must be finite and >= 0");
    if (!(o->rtol > 0.0) || !(o->rtol < 1.0)) return set_error(FEM_EINVAL, "rtol must be in (0, 1)");
    if (o->max_iter < 1) return set_error(FEM_EINVAL, "max_iter must be >= 1");
    if (o->stall_iters < 1 || o->max_replace < 0) return set_error(FEM_EINVAL, "stall_iters >= 1, max_replace >= 0");
    if (o->graph != 0 && o->graph != 1) return set_error(FEM_EINVAL, "graph must be 0 or 1");
    if (o->check_every < 1 || o->check_every > 4096) return set_error(FEM_EINVAL, "check_every must be in [1, 4096]");
    if (o->cycle_dtype != FEM_F64 && o->cycle_dtype != FEM_F32)
        return set_error(FEM_EINVAL, "cycle_dtype: FEM_F64 or FEM_F32");
    if (o->smooth < 0 || o->smooth > 8 || !(o->omega > 0.0) || !(o->omega < 2.0))
        return set_error(FEM_EINVAL, "smooth must be in [0, 8] and omega in (0, 2)");
    if (!d_K_e && plan->dev.n_elems > 0) return set_error(FEM_EINVAL, "NULL argument");
    if (o->nu != 0.0 && !d_M_e) return set_error(FEM_EINVAL, "nu > 0 needs M_e");
    if (o->nu == 0.0 && plan->stats.n_dirichlet == 0)
        return set_error(FEM_ESINGULAR, "nu = 0 needs a Dirichlet part of positive measure");
    if (plan->n_isolated_free > 0)
        return set_error(FEM_ESINGULAR, "a node outside every element is not a Dirichlet node");
    if (net) {
        const int64_t g = o->grid_n;
        if (plan->dev.dim != 2 || g < 8 || (g + 1) * (g + 1) != plan->dev.n_nodes)
            return set_error(FEM_EINVAL, "the network needs a 2D structured grid of (grid_n + 1)^2 nodes");
        if (!std::isfinite(o->cval)) return set_error(FEM_EINVAL, "cval must be finite");
    }
    return 0;
}

}  // namespace

int fem_fcg_precondition(const fem_plan *plan, const fem_fcg_opts *o, fem_unet *net, const void *d_K_e,
                         const void *d_M_e, const double *d_r, double *d_z, void *stream) {
    if (int rc = check_plan(plan)) return rc;
    if (!o) return set_error(FEM_EINVAL, "opts must not be NULL");
    if (int rc = check_fcg(plan, o, net, d_K_e, d_M_e)) return rc;
    if (!d_r || !d_z) return set_error(FEM_EINVAL, "NULL argument");
    if ((const void *)d_r == (const void *)d_z) return set_error(FEM_EINVAL, "z must not alias r");
    return fem::fcg_precondition(plan->dev, o->dtype, d_K_e, o->nu != 0.0 ? d_M_e : nullptr, o->nu, net, o->grid_n,
                                 o->cval, o->smooth, o->omega, o->cycle_dtype == FEM_F32, d_r, d_z, S(stream));
}

int fem_fcg_solve(const fem_plan *plan_c, const fem_fcg_opts *o, fem_unet *net, const void *d_K_e,
                  const void *d_M_e, const double *d_b, double *d_x, fem_fcg_info *info, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (int rc = check_plan(plan_c)) return rc;
    fem_plan *plan = const_cast<fem_plan *>(plan_c);
    if (!o || !info) return set_error(FEM_EINVAL, "opts and info must not be NULL");
    std::memset(info, 0, sizeof(*info));
    info->fell_back = -1;
    if (int rc = check_fcg(plan, o, net, d_K_e, d_M_e)) return rc;
    if (!d_b || !d_x) return set_error(FEM_EINVAL, "NULL argument");
    if ((const void *)d_x == (const void *)d_b) return set_error(FEM_EINVAL, "x must not alias b");
    hipStream_t s = S(stream);
    fem::FcgResult res;
    int rc = fem::solve_fcg(plan->dev, o->dtype, d_K_e, o->nu != 0.0 ? d_M_e : nullptr, o->nu, d_b, d_x, o->rtol,
                            o->max_iter, net, o->grid_n, o->cval, o->smooth, o->omega, o->stall_iters,
                            o->max_replace, o->graph, o->check_every, o->cycle_dtype == FEM_F32, res, s);
    info->iters = res.iters;
    info->precond_calls = res.precond_calls;
    info->fell_back = res.fell_back;
    info->fallback_reason = res.fallback_reason;
    info->replacements = res.replacements;
    info->r0 = res.r0;
    info->relres = res.relres;
    if (rc == fem::kFcgHandover) {
        // Jacobi-PCG from x0 (reset by the FCG phase) to the same absolute
        // target (res.rnorm: the true residual norm of x0)
        fem_solve_opts po;
        fem_solve_opts_default(&po);
        po.dtype = o->dtype;
        po.nu = o->nu;
        po.max_iter = o->max_iter;
        po.rtol = std::min(0.5, o->rtol * res.r0 / std::max(res.rnorm, 1e-300));
        fem_solve_info pi;
        rc = fem_pcg_solve(plan, &po, d_K_e, d_M_e, d_b, d_x, &pi, stream);
        info->pcg_iters = pi.iters;
        info->relres = res.r0 > 0.0 ? pi.relres * pi.r0 / res.r0 : 0.0;
    }
    if (hipStreamSynchronize(s) != hipSuccess && rc == FEM_OK) rc = set_error(FEM_EHIP, "stream synchronisation failed");
    info->status = rc;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

}  // extern "C"

// ---- Element residual without allocation -----------------------------------
// The shared-node partials of the element pass live in one file-scope device
// array instead of the plan's workspace.  In host code `scratch` names a
// host-side stand-in; the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address reaches the kernels.

namespace {

constexpr int64_t kNoAllocPartials = (int64_t)1 << 22;  // FP64 partials: 32 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kNoAllocPartials];

double *g_scratch_addr[kMaxDevices] = {};

int scratch_address(double **out) {
    int dev = 0;
    FEM_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(FEM_EINVAL, "device index beyond the supported range");
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(FEM_EHIP, std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                           hipGetErrorString(e));
        g_scratch_addr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_addr[dev];
    return 0;
}

}  // namespace

extern "C" {

int fem_element_residual_noalloc(const fem_plan *plan, int dtype, const void *d_K_e, const void *d_M_e, double nu,
                                 const double *d_b, const double *d_x, double *d_r, int mask_dirichlet,
                                 void *stream) {
    if (int rc = check_plan(plan)) return rc;
    if (plan->dev.n_partials > kNoAllocPartials)
        return set_error(FEM_EINVAL, "the plan has " + std::to_string(plan->dev.n_partials) +
                                         " shared-node partials; the allocation-free residual holds at most " +
                                         std::to_string(kNoAllocPartials) + " (use smaller meshes or larger chunks)");
    const bool mf = dtype == FEM_MFREE;
    if (!mf && !valid_dtype(dtype)) return set_error(FEM_EINVAL, "unknown dtype");
    if ((!mf && !d_K_e && plan->dev.n_elems > 0) || !d_x || !d_r) return set_error(FEM_EINVAL, "NULL argument");
    if ((mf || d_M_e) && (!std::isfinite(nu) || nu < 0.0)) return set_error(FEM_EINVAL, "nu must be finite and >= 0");
    if ((const void *)d_r == (const void *)d_x || (d_b && (const void *)d_r == (const void *)d_b))
        return set_error(FEM_EINVAL, "r must not alias x or b");
    double *part = nullptr;
    if (int rc = scratch_address(&part)) return rc;
    const int mask = mask_dirichlet ? 1 : 0;
    if (mf) return fem::launch_apply_mf(plan->dev, 1.0, nu, d_x, d_b, d_r, -1.0, mask, part, S(stream));
    return fem::launch_apply64(plan->dev, dtype, d_K_e, (d_M_e && nu != 0.0) ? d_M_e : nullptr, nu, d_x, d_b, d_r,
                               -1.0, mask, part, S(stream));
}

}  // extern "C"
