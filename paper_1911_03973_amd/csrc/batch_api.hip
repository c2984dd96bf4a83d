// batch_api.hip -- C ABI of the batched solver (include/fem.h).
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

struct fem_batch {
    fem::DevPlan dev{};
    fem_plan_stats stats{};
    int nprob = 0;
    void *arena = nullptr;
    int32_t *pchunk0 = nullptr, *pshared0 = nullptr, *pseg0 = nullptr;
    int32_t *pgroup = nullptr, *pitem0 = nullptr;  // work-item schedule (per solve)
    std::vector<int32_t> h_chunk0;
    int64_t *elem0 = nullptr;
    double *scratch64 = nullptr;
    std::vector<int64_t> n_dir, isolated_free;
    int64_t n_seg = 0;
    // solver workspace (allocated on the first solve)
    void *work = nullptr;
    fem::BatchLaunch L{};
    float *Apk = nullptr;
    double *d64 = nullptr, *nu = nullptr;
    double *xl = nullptr, *bl = nullptr;  // x and b in the solver-local node order
    int32_t *perm = nullptr;              // local index -> union node id
    std::vector<fem::BatchProblem> host_prob;
    // captured graph and the arguments it was captured with
    hipGraphExec_t graph = nullptr;
    hipStream_t cap_stream = nullptr;
    const void *g_K = nullptr, *g_M = nullptr, *g_b = nullptr;
    void *g_x = nullptr;
    int g_dtype = -1;
    fem_batch_opts g_opts{};
};

namespace {

using fem::set_error;

size_t align_up(size_t v) { return (v + 255) / 256 * 256; }

struct Layout {
    size_t total = 0;
    size_t add(size_t bytes) {
        size_t off = total;
        total = align_up(total + std::max<size_t>(bytes, 1));
        return off;
    }
};

// perm[local] = union node id: the complete nodes chunk by chunk, then the shared nodes
__global__ void k_batch_perm(const fem::DevPlan P, int32_t *__restrict__ perm) {
    for (int64_t c = blockIdx.x; c < P.n_chunks; c += gridDim.x) {
        const int nb0 = P.chunk_node_off[c], ncomp = P.chunk_info[2 * c], off = P.comp_off[c];
        for (int k = threadIdx.x; k < ncomp; k += blockDim.x) perm[off + k] = P.loc_nodes[nb0 + k];
    }
    const int64_t nc = P.comp_off[P.n_chunks];
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < P.n_shared;
         s += (int64_t)gridDim.x * blockDim.x)
        perm[nc + s] = P.fix_nodes[s];
}

// dst[i] = src[perm[i]] (union order -> local order)
__global__ void k_batch_gather(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ src,
                               double *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = src[perm[i]];
}

// dst[perm[i]] = src[i] (local order -> union order)
__global__ void k_batch_scatter(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ src,
                                double *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[perm[i]] = src[i];
}

// D^{-1} in local order, 0 on Dirichlet nodes
__global__ void k_batch_dinv(int64_t n, const double *__restrict__ d, const uint8_t *__restrict__ mask,
                             const int32_t *__restrict__ perm, double *__restrict__ dinv) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int g = perm[i];
        dinv[i] = (mask[g] || !(d[g] > 0.0)) ? 0.0 : 1.0 / d[g];
    }
}

int alloc_batch_work(fem_batch *B) {
    if (B->work) return FEM_OK;
    const fem::DevPlan &P = B->dev;
    const int64_t n = P.n_nodes, ne = P.n_elems;
    const int64_t npk = (int64_t)fem::packed_count(P.nb) * ne;
    unsigned long long cap = 1;
    // outstanding items: at most one phase per problem, i.e. its CHUNK items
    // (<= its chunks) or its FIX items (its segments) plus one
    while (cap < (unsigned long long)(2 * (P.n_chunks + B->n_seg + B->nprob) + 4096)) cap <<= 1;
    Layout L;
    size_t oA = L.add((size_t)npk * 2 * sizeof(float));
    size_t od = L.add(n * sizeof(double));
    size_t odi = L.add(n * sizeof(double));
    size_t orr = L.add(n * sizeof(double));
    size_t opp = L.add(n * sizeof(double));
    size_t oqq = L.add(n * sizeof(double));
    size_t oxl = L.add(n * sizeof(double));
    size_t obl = L.add(n * sizeof(double));
    size_t operm = L.add(n * sizeof(int32_t));
    size_t opart = L.add(std::max<int64_t>(P.n_partials, 1) * sizeof(double));
    size_t oprob = L.add((size_t)B->nprob * sizeof(fem::BatchProblem));
    size_t ocnt = L.add((size_t)B->nprob * sizeof(int));
    size_t ocd = L.add((size_t)std::max<int64_t>(P.n_chunks, 1) * 7 * sizeof(double));
    size_t osd = L.add((size_t)std::max<int64_t>(B->n_seg, 1) * 7 * sizeof(double));
    size_t oqi = L.add((size_t)cap * sizeof(unsigned long long));
    size_t oqt = L.add((size_t)cap * sizeof(unsigned long long));
    size_t octl = L.add(4 * sizeof(unsigned long long));
    size_t oflags = L.add(4 * sizeof(int));
    size_t onu = L.add((size_t)B->nprob * sizeof(double));
    if (hipMalloc(&B->work, L.total) != hipSuccess) {
        (void)hipGetLastError();
        B->work = nullptr;
        return set_error(FEM_ENOMEM, "device allocation of the batched workspace failed");
    }
    char *b = static_cast<char *>(B->work);
    fem::BatchLaunch &W = B->L;
    W.P = P;
    B->Apk = reinterpret_cast<float *>(b + oA);
    W.A = B->Apk;
    B->d64 = reinterpret_cast<double *>(b + od);
    W.dinv = reinterpret_cast<double *>(b + odi);
    W.r = reinterpret_cast<double *>(b + orr);
    W.p = reinterpret_cast<double *>(b + opp);
    W.q = reinterpret_cast<double *>(b + oqq);
    B->xl = reinterpret_cast<double *>(b + oxl);
    B->bl = reinterpret_cast<double *>(b + obl);
    B->perm = reinterpret_cast<int32_t *>(b + operm);
    W.part = reinterpret_cast<double *>(b + opart);
    W.prob = reinterpret_cast<fem::BatchProblem *>(b + oprob);
    W.cnt = reinterpret_cast<int *>(b + ocnt);
    W.cdots = reinterpret_cast<double *>(b + ocd);
    W.sdots = reinterpret_cast<double *>(b + osd);
    W.qitems = reinterpret_cast<unsigned long long *>(b + oqi);
    W.qtags = reinterpret_cast<unsigned long long *>(b + oqt);
    W.qhead = reinterpret_cast<unsigned long long *>(b + octl);
    W.qtail = W.qhead + 1;
    W.qcap = cap;
    W.ndone = reinterpret_cast<int *>(b + oflags);
    W.abort_flag = W.ndone + 1;
    B->nu = reinterpret_cast<double *>(b + onu);
    W.pchunk0 = B->pchunk0;
    W.pshared0 = B->pshared0;
    W.pseg0 = B->pseg0;
    W.pgroup = B->pgroup;
    W.pitem0 = B->pitem0;
    W.nprob = B->nprob;
    B->host_prob.resize(B->nprob);
    return FEM_OK;
}

// The whole device side of one batched solve, in stream order.
int enqueue_solve(fem_batch *B, const fem_batch_opts *o, const void *K, const void *M, const double *b, double *x,
                  hipStream_t s) {
    fem::BatchLaunch &W = B->L;
    const fem::DevPlan &P = B->dev;
    int rc = fem::batch_pack(P, o->dtype, K, M, B->nu, B->elem0, B->nprob, B->Apk, s);
    if (rc) return rc;
    rc = fem::launch_diag_pk64(P, fem::MAT_F32X2, B->Apk, B->d64, B->scratch64, s);
    if (rc) return rc;
    const int64_t n = P.n_nodes;
    const int gv = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    k_batch_perm<<<gv, 256, 0, s>>>(P, B->perm);
    k_batch_dinv<<<gv, 256, 0, s>>>(n, B->d64, P.mask, B->perm, const_cast<double *>(W.dinv));
    k_batch_gather<<<gv, 256, 0, s>>>(n, B->perm, x, B->xl);
    k_batch_gather<<<gv, 256, 0, s>>>(n, B->perm, b, B->bl);
    FEM_HIP_CHECK(hipGetLastError());
    W.x = B->xl;
    W.b = B->bl;
    W.rtol = o->rtol;
    W.delta = o->refresh;
    W.max_iter = o->max_iter;
    W.max_refresh = o->max_refresh;
    W.watchdog_seconds = o->watchdog_seconds;
    W.block = o->block ? o->block : fem::default_block(P.nb, P.E);
    W.grid = o->grid;
    rc = fem::batch_launch(W, s);
    if (rc) return rc;
    k_batch_scatter<<<gv, 256, 0, s>>>(n, B->perm, B->xl, x);
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

bool same_opts(const fem_batch_opts &a, const fem_batch_opts &b) { return std::memcmp(&a, &b, sizeof(a)) == 0; }

}  // namespace

extern "C" {

void fem_batch_opts_default(fem_batch_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->dtype = FEM_F32X2;
    o->rtol = 1e-8;
    o->max_iter = 20000;
    o->refresh = 0.1;
    o->max_refresh = 200;
    o->block = 0;
    o->grid = 0;
    o->watchdog_seconds = 30.0;
    o->use_graph = 1;
    o->group = 0;
    o->items_per_phase = 4;
    o->inline_segments = 64;
    o->adaptive = 1;
}

int fem_batch_create(int dim, int n_problems, const int64_t *node_off, const int64_t *elem_off,
                     const int64_t *dir_off, const double *d_coords, const int32_t *d_conn,
                     const int32_t *d_dirichlet, int chunk_elems, void *stream, fem_batch **out) {
    fem::last_error().clear();
    if (!out) return set_error(FEM_EINVAL, "out is NULL");
    *out = nullptr;
    if (dim != 2 && dim != 3) return set_error(FEM_EINVAL, "dim must be 2 or 3");
    if (n_problems < 1 || n_problems > (1 << 20)) return set_error(FEM_EINVAL, "n_problems must be in [1, 2^20]");
    if (!node_off || !elem_off || !dir_off) return set_error(FEM_EINVAL, "offset arrays must not be NULL");
    if (node_off[0] != 0 || elem_off[0] != 0 || dir_off[0] != 0) return set_error(FEM_EINVAL, "offsets start at 0");
    for (int p = 0; p < n_problems; ++p)
        if (node_off[p + 1] <= node_off[p] || elem_off[p + 1] < elem_off[p] || dir_off[p + 1] < dir_off[p])
            return set_error(FEM_EINVAL, "offsets must increase (every problem needs a node)");
    const int64_t NN = node_off[n_problems], NE = elem_off[n_problems], ND = dir_off[n_problems];
    if (NN > INT32_MAX || NE > INT32_MAX) return set_error(FEM_EINVAL, "union too large");
    if (!d_coords || (NE > 0 && !d_conn) || (ND > 0 && !d_dirichlet)) return set_error(FEM_EINVAL, "NULL argument");
    const int nb = dim + 1;
    if (chunk_elems == 0) chunk_elems = fem::default_chunk_elems(nb);
    if (!fem::valid_chunk_elems(nb, chunk_elems)) return set_error(FEM_EINVAL, "unsupported chunk_elems");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::vector<double> coords((size_t)dim * NN);
    std::vector<int32_t> conn((size_t)nb * NE), dir((size_t)ND);
    FEM_HIP_CHECK(hipMemcpyAsync(coords.data(), d_coords, coords.size() * 8, hipMemcpyDeviceToHost, s));
    if (NE) FEM_HIP_CHECK(hipMemcpyAsync(conn.data(), d_conn, conn.size() * 4, hipMemcpyDeviceToHost, s));
    if (ND) FEM_HIP_CHECK(hipMemcpyAsync(dir.data(), d_dirichlet, dir.size() * 4, hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    for (double c : coords)
        if (!std::isfinite(c)) return set_error(FEM_EINVAL, "non-finite coordinate");
    fem::BatchHost H;
    std::string err;
    try {
        if (fem::build_batch_plan(dim, n_problems, node_off, elem_off, dir_off, coords.data(), conn.data(),
                                  dir.data(), chunk_elems, H, err))
            return set_error(FEM_EINVAL, err);
    } catch (const std::bad_alloc &) {
        return set_error(FEM_ENOMEM, "host allocation failed while building the batch");
    }
    // global connectivity for the union-level element kernels
    for (int p = 0; p < n_problems; ++p)
        for (int a = 0; a < nb; ++a)
            for (int64_t e = elem_off[p]; e < elem_off[p + 1]; ++e) conn[(size_t)a * NE + e] += (int32_t)node_off[p];
    std::vector<int32_t> pseg(n_problems + 1, 0);
    for (int p = 0; p < n_problems; ++p) {
        const int ns = H.shared0[p + 1] - H.shared0[p];
        pseg[p + 1] = pseg[p] + (ns + fem::kBatchSeg - 1) / fem::kBatchSeg;
    }
    const fem::HostPlan &U = H.U;
    Layout L;
    const size_t o_coords = L.add(coords.size() * 8), o_conn = L.add(conn.size() * 4);
    const size_t o_cno = L.add(U.chunk_node_off.size() * 4), o_cin = L.add(U.chunk_info.size() * 4);
    const size_t o_ln = L.add(U.loc_nodes.size() * 4), o_le = L.add(U.loc_end.size() * 2);
    const size_t o_sl = L.add(U.slots.size() * 2), o_fn = L.add(U.fix_nodes.size() * 4);
    const size_t o_fo = L.add(U.fix_off.size() * 4), o_fp = L.add(U.fix_parts.size() * 4);
    const size_t o_po = L.add(U.part_owner.size() * 4), o_mask = L.add(U.mask.size());
    const size_t o_co = L.add(U.comp_off.size() * 4);
    const size_t o_ce = L.add(H.chunk_elem0.size() * 8);
    const size_t o_pc = L.add((n_problems + 1) * 4), o_ps = L.add((n_problems + 1) * 4);
    const size_t o_pg = L.add((n_problems + 1) * 4), o_pe = L.add((n_problems + 1) * 8);
    const size_t o_grp = L.add((n_problems + 1) * 4), o_it0 = L.add((n_problems + 1) * 4);
    const size_t o_s64 = L.add(std::max<int64_t>(U.n_partials, 1) * 8);
    fem_batch *B = new (std::nothrow) fem_batch();
    if (!B) return set_error(FEM_ENOMEM, "host allocation failed");
    if (hipMalloc(&B->arena, L.total) != hipSuccess) {
        (void)hipGetLastError();
        delete B;
        return set_error(FEM_ENOMEM, "device allocation of the batch failed");
    }
    char *b = static_cast<char *>(B->arena);
    int bad = 0;
    auto up = [&](size_t off, const void *src, size_t bytes) {
        if (bytes && hipMemcpyAsync(b + off, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess) bad = 1;
    };
    up(o_coords, coords.data(), coords.size() * 8);
    up(o_conn, conn.data(), conn.size() * 4);
    up(o_cno, U.chunk_node_off.data(), U.chunk_node_off.size() * 4);
    up(o_cin, U.chunk_info.data(), U.chunk_info.size() * 4);
    up(o_ln, U.loc_nodes.data(), U.loc_nodes.size() * 4);
    up(o_le, U.loc_end.data(), U.loc_end.size() * 2);
    up(o_sl, U.slots.data(), U.slots.size() * 2);
    up(o_fn, U.fix_nodes.data(), U.fix_nodes.size() * 4);
    up(o_fo, U.fix_off.data(), U.fix_off.size() * 4);
    up(o_fp, U.fix_parts.data(), U.fix_parts.size() * 4);
    up(o_po, U.part_owner.data(), U.part_owner.size() * 4);
    up(o_co, U.comp_off.data(), U.comp_off.size() * 4);
    up(o_mask, U.mask.data(), U.mask.size());
    up(o_ce, H.chunk_elem0.data(), H.chunk_elem0.size() * 8);
    up(o_pc, H.chunk0.data(), (n_problems + 1) * 4);
    up(o_ps, H.shared0.data(), (n_problems + 1) * 4);
    up(o_pg, pseg.data(), (n_problems + 1) * 4);
    up(o_pe, H.elem0.data(), (n_problems + 1) * 8);
    if (bad || hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(B->arena);
        delete B;
        return set_error(FEM_EHIP, "upload of the batch failed");
    }
    fem::DevPlan &D = B->dev;
    D.dim = dim;
    D.nb = nb;
    D.E = chunk_elems;
    D.n_nodes = NN;
    D.n_elems = NE;
    D.n_chunks = U.n_chunks;
    D.n_local = U.n_local;
    D.n_shared = U.n_shared;
    D.n_partials = U.n_partials;
    D.max_local = 0;
    for (size_t c = 0; c + 1 < U.chunk_node_off.size(); ++c)
        D.max_local = std::max(D.max_local, U.chunk_node_off[c + 1] - U.chunk_node_off[c]);
    D.chunk_elem0 = reinterpret_cast<const int64_t *>(b + o_ce);
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
    D.comp_off = reinterpret_cast<const int32_t *>(b + o_co);
    D.mask = reinterpret_cast<const uint8_t *>(b + o_mask);
    B->pchunk0 = reinterpret_cast<int32_t *>(b + o_pc);
    B->pshared0 = reinterpret_cast<int32_t *>(b + o_ps);
    B->pseg0 = reinterpret_cast<int32_t *>(b + o_pg);
    B->elem0 = reinterpret_cast<int64_t *>(b + o_pe);
    B->pgroup = reinterpret_cast<int32_t *>(b + o_grp);
    B->pitem0 = reinterpret_cast<int32_t *>(b + o_it0);
    B->h_chunk0 = H.chunk0;
    B->scratch64 = reinterpret_cast<double *>(b + o_s64);
    B->nprob = n_problems;
    B->n_dir = H.n_dir;
    B->isolated_free = H.isolated_free;
    B->n_seg = pseg[n_problems];
    fem_plan_stats &st = B->stats;
    st.dim = dim;
    st.n_b = nb;
    st.n_nodes = NN;
    st.n_elems = NE;
    st.n_dirichlet = U.n_dirichlet;
    st.chunk_elems = chunk_elems;
    st.n_chunks = U.n_chunks;
    st.n_local = U.n_local;
    st.n_shared = U.n_shared;
    st.n_partials = U.n_partials;
    st.index_bytes = (int64_t)(o_s64 - o_cno);
    *out = B;
    return FEM_OK;
}

int fem_batch_destroy(fem_batch *B) {
    if (!B) return FEM_OK;
    if (B->graph) (void)hipGraphExecDestroy(B->graph);
    if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
    if (B->work) (void)hipFree(B->work);
    if (B->arena) (void)hipFree(B->arena);
    delete B;
    return FEM_OK;
}

int fem_batch_get_stats(const fem_batch *B, fem_plan_stats *out) {
    if (!B || !out) return set_error(FEM_EINVAL, "NULL argument");
    *out = B->stats;
    return FEM_OK;
}

int fem_batch_build_local_matrices(const fem_batch *B, int dtype, void *d_K_e, void *d_M_e, void *stream) {
    if (!B) return set_error(FEM_EINVAL, "batch is NULL");
    if (dtype != FEM_F64 && dtype != FEM_F32 && dtype != FEM_F32X2) return set_error(FEM_EINVAL, "unknown dtype");
    if (B->dev.n_elems == 0 || (!d_K_e && !d_M_e)) return FEM_OK;
    return fem::launch_local_matrices(B->dev, dtype, d_K_e, d_M_e, nullptr, reinterpret_cast<hipStream_t>(stream));
}

int fem_batch_assemble_rhs(const fem_batch *B, int dtype, const void *d_M_e, const double *d_f, double *d_b,
                           void *stream) {
    if (!B) return set_error(FEM_EINVAL, "batch is NULL");
    if (dtype != FEM_F64 && dtype != FEM_F32 && dtype != FEM_F32X2) return set_error(FEM_EINVAL, "unknown dtype");
    if ((!d_M_e && B->dev.n_elems > 0) || !d_f || !d_b || (const void *)d_f == (const void *)d_b)
        return set_error(FEM_EINVAL, "bad argument");
    return fem::launch_apply64(B->dev, dtype, d_M_e, nullptr, 0.0, d_f, nullptr, d_b, 1.0, 0, B->scratch64,
                               reinterpret_cast<hipStream_t>(stream));
}

int fem_batch_solve(fem_batch *B, const fem_batch_opts *o, const void *d_K_e, const void *d_M_e, const double *h_nu,
                    const double *d_b, double *d_x, fem_batch_result *results, double *seconds, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!B || !o || !h_nu || !results) return set_error(FEM_EINVAL, "NULL argument");
    if (o->dtype != FEM_F64 && o->dtype != FEM_F32 && o->dtype != FEM_F32X2)
        return set_error(FEM_EINVAL, "unknown dtype");
    if (!(o->rtol > 0.0 && o->rtol < 1.0) || o->max_iter < 1 || !(o->refresh > 0.0 && o->refresh < 1.0) ||
        o->max_refresh < 1 || !(o->watchdog_seconds > 0.0 && o->watchdog_seconds <= 600.0) || o->grid < 0)
        return set_error(FEM_EINVAL, "bad solver options");
    if (o->block != 0 && o->block != 256 && o->block != 512 && o->block != 1024)
        return set_error(FEM_EINVAL, "block must be 0, 256, 512 or 1024");
    if ((!d_K_e || !d_M_e) && B->dev.n_elems > 0) return set_error(FEM_EINVAL, "K_e and M_e are needed");
    if (!d_b || !d_x || (const void *)d_b == (const void *)d_x) return set_error(FEM_EINVAL, "bad b / x");
    for (int p = 0; p < B->nprob; ++p) {
        if (!std::isfinite(h_nu[p]) || h_nu[p] < 0.0) return set_error(FEM_EINVAL, "nu must be finite and >= 0");
        if (h_nu[p] == 0.0 && B->n_dir[p] == 0)
            return set_error(FEM_ESINGULAR, "problem " + std::to_string(p) + ": nu = 0 without Dirichlet nodes");
        if (B->isolated_free[p] > 0)
            return set_error(FEM_ESINGULAR, "problem " + std::to_string(p) + ": node outside every element");
    }
    if (o->group < 0 || o->items_per_phase < 1 || o->inline_segments < 0 || (o->adaptive != 0 && o->adaptive != 1))
        return set_error(FEM_EINVAL, "bad work-item schedule");
    if (int rc = alloc_batch_work(B)) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // work-item schedule: chunks per item for every problem, and the prefix
    // of items of one chunk round
    std::vector<int32_t> grp(B->nprob), it0(B->nprob + 1, 0);
    for (int p = 0; p < B->nprob; ++p) {
        const int nch = B->h_chunk0[p + 1] - B->h_chunk0[p];
        grp[p] = o->group > 0 ? o->group : std::max(1, (nch + o->items_per_phase - 1) / o->items_per_phase);
        it0[p + 1] = it0[p] + (nch + grp[p] - 1) / grp[p];
    }
    B->L.n_seed = it0[B->nprob];
    B->L.inline_segs = o->inline_segments;
    B->L.adaptive = o->group > 0 ? 0 : o->adaptive;
    FEM_HIP_CHECK(hipMemcpyAsync(B->pgroup, grp.data(), B->nprob * sizeof(int32_t), hipMemcpyHostToDevice, s));
    FEM_HIP_CHECK(hipMemcpyAsync(B->pitem0, it0.data(), (B->nprob + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    FEM_HIP_CHECK(hipMemcpyAsync(B->nu, h_nu, B->nprob * sizeof(double), hipMemcpyHostToDevice, s));
    int rc = 0;
    if (o->use_graph) {
        const bool reuse = B->graph && B->g_K == d_K_e && B->g_M == d_M_e && B->g_b == d_b && B->g_x == d_x &&
                           B->g_dtype == o->dtype && same_opts(B->g_opts, *o);
        if (!reuse) {
            if (B->graph) {
                (void)hipGraphExecDestroy(B->graph);
                B->graph = nullptr;
            }
            if (!B->cap_stream) FEM_HIP_CHECK(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
            FEM_HIP_CHECK(hipStreamSynchronize(s));
            hipGraph_t g;
            FEM_HIP_CHECK(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
            rc = enqueue_solve(B, o, d_K_e, d_M_e, d_b, d_x, B->cap_stream);
            hipError_t e = hipStreamEndCapture(B->cap_stream, &g);
            if (rc) return rc;
            if (e != hipSuccess) return set_error(FEM_EHIP, "graph capture failed");
            e = hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                B->graph = nullptr;
                return set_error(FEM_EHIP, "graph instantiation failed");
            }
            B->g_K = d_K_e;
            B->g_M = d_M_e;
            B->g_b = d_b;
            B->g_x = d_x;
            B->g_dtype = o->dtype;
            B->g_opts = *o;
        }
        FEM_HIP_CHECK(hipGraphLaunch(B->graph, s));
    } else {
        rc = enqueue_solve(B, o, d_K_e, d_M_e, d_b, d_x, s);
        if (rc) return rc;
    }
    int flags[2] = {0, 0};
    FEM_HIP_CHECK(hipMemcpyAsync(B->host_prob.data(), B->L.prob, B->nprob * sizeof(fem::BatchProblem),
                                 hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipMemcpyAsync(flags, B->L.ndone, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int status = FEM_OK;
    for (int p = 0; p < B->nprob; ++p) {
        const fem::BatchProblem &h = B->host_prob[p];
        results[p].status = h.flag ? h.status : FEM_ENOCONV;
        results[p].iters = h.iters;
        results[p].refreshes = h.refreshes;
        results[p].r0 = h.r0;
        results[p].relres = h.r0 > 0.0 ? std::sqrt(h.rr_true) / h.r0 : 0.0;
        if (status == FEM_OK && results[p].status != FEM_OK) status = results[p].status;
    }
    if (flags[1]) return set_error(FEM_EHIP, "batched solver: the watchdog ended the launch (queue stayed empty)");
    if (status != FEM_OK) set_error(status, "a problem of the batch did not converge");
    return status;
}

}  // extern "C"
