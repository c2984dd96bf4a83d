// plan_check.cpp -- host-only parts of the C ABI: the error message, the
// chunk-size rules and the host dry run of the planner (fem_plan_check_host,
// fem_plan_check_host_p2).  Plain C++ with no HIP, so that the planner can
// also be built and exercised with the host sanitizers.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "fem.h"
#include "plan.h"

namespace fem {

std::string &last_error() {
    static thread_local std::string msg;
    return msg;
}

int set_error(int code, const std::string &msg) {
    last_error() = msg;
    return code;
}

bool valid_chunk_elems(int nb, int E) {
    switch (E) {
        case 64: case 128: case 256: case 512: case 1024: case 1536: case 2048: break;
        default: return false;
    }
    // FP64 slot buffer + uint16 slot list within kMaxChunkLds
    return (size_t)nb * E * (8 + 2) <= (size_t)kMaxChunkLds;
}

int default_chunk_elems(int nb) { return nb == 3 ? 1024 : nb == 4 ? 1536 : nb == 6 ? 1024 : 512; }

}  // namespace fem

using fem::set_error;

namespace {

int check_host(int dim, int nb, int64_t n_nodes, int64_t n_elems, const double *coords, const int32_t *conn,
               const int32_t *dirichlet, int64_t n_dirichlet, int chunk_elems, fem_plan_stats *out) {
    fem::last_error().clear();
    if (!out) return set_error(FEM_EINVAL, "out is NULL");
    if (dim != 2 && dim != 3) return set_error(FEM_EINVAL, "dim must be 2 or 3");
    if (n_nodes < 1 || n_nodes > INT32_MAX) return set_error(FEM_EINVAL, "n_nodes must be in [1, 2^31)");
    if (n_elems < 0 || n_elems > INT32_MAX) return set_error(FEM_EINVAL, "n_elems must be in [0, 2^31)");
    if (!coords || (n_elems > 0 && !conn)) return set_error(FEM_EINVAL, "NULL argument");
    if (n_dirichlet < 0 || (n_dirichlet > 0 && !dirichlet)) return set_error(FEM_EINVAL, "bad Dirichlet list");
    if (chunk_elems == 0) chunk_elems = fem::default_chunk_elems(nb);
    if (!fem::valid_chunk_elems(nb, chunk_elems))
        return set_error(FEM_EINVAL, nb == 3    ? "chunk_elems must be one of 64, 128, 256, 512, 1024, 1536, 2048"
                                     : nb == 4  ? "chunk_elems must be one of 64, 128, 256, 512, 1024, 1536"
                                     : nb == 6  ? "chunk_elems must be one of 64, 128, 256, 512, 1024"
                                                : "chunk_elems must be one of 64, 128, 256, 512");
    for (int64_t i = 0; i < (int64_t)dim * n_nodes; ++i)
        if (!std::isfinite(coords[i])) return set_error(FEM_EINVAL, "non-finite coordinate");
    fem::HostPlan H;
    std::string err;
    try {
        if (fem::build_host_plan(dim, nb, n_nodes, n_elems, coords, conn, dirichlet, n_dirichlet, chunk_elems, H, err))
            return set_error(FEM_EINVAL, err);
    } catch (const std::bad_alloc &) {
        return set_error(FEM_ENOMEM, "host allocation failed while building the plan");
    }
    std::memset(out, 0, sizeof(*out));
    out->dim = dim;
    out->n_b = nb;
    out->n_nodes = n_nodes;
    out->n_elems = n_elems;
    out->n_dirichlet = H.n_dirichlet;
    out->chunk_elems = chunk_elems;
    out->n_chunks = H.n_chunks;
    out->n_local = H.n_local;
    out->n_shared = H.n_shared;
    out->n_partials = H.n_partials;
    out->index_bytes = (int64_t)(H.chunk_node_off.size() * 4 + H.chunk_info.size() * 4 + H.loc_nodes.size() * 4 +
                                 H.loc_end.size() * 2 + H.slots.size() * 2 + H.fix_nodes.size() * 4 +
                                 H.fix_off.size() * 4 + H.fix_parts.size() * 8 + H.comp_off.size() * 4 +
                                 H.fix_rec.size() * 4 +
                                 H.mask.size());
    return FEM_OK;
}
}  // namespace

extern "C" {

int fem_plan_check_host(int dim, int64_t n_nodes, int64_t n_elems, const double *coords, const int32_t *conn,
                        const int32_t *dirichlet, int64_t n_dirichlet, int chunk_elems, fem_plan_stats *out) {
    return check_host(dim, dim + 1, n_nodes, n_elems, coords, conn, dirichlet, n_dirichlet, chunk_elems, out);
}

int fem_plan_check_host_p2(int dim, int64_t n_nodes, int64_t n_elems, const double *coords, const int32_t *conn,
                           const int32_t *dirichlet, int64_t n_dirichlet, int chunk_elems, fem_plan_stats *out) {
    return check_host(dim, dim == 2 ? 6 : 10, n_nodes, n_elems, coords, conn, dirichlet, n_dirichlet, chunk_elems,
                      out);
}

}  // extern "C"
