// plan.h -- chunked element -> node index (host side) and its device mirror.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fem {

// Largest chunk the kernels accept: the FP64 slot buffer plus the uint16 slot
// list of one chunk must fit in 64 KiB of LDS.
constexpr int kMaxChunkLds = 65536;

bool valid_chunk_elems(int nb, int E);
int default_chunk_elems(int nb);

// Thread-local message of the last failed call, and the setter every error
// path uses (returns code).
std::string &last_error();
int set_error(int code, const std::string &msg);

struct HostPlan {
    int dim = 0, nb = 0, E = 0;
    int64_t n_nodes = 0, n_elems = 0, n_chunks = 0;
    int64_t n_local = 0, n_shared = 0, n_partials = 0, n_dirichlet = 0;
    int64_t n_isolated = 0, n_isolated_free = 0;
    std::vector<int32_t> chunk_node_off;  // [n_chunks+1] into loc_nodes / loc_end
    std::vector<int32_t> chunk_info;      // [n_chunks][2]: n_complete, partial_base
    std::vector<int32_t> loc_nodes;       // [n_local] global node ids
    std::vector<uint16_t> loc_end;        // [n_local] end of the node's slot run
    std::vector<uint16_t> slots;          // [n_chunks][nb*E] slot ids grouped by node
    std::vector<int32_t> fix_nodes;       // [n_shared] nodes in != 1 chunk (incl. isolated)
    std::vector<int32_t> fix_off;         // [n_shared+1]
    std::vector<int32_t> fix_parts;       // [n_partials]
    std::vector<int32_t> part_owner;      // [n_partials] shared-node index of each partial slot
    // [n_shared][4] the first partial slots of each shared node (ascending
    // chunk order), -1 where it has fewer; with more than four, entry 3 is
    // -2 - k and the slots from the fourth on are fix_parts[k .. fix_off[s+1])
    std::vector<int32_t> fix_rec;
    std::vector<int32_t> comp_off;        // [n_chunks+1] prefix of the complete-node counts
    std::vector<uint8_t> mask;            // [n_nodes] Dirichlet flags
};

// Device-resident index (raw pointers into plan-owned allocations).
struct DevPlan {
    int dim, nb, E;
    int max_local;  // most distinct nodes of one chunk
    int64_t n_nodes, n_elems, n_chunks, n_local, n_shared, n_partials;
    const int64_t *chunk_elem0;  // [n_chunks+1] first element of each chunk; NULL: chunk c starts at c*E
    const double *coords;        // [dim][n_nodes]
    const int32_t *conn;         // [nb][n_elems]
    const int32_t *chunk_node_off;
    const int32_t *chunk_info;
    const int32_t *loc_nodes;
    const uint16_t *loc_end;
    const uint16_t *slots;
    const int32_t *fix_nodes;
    const int32_t *fix_off;
    const int32_t *fix_parts;
    const int32_t *part_owner;
    const int32_t *fix_rec;  // HostPlan::fix_rec; NULL: sum through fix_off / fix_parts
    // [n_chunks+1] prefix of the complete-node counts: complete node k of chunk
    // c has solver-local index comp_off[c] + k, shared node s has
    // comp_off[n_chunks] + s (a permutation of all nodes; for a batch, of the
    // union of its problems).
    const int32_t *comp_off;
    const uint8_t *mask;
};

// nb = dim + 1 (linear simplices) or, in 2D, 6 (quadratic triangles: the
// three vertices, then the midpoints of edges (0,1), (1,2), (2,0); the volume
// check uses the vertices).
int build_host_plan(int dim, int nb, int64_t n_nodes, int64_t n_elems, const double *coords,
                    const int32_t *conn, const int32_t *dirichlet, int64_t n_dir, int chunk_elems,
                    HostPlan &P, std::string &err);

// Many independent meshes as one: every problem is chunked on its own (no
// chunk straddles two problems) and the index arrays are concatenated with
// node, element, chunk, shared-node and partial offsets.
struct BatchHost {
    HostPlan U;                           // union arrays (global ids)
    std::vector<int64_t> chunk_elem0;     // [n_chunks+1]
    std::vector<int64_t> node0, elem0;    // [P+1]
    std::vector<int32_t> chunk0, shared0; // [P+1]
    std::vector<int64_t> part0;           // [P+1]
    std::vector<int64_t> n_dir;           // [P] distinct Dirichlet nodes
    std::vector<int64_t> isolated_free;   // [P]
};

// coords: union SoA [dim][total nodes]; conn: union SoA [nb][total elems] with
// problem-local node ids; dirichlet: concatenated problem-local ids.
int build_batch_plan(int dim, int n_problems, const int64_t *node_off, const int64_t *elem_off,
                     const int64_t *dir_off, const double *coords, const int32_t *conn, const int32_t *dirichlet,
                     int chunk_elems, BatchHost &B, std::string &err);

}  // namespace fem
