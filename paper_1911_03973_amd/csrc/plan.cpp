// plan.cpp -- host construction of the chunked element -> node index.
//
// The paper replaces the Boolean restriction / assembly matrices R_e, C_e of
// eq. (3) and Algorithm 1 by index arrays (Section 2, the two index arrays
// after the residual listing).  On the GPU the assembly r = sum_e C_e^T r_e
// must be deterministic and free of floating-point atomics, so the element
// list is cut into chunks of consecutive elements, one workgroup pass each:
//
//   * every chunk lists the distinct nodes its elements touch ("local
//     nodes"): first the nodes touched by no other chunk ("complete"), then
//     the nodes shared with other chunks, each group in ascending node id;
//   * for every local node the chunk stores the list of its slots
//     (local element * n_b + local vertex) in ascending slot order, so the
//     in-chunk sum over a node's incident elements has a fixed order;
//   * the chunk's partial sum for a shared node goes to a partial slot; a
//     fix-up pass adds the partials of each shared node in ascending chunk
//     order.
//
// Everything here is plain host C++; the arrays are uploaded once.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

namespace fem {

namespace {

template <class F>
void parallel_for(int64_t n, F &&f) {
    unsigned hw = std::thread::hardware_concurrency();
    int nt = (int)std::min<int64_t>(n, std::max(1u, std::min(hw, 16u)));
    if (nt <= 1 || n < 64) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t) {
        th.emplace_back([&, t]() {
            int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
            for (int64_t i = lo; i < hi; ++i) f(i);
        });
    }
    for (auto &x : th) x.join();
}

}  // namespace

int build_host_plan(int dim, int nb, int64_t n_nodes, int64_t n_elems, const double *coords,
                    const int32_t *conn, const int32_t *dirichlet, int64_t n_dir, int chunk_elems,
                    HostPlan &P, std::string &err) {
    if (nb != dim + 1 && !(dim == 2 && nb == 6) && !(dim == 3 && nb == 10)) {
        err = "elements must be linear or quadratic simplices";
        return -1;
    }
    P = HostPlan();
    P.dim = dim;
    P.nb = nb;
    P.n_nodes = n_nodes;
    P.n_elems = n_elems;
    P.E = chunk_elems;
    P.n_chunks = (n_elems + chunk_elems - 1) / chunk_elems;

    // ---- validation: ids in range, distinct vertices, non-zero volume ----
    std::vector<int> bad(P.n_chunks, 0);
    parallel_for(P.n_chunks, [&](int64_t c) {
        int64_t e0 = c * chunk_elems, e1 = std::min<int64_t>(n_elems, e0 + chunk_elems);
        for (int64_t e = e0; e < e1 && !bad[c]; ++e) {
            int32_t v[10];
            for (int a = 0; a < nb; ++a) {
                v[a] = conn[(int64_t)a * n_elems + e];
                if (v[a] < 0 || v[a] >= n_nodes) { bad[c] = 1; break; }
            }
            if (bad[c]) break;
            for (int a = 0; a < nb; ++a)
                for (int b2 = a + 1; b2 < nb; ++b2)
                    if (v[a] == v[b2]) bad[c] = 2;
            if (bad[c]) break;
            double B[3][3];
            for (int r = 0; r < dim; ++r)
                for (int k = 0; k < dim; ++k)
                    B[r][k] = coords[(int64_t)r * n_nodes + v[k + 1]] - coords[(int64_t)r * n_nodes + v[0]];
            double det;
            if (dim == 2) det = B[0][0] * B[1][1] - B[0][1] * B[1][0];
            else
                det = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
                      B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                      B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
            if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) bad[c] = 3;
        }
    });
    for (int64_t c = 0; c < P.n_chunks; ++c) {
        if (bad[c] == 1) { err = "connectivity holds a node id outside [0, n_nodes)"; return -1; }
        if (bad[c] == 2) { err = "an element repeats a node"; return -1; }
        if (bad[c] == 3) { err = "an element has zero or non-finite volume"; return -1; }
    }
    P.mask.assign(n_nodes, 0);
    for (int64_t k = 0; k < n_dir; ++k) {
        if (dirichlet[k] < 0 || dirichlet[k] >= n_nodes) {
            err = "Dirichlet node id outside [0, n_nodes)";
            return -1;
        }
        P.mask[dirichlet[k]] = 1;
    }
    P.n_dirichlet = 0;
    for (int64_t i = 0; i < n_nodes; ++i) P.n_dirichlet += P.mask[i];

    // ---- pass 1: per chunk, sort (node, slot) pairs -> local nodes, slot runs ----
    std::vector<std::vector<int32_t>> cnodes(P.n_chunks);
    std::vector<std::vector<uint16_t>> cend(P.n_chunks);
    std::vector<std::vector<uint16_t>> cslots(P.n_chunks);
    parallel_for(P.n_chunks, [&](int64_t c) {
        int64_t e0 = c * chunk_elems, e1 = std::min<int64_t>(n_elems, e0 + chunk_elems);
        int ne = (int)(e1 - e0);
        std::vector<uint64_t> pairs((size_t)ne * nb);
        for (int le = 0; le < ne; ++le)
            for (int a = 0; a < nb; ++a) {
                uint64_t node = (uint64_t)(uint32_t)conn[(int64_t)a * n_elems + e0 + le];
                pairs[(size_t)le * nb + a] = (node << 16) | (uint64_t)(le * nb + a);
            }
        std::sort(pairs.begin(), pairs.end());
        auto &nodes = cnodes[c];
        auto &ends = cend[c];
        auto &sl = cslots[c];
        sl.resize(pairs.size());
        for (size_t k = 0; k < pairs.size(); ++k) {
            int32_t node = (int32_t)(pairs[k] >> 16);
            sl[k] = (uint16_t)(pairs[k] & 0xFFFF);
            if (nodes.empty() || nodes.back() != node) {
                if (!nodes.empty()) ends.push_back((uint16_t)k);
                nodes.push_back(node);
            }
        }
        ends.push_back((uint16_t)pairs.size());
    });

    // ---- chunk multiplicity of every node ----
    std::vector<int32_t> mult(n_nodes, 0);
    for (int64_t c = 0; c < P.n_chunks; ++c)
        for (int32_t g : cnodes[c]) mult[g]++;

    // ---- pass 2: order local nodes [complete..., shared...], keep slot runs ----
    P.chunk_node_off.assign(P.n_chunks + 1, 0);
    for (int64_t c = 0; c < P.n_chunks; ++c)
        P.chunk_node_off[c + 1] = P.chunk_node_off[c] + (int32_t)cnodes[c].size();
    P.n_local = P.chunk_node_off[P.n_chunks];
    P.loc_nodes.resize(P.n_local);
    P.loc_end.resize(P.n_local);
    P.slots.assign((size_t)P.n_chunks * nb * chunk_elems, 0);
    P.chunk_info.assign((size_t)P.n_chunks * 2, 0);
    std::vector<int32_t> nshared_c(P.n_chunks, 0);
    parallel_for(P.n_chunks, [&](int64_t c) {
        const auto &nodes = cnodes[c];
        const auto &ends = cend[c];
        const auto &sl = cslots[c];
        int nl = (int)nodes.size();
        std::vector<int> order;
        order.reserve(nl);
        for (int k = 0; k < nl; ++k)
            if (mult[nodes[k]] == 1) order.push_back(k);
        int ncomplete = (int)order.size();
        for (int k = 0; k < nl; ++k)
            if (mult[nodes[k]] > 1) order.push_back(k);
        int32_t base = P.chunk_node_off[c];
        uint16_t *dst = P.slots.data() + (size_t)c * nb * chunk_elems;
        int pos = 0;
        for (int t = 0; t < nl; ++t) {
            int k = order[t];
            int s0 = k ? ends[k - 1] : 0, s1 = ends[k];
            for (int s = s0; s < s1; ++s) dst[pos++] = sl[s];
            P.loc_nodes[base + t] = nodes[k];
            P.loc_end[base + t] = (uint16_t)pos;
        }
        P.chunk_info[2 * c] = ncomplete;
        nshared_c[c] = nl - ncomplete;
    });

    // ---- partial slots and the fix-up CSR (ascending chunk order per node) ----
    int64_t np = 0;
    for (int64_t c = 0; c < P.n_chunks; ++c) {
        P.chunk_info[2 * c + 1] = (int32_t)np;
        np += nshared_c[c];
    }
    P.n_partials = np;
    std::vector<int32_t> shared_index(n_nodes, -1);
    P.fix_nodes.clear();
    // Nodes touched by several chunks, and nodes touched by none (isolated:
    // their sum is empty, the fix-up still writes their output).
    for (int64_t g = 0; g < n_nodes; ++g)
        if (mult[g] != 1) {
            shared_index[g] = (int32_t)P.fix_nodes.size();
            P.fix_nodes.push_back((int32_t)g);
        }
    P.n_shared = (int64_t)P.fix_nodes.size();
    P.n_isolated = 0;
    P.n_isolated_free = 0;
    for (int64_t g = 0; g < n_nodes; ++g)
        if (mult[g] == 0) {
            P.n_isolated++;
            if (!P.mask[g]) P.n_isolated_free++;
        }
    P.fix_off.assign(P.n_shared + 1, 0);
    for (int64_t s = 0; s < P.n_shared; ++s) P.fix_off[s + 1] = P.fix_off[s] + mult[P.fix_nodes[s]];
    P.fix_parts.assign(np, 0);
    std::vector<int32_t> fill(P.n_shared, 0);
    for (int64_t c = 0; c < P.n_chunks; ++c) {
        int32_t base = P.chunk_node_off[c];
        int ncomp = P.chunk_info[2 * c];
        int nl = (int)cnodes[c].size();
        for (int t = ncomp; t < nl; ++t) {
            int32_t s = shared_index[P.loc_nodes[base + t]];
            P.fix_parts[P.fix_off[s] + fill[s]++] = P.chunk_info[2 * c + 1] + (t - ncomp);
        }
    }
    P.fix_rec.assign((size_t)4 * P.n_shared, -1);
    for (int64_t s = 0; s < P.n_shared; ++s) {
        const int32_t k0 = P.fix_off[s], cnt = P.fix_off[s + 1] - k0;
        for (int i = 0; i < std::min(cnt, 4); ++i) P.fix_rec[4 * s + i] = P.fix_parts[k0 + i];
        if (cnt > 4) P.fix_rec[4 * s + 3] = -2 - (k0 + 3);
    }
    P.part_owner.assign(np, 0);
    for (int64_t s = 0; s < P.n_shared; ++s)
        for (int32_t k = P.fix_off[s]; k < P.fix_off[s + 1]; ++k) P.part_owner[P.fix_parts[k]] = (int32_t)s;
    P.comp_off.assign(P.n_chunks + 1, 0);
    for (int64_t c = 0; c < P.n_chunks; ++c) P.comp_off[c + 1] = P.comp_off[c] + P.chunk_info[2 * c];
    if ((int64_t)P.comp_off[P.n_chunks] + P.n_shared != n_nodes) {
        err = "internal error: complete and shared nodes do not partition the nodes";
        return -1;
    }
    return 0;
}

int build_batch_plan(int dim, int n_problems, const int64_t *node_off, const int64_t *elem_off,
                     const int64_t *dir_off, const double *coords, const int32_t *conn, const int32_t *dirichlet,
                     int chunk_elems, BatchHost &B, std::string &err) {
    const int nb = dim + 1;
    const int64_t NN = node_off[n_problems], NE = elem_off[n_problems];
    std::vector<HostPlan> parts(n_problems);
    std::vector<std::string> errs(n_problems);
    std::vector<int> rcs(n_problems, 0);
    parallel_for(n_problems, [&](int64_t p) {
        const int64_t nn = node_off[p + 1] - node_off[p], ne = elem_off[p + 1] - elem_off[p];
        std::vector<double> lc((size_t)dim * nn);
        for (int r = 0; r < dim; ++r)
            for (int64_t i = 0; i < nn; ++i) lc[(size_t)r * nn + i] = coords[(size_t)r * NN + node_off[p] + i];
        std::vector<int32_t> le((size_t)nb * ne);
        for (int a = 0; a < nb; ++a)
            for (int64_t e = 0; e < ne; ++e) le[(size_t)a * ne + e] = conn[(size_t)a * NE + elem_off[p] + e];
        rcs[p] = build_host_plan(dim, dim + 1, nn, ne, lc.data(), le.data(), dirichlet + dir_off[p], dir_off[p + 1] - dir_off[p],
                                 chunk_elems, parts[p], errs[p]);
    });
    for (int p = 0; p < n_problems; ++p)
        if (rcs[p]) {
            err = "problem " + std::to_string(p) + ": " + errs[p];
            return -1;
        }
    HostPlan &U = B.U;
    U = HostPlan();
    U.dim = dim;
    U.nb = nb;
    U.E = chunk_elems;
    U.n_nodes = NN;
    U.n_elems = NE;
    B.node0.assign(node_off, node_off + n_problems + 1);
    B.elem0.assign(elem_off, elem_off + n_problems + 1);
    B.chunk0.assign(n_problems + 1, 0);
    B.shared0.assign(n_problems + 1, 0);
    B.part0.assign(n_problems + 1, 0);
    B.n_dir.assign(n_problems, 0);
    B.isolated_free.assign(n_problems, 0);
    for (int p = 0; p < n_problems; ++p) {
        B.chunk0[p + 1] = B.chunk0[p] + (int32_t)parts[p].n_chunks;
        B.shared0[p + 1] = B.shared0[p] + (int32_t)parts[p].n_shared;
        B.part0[p + 1] = B.part0[p] + parts[p].n_partials;
        B.n_dir[p] = parts[p].n_dirichlet;
        B.isolated_free[p] = parts[p].n_isolated_free;
    }
    U.n_chunks = B.chunk0[n_problems];
    U.n_shared = B.shared0[n_problems];
    U.n_partials = B.part0[n_problems];
    U.chunk_node_off.assign(U.n_chunks + 1, 0);
    U.chunk_info.assign((size_t)U.n_chunks * 2, 0);
    U.slots.assign((size_t)U.n_chunks * nb * chunk_elems, 0);
    U.fix_off.assign(U.n_shared + 1, 0);
    U.fix_nodes.resize(U.n_shared);
    U.fix_parts.resize(U.n_partials);
    U.part_owner.resize(U.n_partials);
    U.mask.resize(NN);
    B.chunk_elem0.assign(U.n_chunks + 1, 0);
    int64_t nloc = 0;
    std::vector<int64_t> loc0(n_problems + 1, 0);
    for (int p = 0; p < n_problems; ++p) loc0[p + 1] = loc0[p] + parts[p].n_local;
    U.n_local = loc0[n_problems];
    U.loc_nodes.resize(U.n_local);
    U.loc_end.resize(U.n_local);
    parallel_for(n_problems, [&](int64_t p) {
        const HostPlan &H = parts[p];
        const int32_t c0 = B.chunk0[p];
        for (int64_t c = 0; c < H.n_chunks; ++c) {
            U.chunk_node_off[c0 + c] = (int32_t)(loc0[p] + H.chunk_node_off[c]);
            U.chunk_info[2 * (c0 + c)] = H.chunk_info[2 * c];
            U.chunk_info[2 * (c0 + c) + 1] = (int32_t)(B.part0[p] + H.chunk_info[2 * c + 1]);
            B.chunk_elem0[c0 + c] = elem_off[p] + c * chunk_elems;
        }
        std::copy(H.slots.begin(), H.slots.end(), U.slots.begin() + (size_t)c0 * nb * chunk_elems);
        for (int64_t k = 0; k < H.n_local; ++k) {
            U.loc_nodes[loc0[p] + k] = (int32_t)(node_off[p] + H.loc_nodes[k]);
            U.loc_end[loc0[p] + k] = H.loc_end[k];
        }
        const int32_t s0 = B.shared0[p];
        for (int64_t k = 0; k < H.n_shared; ++k) {
            U.fix_nodes[s0 + k] = (int32_t)(node_off[p] + H.fix_nodes[k]);
            U.fix_off[s0 + k] = (int32_t)(B.part0[p] + H.fix_off[k]);
        }
        for (int64_t k = 0; k < H.n_partials; ++k) {
            U.fix_parts[B.part0[p] + k] = (int32_t)(B.part0[p] + H.fix_parts[k]);
            U.part_owner[B.part0[p] + k] = s0 + H.part_owner[k];
        }
        std::copy(H.mask.begin(), H.mask.end(), U.mask.begin() + node_off[p]);
    });
    U.chunk_node_off[U.n_chunks] = (int32_t)U.n_local;
    U.fix_off[U.n_shared] = (int32_t)U.n_partials;
    U.comp_off.assign(U.n_chunks + 1, 0);
    for (int64_t c = 0; c < U.n_chunks; ++c) U.comp_off[c + 1] = U.comp_off[c] + U.chunk_info[2 * c];
    if ((int64_t)U.comp_off[U.n_chunks] + U.n_shared != NN) {
        err = "internal error: complete and shared nodes do not partition the nodes";
        return -1;
    }
    B.chunk_elem0[U.n_chunks] = NE;
    (void)nloc;
    U.n_dirichlet = 0;
    for (int64_t i = 0; i < NN; ++i) U.n_dirichlet += U.mask[i];
    return 0;
}

}  // namespace fem
