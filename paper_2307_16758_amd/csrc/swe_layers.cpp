// Ghost layers built the way Sec. 3.2 of Delmas & Soulaimani describes for
// distributed memory (Fig. `mainalg`): every part works from its own cells
// only, exchanges a few numbers and its inner boundary layers with the parts
// that may touch it, and finds its ghosts by following the connectivity
// through what it received.  Here the parts are workers on host threads and
// the exchanges go through a shared board written in one phase and read in
// the next (the phase boundaries play the role of the collective steps):
//
//  A. each part gathers its cells (node ids, node coordinates, boundary
//     tags), matches its own edges, computes the bounding box of its nodes
//     and of its cell centroids, and builds its k inner boundary layers:
//     layer 1 = its cells with an edge not shared with another of its cells,
//     layer j + 1 = its cells across an edge from layer j;
//  B. every part reads all bounding boxes (the all-gather), keeps as
//     potential neighbours the parts whose node boxes meet its own (closed
//     boxes: touching counts), receives their inner layers, matches the
//     edges of its cells and the received ones, and takes as ghost layer j
//     the received cells j edges away from its own cells (j <= k); it posts,
//     per owner, the cells it receives and their layer;
//  C. every part reads what its potential neighbours asked of it (its send
//     lists) and numbers its cells exactly as swe_subdomain_build does.
//
// With layers narrower than the gap between parts that do not touch, the
// result equals the global breadth-first build.  Where a part lies within k
// layers of a part whose box does not meet its own (a thin part between
// them), the ghosts owned by that far part are missed, as the paper notes;
// the edges towards them then read as sub-domain cuts (SWE_BC_HALO).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <limits>
#include <system_error>
#include <thread>
#include <vector>

#include "swe_internal.h"

namespace {

struct Box { double lo_x, lo_y, hi_x, hi_y; };

// a cell as a part holds it or sends it: global id, nodes, their
// coordinates, the boundary tag of each edge (negative on the domain
// boundary, 0 inside)
struct CellRec {
    int32_t gid;
    int32_t node[3];
    double x[3], y[3];
    int8_t bc[3];
};

struct Request { int32_t gid, layer; };

struct Board {
    std::vector<Box> node_box, cen_box;                 // [P]
    std::vector<std::vector<CellRec>> layers;           // [P]: inner boundary layers
    std::vector<std::vector<std::vector<Request>>> req; // [P][P]: cells p receives from q
};

struct Part {
    std::vector<CellRec> own;           // sorted by gid
    std::vector<int32_t> potential;     // potential neighbours, ascending
    std::vector<CellRec> recv;          // received inner layers
    std::vector<int32_t> recv_owner;    // owner of each received cell
    // after B: union U = own ++ recv, its edge matching, ghost layers
    std::vector<int32_t> across;        // [3 |U|]: index in U across each edge, -1 none
    std::vector<int32_t> dist;          // [|U|]: 0 own, j ghost layer, -1 neither
    std::vector<uint32_t> key;          // [|U|]: Morton key (own and ghosts)
    int error = SWE_OK;
};

uint32_t spread16(uint32_t v)
{
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// centroid as the whole-mesh numbering computes it
void centroid(const CellRec &c, double &cx, double &cy)
{
    cx = ((c.x[0] + c.x[1]) + c.x[2]) / 3.0;
    cy = ((c.y[0] + c.y[1]) + c.y[2]) / 3.0;
}

// Edge matching over a list of cells by sorting their (min node, max node)
// keys: across[3 i + m] = the other cell of edge m of cell i, -1 if none;
// SWE_ERR_MESH for an edge of more than two cells.
int match_edges(const std::vector<const CellRec *> &cells, std::vector<int32_t> &across)
{
    struct HE { uint64_t key; int32_t cell; int8_t m; };
    std::vector<HE> he;
    he.reserve(3 * cells.size());
    for (size_t i = 0; i < cells.size(); ++i)
        for (int m = 0; m < 3; ++m) {
            const uint64_t p = (uint32_t)cells[i]->node[m], q = (uint32_t)cells[i]->node[(m + 1) % 3];
            he.push_back({(std::min(p, q) << 32) | std::max(p, q), (int32_t)i, (int8_t)m});
        }
    std::sort(he.begin(), he.end(), [](const HE &a, const HE &b) {
        return a.key != b.key ? a.key < b.key : a.cell < b.cell;
    });
    across.assign(3 * cells.size(), -1);
    for (size_t i = 0; i < he.size();) {
        size_t j = i + 1;
        while (j < he.size() && he[j].key == he[i].key) ++j;
        if (j - i > 2) return SWE_ERR_MESH;
        if (j - i == 2) {
            across[3 * (size_t)he[i].cell + he[i].m] = he[i + 1].cell;
            across[3 * (size_t)he[i + 1].cell + he[i + 1].m] = he[i].cell;
        }
        i = j;
    }
    return SWE_OK;
}

// fn(p) for every part on n_threads threads; SWE_ERR_OOM if an allocation
// failed in any of them
template <typename F>
int parallel_parts(int32_t P, int32_t n_threads, F fn)
{
    std::atomic<int32_t> next{0};
    std::atomic<int> status{SWE_OK};
    auto work = [&]() {
        for (int32_t p = next++; p < P; p = next++) {
            try {
                fn(p);
            } catch (const std::bad_alloc &) {
                status = SWE_ERR_OOM;
            }
        }
    };
    std::vector<std::thread> pool;
    try {
        for (int32_t t = 1; t < n_threads; ++t) pool.emplace_back(work);
    } catch (const std::system_error &) {
        // fewer threads than asked: the ones started and this one share the parts
    }
    work();
    for (auto &t : pool) t.join();
    return status.load();
}

// Phase A for part p: its cells, own edge matching, boxes, inner layers.
void phase_a(int32_t p, int32_t n, const double *xy, const int32_t *tri, const int8_t *bc,
             const int32_t *part, int32_t k, Part &W, Board &B)
{
    for (int32_t c = 0; c < n; ++c) {   // the cells this part is handed
        if (part[c] != p) continue;
        CellRec r;
        r.gid = c;
        for (int m = 0; m < 3; ++m) {
            r.node[m] = tri[3 * (size_t)c + m];
            r.x[m] = xy[2 * (size_t)r.node[m]];
            r.y[m] = xy[2 * (size_t)r.node[m] + 1];
            r.bc[m] = bc[3 * (size_t)c + m];
        }
        W.own.push_back(r);
    }
    const double inf = std::numeric_limits<double>::infinity();
    Box nb{inf, inf, -inf, -inf}, cb{inf, inf, -inf, -inf};
    for (const CellRec &r : W.own) {
        for (int m = 0; m < 3; ++m) {
            nb.lo_x = std::min(nb.lo_x, r.x[m]); nb.hi_x = std::max(nb.hi_x, r.x[m]);
            nb.lo_y = std::min(nb.lo_y, r.y[m]); nb.hi_y = std::max(nb.hi_y, r.y[m]);
        }
        double cx, cy;
        centroid(r, cx, cy);
        cb.lo_x = std::min(cb.lo_x, cx); cb.hi_x = std::max(cb.hi_x, cx);
        cb.lo_y = std::min(cb.lo_y, cy); cb.hi_y = std::max(cb.hi_y, cy);
    }
    B.node_box[p] = nb;
    B.cen_box[p] = cb;
    std::vector<const CellRec *> ptrs(W.own.size());
    for (size_t i = 0; i < W.own.size(); ++i) ptrs[i] = &W.own[i];
    std::vector<int32_t> across;
    if (match_edges(ptrs, across) != SWE_OK) { W.error = SWE_ERR_MESH; return; }
    // inner layers: breadth-first inwards from the cells on the part's rim
    std::vector<int32_t> depth(W.own.size(), 0), frontier;
    for (size_t i = 0; i < W.own.size(); ++i)
        for (int m = 0; m < 3; ++m)
            if (across[3 * i + m] < 0) { depth[i] = 1; frontier.push_back((int32_t)i); break; }
    for (int32_t d = 2; d <= k; ++d) {
        std::vector<int32_t> next;
        for (int32_t i : frontier)
            for (int m = 0; m < 3; ++m) {
                const int32_t j = across[3 * (size_t)i + m];
                if (j >= 0 && depth[j] == 0) { depth[j] = d; next.push_back(j); }
            }
        frontier.swap(next);
    }
    if (k > 0)
        for (size_t i = 0; i < W.own.size(); ++i)
            if (depth[i] > 0) B.layers[p].push_back(W.own[i]);
}

bool boxes_meet(const Box &a, const Box &b)
{
    return a.lo_x <= b.hi_x && b.lo_x <= a.hi_x && a.lo_y <= b.hi_y && b.lo_y <= a.hi_y;
}

// Phase B for part p: potential neighbours, received layers, ghost layers,
// Morton keys, requests to the owners.
void phase_b(int32_t p, int32_t P, int32_t k, Part &W, Board &B)
{
    if (W.error != SWE_OK) return;
    for (int32_t q = 0; q < P; ++q)
        if (q != p && !B.layers[q].empty() && boxes_meet(B.node_box[p], B.node_box[q]))
            W.potential.push_back(q);
    for (int32_t q : W.potential)
        for (const CellRec &r : B.layers[q]) {
            W.recv.push_back(r);
            W.recv_owner.push_back(q);
        }
    const size_t no = W.own.size(), nu = no + W.recv.size();
    std::vector<const CellRec *> U(nu);
    for (size_t i = 0; i < no; ++i) U[i] = &W.own[i];
    for (size_t i = 0; i < W.recv.size(); ++i) U[no + i] = &W.recv[i];
    if (match_edges(U, W.across) != SWE_OK) { W.error = SWE_ERR_MESH; return; }
    // ghost layers: breadth-first outwards from the own cells through the
    // received ones
    W.dist.assign(nu, -1);
    std::vector<int32_t> frontier;
    for (size_t i = 0; i < no; ++i) { W.dist[i] = 0; frontier.push_back((int32_t)i); }
    for (int32_t d = 1; d <= k; ++d) {
        std::vector<int32_t> next;
        for (int32_t i : frontier)
            for (int m = 0; m < 3; ++m) {
                const int32_t j = W.across[3 * (size_t)i + m];
                if (j >= 0 && W.dist[j] < 0) { W.dist[j] = d; next.push_back(j); }
            }
        frontier.swap(next);
    }
    // Morton keys over the box of all centroids (the union of the parts' boxes)
    Box cb = B.cen_box[0];
    for (int32_t q = 1; q < P; ++q) {
        cb.lo_x = std::min(cb.lo_x, B.cen_box[q].lo_x); cb.hi_x = std::max(cb.hi_x, B.cen_box[q].hi_x);
        cb.lo_y = std::min(cb.lo_y, B.cen_box[q].lo_y); cb.hi_y = std::max(cb.hi_y, B.cen_box[q].hi_y);
    }
    double S = std::max(cb.hi_x - cb.lo_x, cb.hi_y - cb.lo_y);
    if (!(S > 0.0)) S = 1.0;
    W.key.assign(nu, 0u);
    for (size_t i = 0; i < nu; ++i) {
        if (W.dist[i] < 0) continue;
        double cx, cy;
        centroid(*U[i], cx, cy);
        double qx = std::floor((cx - cb.lo_x) / S * 65536.0);
        double qy = std::floor((cy - cb.lo_y) / S * 65536.0);
        qx = std::min(std::max(qx, 0.0), 65535.0);
        qy = std::min(std::max(qy, 0.0), 65535.0);
        W.key[i] = spread16((uint32_t)qx) | (spread16((uint32_t)qy) << 1);
    }
    for (size_t i = no; i < nu; ++i)
        if (W.dist[i] > 0) B.req[p][W.recv_owner[i - no]].push_back({U[i]->gid, W.dist[i]});
}

// Phase C for part p: send lists from the requests of the potential
// neighbours, then the numbering of swe_subdomain_build.
swe_subdomain *phase_c(int32_t p, Part &W, Board &B)
{
    const size_t no = W.own.size(), nu = no + W.recv.size();
    auto gid = [&](size_t i) { return i < no ? W.own[i].gid : W.recv[i - no].gid; };
    auto owner = [&](size_t i) { return i < no ? p : W.recv_owner[i - no]; };
    auto *S = new swe_subdomain;
    std::vector<int32_t> ghosts;  // indices into U
    for (size_t i = no; i < nu; ++i)
        if (W.dist[i] > 0) ghosts.push_back((int32_t)i);
    for (int32_t i : ghosts) S->peers.push_back(owner(i));
    std::sort(S->peers.begin(), S->peers.end());
    S->peers.erase(std::unique(S->peers.begin(), S->peers.end()), S->peers.end());
    S->n_peers = (int32_t)S->peers.size();
    // own cells by global id (W.own is in ascending gid order)
    auto own_index = [&](int32_t g) -> int32_t {
        auto it = std::lower_bound(W.own.begin(), W.own.end(), g,
                                   [](const CellRec &r, int32_t v) { return r.gid < v; });
        return it != W.own.end() && it->gid == g ? (int32_t)(it - W.own.begin()) : -1;
    };
    std::vector<std::vector<std::pair<int32_t, int32_t>>> sends(S->n_peers);  // (own index, layer)
    std::vector<std::vector<int32_t>> dest(no);
    for (int32_t j = 0; j < S->n_peers; ++j) {
        const int32_t q = S->peers[j];
        for (const Request &r : B.req[q][p]) {
            const int32_t i = own_index(r.gid);
            if (i < 0) { W.error = SWE_ERR_MESH; delete S; return nullptr; }
            sends[j].push_back({i, r.layer});
            dest[i].push_back(q);  // peers visited ascending: tuple stays sorted
        }
    }
    auto by_key = [&](int32_t a, int32_t b) {
        return W.key[a] != W.key[b] ? W.key[a] < W.key[b] : gid(a) < gid(b);
    };
    std::vector<int32_t> send_cells, interior;
    for (size_t i = 0; i < no; ++i) (dest[i].empty() ? interior : send_cells).push_back((int32_t)i);
    std::sort(send_cells.begin(), send_cells.end(), [&](int32_t a, int32_t b) {
        if (dest[a] != dest[b])
            return std::lexicographical_compare(dest[a].begin(), dest[a].end(), dest[b].begin(),
                                                dest[b].end());
        return by_key(a, b);
    });
    std::sort(interior.begin(), interior.end(), by_key);
    std::sort(ghosts.begin(), ghosts.end(), [&](int32_t a, int32_t b) {
        if (owner(a) != owner(b)) return owner(a) < owner(b);
        if (W.dist[a] != W.dist[b]) return W.dist[a] < W.dist[b];
        return by_key(a, b);
    });
    std::vector<int32_t> order = send_cells;  // local numbering -> index into U
    order.insert(order.end(), interior.begin(), interior.end());
    S->n_owned = (int32_t)order.size();
    order.insert(order.end(), ghosts.begin(), ghosts.end());
    S->n_total = (int32_t)order.size();
    std::vector<int32_t> u2l(nu, -1);
    S->l2g.resize(S->n_total);
    S->layer.resize(S->n_total);
    S->owner.resize(S->n_total);
    for (int32_t l = 0; l < S->n_total; ++l) {
        const int32_t i = order[l];
        u2l[i] = l;
        S->l2g[l] = gid(i);
        S->layer[l] = l < S->n_owned ? 0 : W.dist[i];
        S->owner[l] = owner(i);
    }
    S->recv_off.assign(S->n_peers + 1, 0);
    for (int32_t l = S->n_owned; l < S->n_total; ++l) {
        const int32_t j = (int32_t)(std::lower_bound(S->peers.begin(), S->peers.end(), S->owner[l]) -
                                    S->peers.begin());
        S->recv_off[j + 1]++;
    }
    for (int32_t j = 0; j < S->n_peers; ++j) S->recv_off[j + 1] += S->recv_off[j];
    // neighbours: a matched cell of the sub-domain, else a cut (SWE_BC_HALO)
    // where the edge is not on the domain boundary, else its tag
    S->nbr.resize(3 * (size_t)S->n_total);
    for (int32_t l = 0; l < S->n_total; ++l) {
        const int32_t i = order[l];
        const CellRec &r = i < (int32_t)no ? W.own[i] : W.recv[i - no];
        for (int m = 0; m < 3; ++m) {
            const int32_t j = W.across[3 * (size_t)i + m];
            int32_t v;
            if (j >= 0 && u2l[j] >= 0) v = u2l[j];
            else if (r.bc[m] < 0) v = r.bc[m];
            else v = SWE_BC_HALO;
            S->nbr[3 * (size_t)l + m] = v;
        }
    }
    S->send_off.assign(S->n_peers + 1, 0);
    for (int32_t j = 0; j < S->n_peers; ++j) {
        auto &v = sends[j];
        std::sort(v.begin(), v.end(), [&](const std::pair<int32_t, int32_t> &a,
                                          const std::pair<int32_t, int32_t> &b) {
            if (a.second != b.second) return a.second < b.second;
            return by_key(a.first, b.first);
        });
        for (auto &e : v) S->send_idx.push_back(u2l[e.first]);
        S->send_off[j + 1] = (int32_t)S->send_idx.size();
    }
    S->n_send = (int32_t)S->send_idx.size();
    return S;
}

}  // namespace

extern "C" {

int swe_subdomain_build_layers(int32_t n_nodes, const double *xy, int32_t n, const int32_t *tri,
                               const int8_t *bc, const int32_t *part, int32_t P, int32_t k,
                               int32_t n_threads, swe_subdomain **out, int32_t *n_potential)
{
    if (!out || !xy || !tri || !bc || !part || P <= 0 || k < 0 || n <= 0 || n_nodes <= 0)
        return SWE_ERR_ARG;
    for (int32_t p = 0; p < P; ++p) out[p] = nullptr;
    for (int32_t c = 0; c < n; ++c) {
        if (part[c] < 0 || part[c] >= P) return SWE_ERR_ARG;
        for (int m = 0; m < 3; ++m)
            if (tri[3 * (size_t)c + m] < 0 || tri[3 * (size_t)c + m] >= n_nodes) return SWE_ERR_MESH;
    }
    if (n_threads <= 0) n_threads = (int32_t)std::max(1u, std::thread::hardware_concurrency());
    n_threads = std::min(n_threads, P);
    int status = SWE_OK;
    try {
        std::vector<Part> W(P);
        Board B;
        B.node_box.resize(P);
        B.cen_box.resize(P);
        B.layers.resize(P);
        B.req.assign(P, std::vector<std::vector<Request>>(P));
        status = parallel_parts(P, n_threads, [&](int32_t p) { phase_a(p, n, xy, tri, bc, part, k, W[p], B); });
        for (int32_t p = 0; p < P && status == SWE_OK; ++p) status = W[p].error;
        if (status == SWE_OK)
            status = parallel_parts(P, n_threads, [&](int32_t p) { phase_b(p, P, k, W[p], B); });
        for (int32_t p = 0; p < P && status == SWE_OK; ++p) status = W[p].error;
        if (status == SWE_OK)
            status = parallel_parts(P, n_threads, [&](int32_t p) { out[p] = phase_c(p, W[p], B); });
        for (int32_t p = 0; p < P && status == SWE_OK; ++p)
            if (!out[p]) status = W[p].error != SWE_OK ? W[p].error : SWE_ERR_MESH;
        if (n_potential)
            for (int32_t p = 0; p < P; ++p) n_potential[p] = (int32_t)W[p].potential.size();
    } catch (const std::bad_alloc &) {
        status = SWE_ERR_OOM;
    }
    if (status != SWE_OK)
        for (int32_t p = 0; p < P; ++p) {
            delete out[p];
            out[p] = nullptr;
        }
    return status;
}

}  // extern "C"
