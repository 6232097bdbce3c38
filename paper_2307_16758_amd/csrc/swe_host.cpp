// Host mesh toolkit of libswe.so (CPU): dual graph, greedy breadth-first
// partition, Morton keys, k-layer ghost sub-domains with in-place receive
// numbering (Delmas & Soulaimani, Sec. 3.1 - 3.3), and the per-cell /
// per-half-edge geometry the device kernels read (Sec. 6.1).
//
// Built with -ffp-contract=off so that the Morton quantisation and the
// geometry are the plain double-precision expressions written here.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <numeric>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "swe_internal.h"

namespace {

// Dual graph by sorting the 3n half-edges on their (min node, max node) key.
int dual_graph(int32_t n_nodes, int32_t n, const int32_t *tri, int32_t *nbr)
{
    struct HalfEdge { uint64_t key; int32_t cell; int8_t m; int8_t fwd; };
    std::vector<HalfEdge> he(3 * (size_t)n);
    for (int32_t c = 0; c < n; ++c)
        for (int m = 0; m < 3; ++m) {
            int32_t p = tri[3 * c + m], q = tri[3 * c + (m + 1) % 3];
            if (p < 0 || q < 0 || p >= n_nodes || q >= n_nodes || p == q) return SWE_ERR_MESH;
            uint64_t lo = std::min(p, q), hi = std::max(p, q);
            he[3 * (size_t)c + m] = {lo * (uint64_t)n_nodes + hi, c, (int8_t)m, (int8_t)(p < q)};
        }
    std::sort(he.begin(), he.end(), [](const HalfEdge &a, const HalfEdge &b) {
        return a.key != b.key ? a.key < b.key : a.cell < b.cell;
    });
    for (size_t i = 0; i < he.size();) {
        size_t j = i + 1;
        while (j < he.size() && he[j].key == he[i].key) ++j;
        if (j - i == 1) {
            nbr[3 * (size_t)he[i].cell + he[i].m] = -1;
        } else if (j - i == 2 && he[i].fwd != he[i + 1].fwd) {
            nbr[3 * (size_t)he[i].cell + he[i].m] = he[i + 1].cell;
            nbr[3 * (size_t)he[i + 1].cell + he[i + 1].m] = he[i].cell;
        } else {
            return SWE_ERR_MESH;  // non-manifold edge or inconsistent orientation
        }
        i = j;
    }
    return SWE_OK;
}

uint32_t spread16(uint32_t v)
{
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

void morton(int32_t n, const double *xy, const int32_t *tri, std::vector<uint32_t> &key)
{
    std::vector<double> cx(n), cy(n);
    double lo_x = std::numeric_limits<double>::infinity(), lo_y = lo_x;
    double hi_x = -lo_x, hi_y = -lo_x;
    for (int32_t c = 0; c < n; ++c) {
        const int32_t *t = tri + 3 * (size_t)c;
        cx[c] = ((xy[2 * t[0]] + xy[2 * t[1]]) + xy[2 * t[2]]) / 3.0;
        cy[c] = ((xy[2 * t[0] + 1] + xy[2 * t[1] + 1]) + xy[2 * t[2] + 1]) / 3.0;
        lo_x = std::min(lo_x, cx[c]); hi_x = std::max(hi_x, cx[c]);
        lo_y = std::min(lo_y, cy[c]); hi_y = std::max(hi_y, cy[c]);
    }
    double S = std::max(hi_x - lo_x, hi_y - lo_y);
    if (!(S > 0.0)) S = 1.0;
    key.resize(n);
    for (int32_t c = 0; c < n; ++c) {
        double qx = std::floor((cx[c] - lo_x) / S * 65536.0);
        double qy = std::floor((cy[c] - lo_y) / S * 65536.0);
        qx = std::min(std::max(qx, 0.0), 65535.0);
        qy = std::min(std::max(qy, 0.0), 65535.0);
        key[c] = spread16((uint32_t)qx) | (spread16((uint32_t)qy) << 1);
    }
}

}  // namespace

extern "C" {

int swe_dual_graph(int32_t n_nodes, int32_t n_cells, const int32_t *cell_nodes, int32_t *nbr)
{
    if (n_nodes < 0 || n_cells < 0 || (n_cells > 0 && (!cell_nodes || !nbr))) return SWE_ERR_ARG;
    return dual_graph(n_nodes, n_cells, cell_nodes, nbr);
}

int swe_partition_bfs(int32_t n, const int32_t *nbr, int32_t P, int32_t *part)
{
    if (n < 0 || P <= 0 || (n > 0 && (!nbr || !part))) return SWE_ERR_ARG;
    std::fill(part, part + n, -1);
    std::vector<int32_t> fifo;
    fifo.reserve(n);
    int32_t next_seed = 0;
    for (int32_t p = 0; p < P; ++p) {
        const int64_t quota = n / P + (p < n % P ? 1 : 0);
        int64_t have = 0;
        fifo.clear();
        size_t head = 0;
        while (have < quota) {
            if (head == fifo.size()) {  // (re)seed at the lowest free id
                while (next_seed < n && part[next_seed] != -1) ++next_seed;
                if (next_seed == n) break;
                part[next_seed] = p;
                fifo.push_back(next_seed);
                ++have;
                continue;
            }
            const int32_t c = fifo[head++];
            for (int m = 0; m < 3 && have < quota; ++m) {
                const int32_t d = nbr[3 * (size_t)c + m];
                if (d < 0 || part[d] != -1) continue;
                part[d] = p;
                fifo.push_back(d);
                ++have;
            }
        }
    }
    return SWE_OK;
}

int swe_edge_length_sum(int32_t n_nodes, const double *xy, int32_t n, const int32_t *tri,
                        const int8_t *bc, int32_t tag, double *out)
{
    if (n_nodes <= 0 || n < 0 || !xy || !out || (n > 0 && (!tri || !bc))) return SWE_ERR_ARG;
    double sum = 0.0;
    for (int32_t c = 0; c < n; ++c)
        for (int m = 0; m < 3; ++m) {
            if (bc[3 * (size_t)c + m] != tag) continue;
            const int32_t a = tri[3 * (size_t)c + m], b = tri[3 * (size_t)c + (m + 1) % 3];
            if (a < 0 || b < 0 || a >= n_nodes || b >= n_nodes) return SWE_ERR_MESH;
            const double dx = xy[2 * b] - xy[2 * a], dy = xy[2 * b + 1] - xy[2 * a + 1];
            sum += std::sqrt(dx * dx + dy * dy);
        }
    *out = sum;
    return SWE_OK;
}

int swe_morton_keys(int32_t n_nodes, const double *xy, int32_t n, const int32_t *tri,
                    uint32_t *key)
{
    if (n_nodes <= 0 || n < 0 || !xy || (n > 0 && (!tri || !key))) return SWE_ERR_ARG;
    std::vector<uint32_t> k;
    morton(n, xy, tri, k);
    std::copy(k.begin(), k.end(), key);
    return SWE_OK;
}

int swe_subdomain_build(int32_t n_nodes, const double *xy, int32_t n, const int32_t *tri,
                        const int32_t *nbr, const int8_t *bc, const int32_t *part, int32_t P,
                        int32_t p, int32_t k, swe_subdomain **out)
{
    if (!out || !xy || !tri || !nbr || !bc || !part || P <= 0 || p < 0 || p >= P || k < 0 ||
        n <= 0 || n_nodes <= 0)
        return SWE_ERR_ARG;
    *out = nullptr;
    std::vector<uint32_t> key;
    morton(n, xy, tri, key);

    // Cells of every part that touch another part: the sources of the
    // distance searches (a shortest path into a part leaves through them).
    std::vector<std::vector<int32_t>> rim(P);
    for (int32_t c = 0; c < n; ++c) {
        if (part[c] < 0 || part[c] >= P) return SWE_ERR_ARG;
        for (int m = 0; m < 3; ++m) {
            int32_t d = nbr[3 * (size_t)c + m];
            if (d >= 0 && part[d] != part[c]) { rim[part[c]].push_back(c); break; }
        }
    }
    // distance (<= k) of cells outside part q to part q, by BFS from q's rim
    std::vector<int32_t> dist(n, -1);
    auto layers_of = [&](int32_t q, std::vector<int32_t> &reached) {
        reached.clear();
        for (int32_t c : rim[q]) { dist[c] = 0; reached.push_back(c); }
        size_t lo = 0;
        for (int32_t d = 1; d <= k; ++d) {
            size_t hi = reached.size();
            for (size_t i = lo; i < hi; ++i) {
                const int32_t c = reached[i];
                for (int m = 0; m < 3; ++m) {
                    const int32_t e = nbr[3 * (size_t)c + m];
                    if (e >= 0 && dist[e] < 0 && part[e] != q) { dist[e] = d; reached.push_back(e); }
                }
            }
            lo = hi;
        }
    };
    auto clear = [&](const std::vector<int32_t> &reached) { for (int32_t c : reached) dist[c] = -1; };

    auto *S = new swe_subdomain;
    std::vector<int32_t> reached;
    // ghosts of p, with their layer
    layers_of(p, reached);
    std::vector<int32_t> ghosts;
    std::vector<int32_t> glayer_of;  // parallel to ghosts
    for (int32_t c : reached)
        if (dist[c] > 0) { ghosts.push_back(c); glayer_of.push_back(dist[c]); }
    std::vector<int32_t> gl(n, 0);
    for (size_t i = 0; i < ghosts.size(); ++i) gl[ghosts[i]] = glayer_of[i];
    clear(reached);
    for (int32_t c : ghosts) S->peers.push_back(part[c]);
    std::sort(S->peers.begin(), S->peers.end());
    S->peers.erase(std::unique(S->peers.begin(), S->peers.end()), S->peers.end());
    S->n_peers = (int32_t)S->peers.size();

    // send sets: cells of p within distance k of q, with that distance
    std::vector<std::vector<std::pair<int32_t, int32_t>>> sends(S->n_peers);
    std::vector<int32_t> slot(n, -1);  // index of p's cells in dest
    int32_t n_mine = 0;
    for (int32_t c = 0; c < n; ++c)
        if (part[c] == p) slot[c] = n_mine++;
    std::vector<std::vector<int32_t>> dest(n_mine);
    for (int32_t j = 0; j < S->n_peers; ++j) {
        const int32_t q = S->peers[j];
        layers_of(q, reached);
        for (int32_t c : reached)
            if (dist[c] > 0 && part[c] == p) {
                sends[j].push_back({c, dist[c]});
                dest[slot[c]].push_back(q);  // peers visited ascending: tuple stays sorted
            }
        clear(reached);
    }
    // owned ordering
    std::vector<int32_t> send_cells, interior;
    for (int32_t c = 0; c < n; ++c)
        if (part[c] == p) (dest[slot[c]].empty() ? interior : send_cells).push_back(c);
    auto by_key = [&](int32_t a, int32_t b) { return key[a] != key[b] ? key[a] < key[b] : a < b; };
    std::sort(send_cells.begin(), send_cells.end(), [&](int32_t a, int32_t b) {
        const auto &da = dest[slot[a]], &db = dest[slot[b]];
        if (da != db)
            return std::lexicographical_compare(da.begin(), da.end(), db.begin(), db.end());
        return by_key(a, b);
    });
    std::sort(interior.begin(), interior.end(), by_key);
    std::sort(ghosts.begin(), ghosts.end(), [&](int32_t a, int32_t b) {
        if (part[a] != part[b]) return part[a] < part[b];
        if (gl[a] != gl[b]) return gl[a] < gl[b];
        return by_key(a, b);
    });
    S->l2g = send_cells;
    S->l2g.insert(S->l2g.end(), interior.begin(), interior.end());
    S->n_owned = (int32_t)S->l2g.size();
    S->l2g.insert(S->l2g.end(), ghosts.begin(), ghosts.end());
    S->n_total = (int32_t)S->l2g.size();
    std::vector<int32_t> g2l(n, -1);
    S->layer.resize(S->n_total);
    S->owner.resize(S->n_total);
    for (int32_t i = 0; i < S->n_total; ++i) {
        const int32_t c = S->l2g[i];
        g2l[c] = i;
        S->layer[i] = i < S->n_owned ? 0 : gl[c];
        S->owner[i] = part[c];
    }
    S->recv_off.assign(S->n_peers + 1, 0);
    for (int32_t i = S->n_owned; i < S->n_total; ++i) {
        const int32_t j = (int32_t)(std::lower_bound(S->peers.begin(), S->peers.end(),
                                                     part[S->l2g[i]]) - S->peers.begin());
        S->recv_off[j + 1]++;
    }
    for (int32_t j = 0; j < S->n_peers; ++j) S->recv_off[j + 1] += S->recv_off[j];
    S->nbr.resize(3 * (size_t)S->n_total);
    for (int32_t i = 0; i < S->n_total; ++i)
        for (int m = 0; m < 3; ++m) {
            const int32_t c = S->l2g[i], d = nbr[3 * (size_t)c + m];
            int32_t v;
            if (d >= 0) v = g2l[d] >= 0 ? g2l[d] : SWE_BC_HALO;
            else v = bc[3 * (size_t)c + m] < 0 ? bc[3 * (size_t)c + m] : SWE_BC_WALL;
            S->nbr[3 * (size_t)i + m] = v;
        }
    S->send_off.assign(S->n_peers + 1, 0);
    for (int32_t j = 0; j < S->n_peers; ++j) {
        auto &v = sends[j];
        std::sort(v.begin(), v.end(), [&](const std::pair<int32_t, int32_t> &a,
                                          const std::pair<int32_t, int32_t> &b) {
            if (a.second != b.second) return a.second < b.second;
            return by_key(a.first, b.first);
        });
        for (auto &e : v) S->send_idx.push_back(g2l[e.first]);
        S->send_off[j + 1] = (int32_t)S->send_idx.size();
    }
    S->n_send = (int32_t)S->send_idx.size();
    *out = S;
    return SWE_OK;
}

int swe_subdomain_build_all(int32_t n_nodes, const double *xy, int32_t n, const int32_t *tri,
                            const int32_t *nbr, const int8_t *bc, const int32_t *part, int32_t P,
                            int32_t k, int32_t n_threads, swe_subdomain **out)
{
    if (!out || P <= 0) return SWE_ERR_ARG;
    for (int32_t p = 0; p < P; ++p) out[p] = nullptr;
    if (n_threads <= 0) n_threads = (int32_t)std::max(1u, std::thread::hardware_concurrency());
    n_threads = std::min(n_threads, P);
    // parts are independent given the dual graph and the partition: each
    // worker claims the next part and builds it exactly as a single call does
    std::atomic<int32_t> next{0};
    std::atomic<int> status{SWE_OK};
    auto work = [&]() {
        for (int32_t p = next++; p < P && status.load() == SWE_OK; p = next++) {
            int rc;
            try {
                rc = swe_subdomain_build(n_nodes, xy, n, tri, nbr, bc, part, P, p, k, &out[p]);
            } catch (const std::bad_alloc &) {
                rc = SWE_ERR_OOM;
            }
            if (rc != SWE_OK) {
                int ok = SWE_OK;
                status.compare_exchange_strong(ok, rc);
            }
        }
    };
    std::vector<std::thread> pool;
    try {
        for (int32_t t = 1; t < n_threads; ++t) pool.emplace_back(work);
    } catch (const std::system_error &) {
        // fewer threads than asked: the ones started and this one finish the parts
    }
    work();
    for (auto &t : pool) t.join();
    if (status.load() != SWE_OK) {
        for (int32_t p = 0; p < P; ++p) {
            delete out[p];
            out[p] = nullptr;
        }
        return status.load();
    }
    return SWE_OK;
}

int swe_subdomain_view_get(const swe_subdomain *sd, swe_subdomain_view *v)
{
    if (!sd || !v) return SWE_ERR_ARG;
    v->n_owned = sd->n_owned; v->n_total = sd->n_total;
    v->n_peers = sd->n_peers; v->n_send = sd->n_send;
    v->l2g = sd->l2g.data(); v->layer = sd->layer.data(); v->owner = sd->owner.data();
    v->nbr = sd->nbr.data(); v->peers = sd->peers.data(); v->recv_off = sd->recv_off.data();
    v->send_off = sd->send_off.data(); v->send_idx = sd->send_idx.data();
    return SWE_OK;
}

void swe_subdomain_free(swe_subdomain *sd) { delete sd; }

}  // extern "C"

namespace swe {

// Geometry of Sec. 6.1 in double precision, plus the MUSCL distances of
// Sec. 6.2.3 (|x_RL - x_L| to the edge midpoint, |x_L - x_Lupw| to the mean
// of the upwind centroids, |x_R - x_L| across the edge, |x_R - x_Lupw| for the
// central slope) for every half-edge.
int prepare_geometry(const swe_mesh &M, int scenario, HostGeometry &g, std::string &msg)
{
    const int32_t n = M.n_total;
    if (n <= 0 || M.n_owned < 0 || M.n_owned > n || M.n_nodes <= 0 || !M.node_xy ||
        !M.cell_nodes || !M.cell_gid || !M.cell_nbr || !M.cell_b || !M.cell_manning) {
        msg = "mesh: missing array or bad size";
        return SWE_ERR_MESH;
    }
    if (scenario < 0 || scenario >= kMaxScenarios) { msg = "scenario index"; return SWE_ERR_ARG; }
    g.cell.assign(4 * (size_t)n, 0.0);
    g.he_geo.assign(12 * (size_t)n, 0.0);
    g.he_dist.assign(12 * (size_t)n, 0.0);
    g.nbr4.assign(4 * (size_t)n, 0);
    g.inflow_length = 0.0;
    std::vector<double> cx(n), cy(n);
    const double *xy = M.node_xy;
    for (int32_t c = 0; c < n; ++c) {
        const int32_t *t = M.cell_nodes + 3 * (size_t)c;
        for (int i = 0; i < 3; ++i)
            if (t[i] < 0 || t[i] >= M.n_nodes) { msg = "mesh: node index out of range"; return SWE_ERR_MESH; }
        const double x0 = xy[2 * t[0]], y0 = xy[2 * t[0] + 1], x1 = xy[2 * t[1]],
                     y1 = xy[2 * t[1] + 1], x2 = xy[2 * t[2]], y2 = xy[2 * t[2] + 1];
        const double twice = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
        if (!(twice > 0.0)) { msg = "mesh: cell " + std::to_string(c) + " is not counter-clockwise"; return SWE_ERR_MESH; }
        cx[c] = ((x0 + x1) + x2) / 3.0;
        cy[c] = ((y0 + y1) + y2) / 3.0;
        const double man = M.cell_manning[c];
        if (!(man >= 0.0) || !std::isfinite(M.cell_b[c])) { msg = "mesh: bad bed or Manning value"; return SWE_ERR_MESH; }
        double perim = 0.0;
        for (int m = 0; m < 3; ++m) {
            const int32_t a = t[m], b = t[(m + 1) % 3];
            const double dx = xy[2 * b] - xy[2 * a], dy = xy[2 * b + 1] - xy[2 * a + 1];
            const double L = std::sqrt(dx * dx + dy * dy);
            double *ge = &g.he_geo[12 * (size_t)c + 4 * m];
            ge[0] = dy / L;
            ge[1] = -dx / L;
            ge[2] = L;
            perim += L;
        }
        g.cell[4 * (size_t)c + 0] = 2.0 / twice;
        g.cell[4 * (size_t)c + 1] = twice / perim;
        g.cell[4 * (size_t)c + 2] = man * man;
    }
    for (int32_t c = 0; c < n; ++c) {
        const int32_t *t = M.cell_nodes + 3 * (size_t)c;
        const int32_t *nb = M.cell_nbr + 3 * (size_t)c;
        uint32_t word = (uint32_t)scenario << kScenShift;
        if (c < M.n_owned) word |= 1u << kOwnedBit;
        for (int m = 0; m < 3; ++m) {
            const int32_t k = nb[m];
            g.nbr4[4 * (size_t)c + m] = k;
            double *ge = &g.he_geo[12 * (size_t)c + 4 * m];
            double *gd = &g.he_dist[12 * (size_t)c + 4 * m];
            const int32_t a = t[m], b = t[(m + 1) % 3];
            const double mx = 0.5 * (xy[2 * a] + xy[2 * b]), my = 0.5 * (xy[2 * a + 1] + xy[2 * b + 1]);
            ge[3] = std::hypot(mx - cx[c], my - cy[c]);
            if (k < 0) {
                if (k < SWE_BC_HALO) { msg = "mesh: unknown boundary tag"; return SWE_ERR_MESH; }
                if (k == SWE_BC_INFLOW && c < M.n_owned) g.inflow_length += ge[2];
                continue;
            }
            if (k >= n) { msg = "mesh: neighbour index out of range"; return SWE_ERR_MESH; }
            int back = -1;
            for (int j = 0; j < 3; ++j)
                if (M.cell_nbr[3 * (size_t)k + j] == c) back = j;
            if (back < 0) { msg = "mesh: neighbour table not symmetric at cell " + std::to_string(c); return SWE_ERR_MESH; }
            const int32_t *tk = M.cell_nodes + 3 * (size_t)k;
            if (!(tk[back] == b && tk[(back + 1) % 3] == a)) { msg = "mesh: neighbours do not share the edge"; return SWE_ERR_MESH; }
            if (M.cell_gid[c] == M.cell_gid[k]) { msg = "mesh: duplicate global id"; return SWE_ERR_MESH; }
            word |= (uint32_t)back << (2 * m);
            if (M.cell_gid[c] < M.cell_gid[k]) word |= 1u << (6 + m);
            const double df = std::hypot(cx[k] - cx[c], cy[k] - cy[c]);
            const int32_t ua = nb[(m + 1) % 3], ub = nb[(m + 2) % 3];
            if ((ua >= n) || (ub >= n)) { msg = "mesh: neighbour index out of range"; return SWE_ERR_MESH; }
            double ux = 0.0, uy = 0.0;
            bool up = true;
            if (ua >= 0 && ub >= 0) { ux = 0.5 * (cx[ua] + cx[ub]); uy = 0.5 * (cy[ua] + cy[ub]); }
            else if (ua >= 0) { ux = cx[ua]; uy = cy[ua]; }
            else if (ub >= 0) { ux = cx[ub]; uy = cy[ub]; }
            else up = false;
            gd[0] = up ? 1.0 / std::hypot(cx[c] - ux, cy[c] - uy) : 0.0;
            gd[1] = 1.0 / df;
            gd[2] = up ? 1.0 / std::hypot(cx[k] - ux, cy[k] - uy) : 0.0;
            gd[3] = df;
        }
        g.nbr4[4 * (size_t)c + 3] = (int32_t)word;
    }
    return SWE_OK;
}

}  // namespace swe
