/*
 * decomp_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Serial reference for the mesh-side machinery of one sub-domain with k
 * layers of ghost cells (Delmas & Soulaimani, Sec. 3.1 - 3.3): dual graph,
 * a greedy breadth-first partition standing in for ParMETIS, ghost layers by
 * following the connectivity, and the renumbering that makes every receive
 * contiguous.  Loaded only by the tests, the smoke check and the CPU-baseline
 * leg of the benchmark; shares no code with the library.
 * Not thread-safe (qsort comparators read file-scope keys).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { BC_HALO = -5 };

/* ------------------------------------------------------------------------
 * Dual graph (Sec. 3.1): two cells are adjacent when they share an edge.
 * Every node keeps the list of its cells; the cell across local edge m of c
 * (nodes p = tri[m], q = tri[m+1]) is the other cell incident to both p and
 * q.  Returns -1 where none, and an error (-2) for an edge shared by more than
 * two cells or traversed in the same direction by both (inconsistent
 * orientation).
 * ---------------------------------------------------------------------- */
int od_neighbors(int nn, int nc, const int *tri, int *nbr)
{
    int *cnt = calloc((size_t)nn + 1, sizeof(int));
    for (int i = 0; i < 3 * nc; ++i) cnt[tri[i] + 1]++;
    for (int i = 0; i < nn; ++i) cnt[i + 1] += cnt[i];
    int *pos = malloc(sizeof(int) * ((size_t)nn + 1));
    memcpy(pos, cnt, sizeof(int) * ((size_t)nn + 1));
    int *cells = malloc(sizeof(int) * 3 * (size_t)nc);
    for (int c = 0; c < nc; ++c)
        for (int m = 0; m < 3; ++m) cells[pos[tri[3 * c + m]]++] = c;
    int rc = 0;
    for (int c = 0; c < nc && rc == 0; ++c)
        for (int m = 0; m < 3; ++m) {
            int p = tri[3 * c + m], q = tri[3 * c + (m + 1) % 3];
            int found = -1;
            for (int i = cnt[p]; i < cnt[p + 1]; ++i) {
                int d = cells[i];
                if (d == c) continue;
                for (int k = 0; k < 3; ++k) {
                    if (tri[3 * d + k] != q) continue;
                    /* d contains p and q: shared edge; d must traverse q -> p */
                    if (tri[3 * d + (k + 1) % 3] != p) { rc = -2; break; }
                    if (found >= 0) { rc = -2; break; }
                    found = d;
                }
            }
            nbr[3 * c + m] = found;
        }
    free(cnt); free(pos); free(cells);
    return rc;
}

/* ------------------------------------------------------------------------
 * Greedy breadth-first partition (stand-in for the ParMETIS step of
 * Sec. 3.1).  Part p receives floor(n/P) + (p < n mod P) cells.  It starts at
 * the unassigned cell of lowest id and grows first-in first-out, visiting the
 * neighbours of a cell in local-edge order 0, 1, 2 and assigning a cell when
 * it is enqueued, until the part is full; an exhausted queue restarts at the
 * next unassigned cell of lowest id.
 * ---------------------------------------------------------------------- */
int od_partition(int nc, const int *nbr, int P, int *part)
{
    if (P <= 0) return -1;
    for (int c = 0; c < nc; ++c) part[c] = -1;
    int *queue = malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    int cursor = 0;
    for (int p = 0; p < P; ++p) {
        int target = nc / P + (p < nc % P ? 1 : 0);
        int count = 0, head = 0, tail = 0;
        while (count < target) {
            if (head == tail) {
                while (cursor < nc && part[cursor] >= 0) ++cursor;
                if (cursor >= nc) break;
                part[cursor] = p; ++count; queue[tail++] = cursor;
                continue;
            }
            int c = queue[head++];
            for (int m = 0; m < 3 && count < target; ++m) {
                int d = nbr[3 * c + m];
                if (d >= 0 && part[d] < 0) { part[d] = p; ++count; queue[tail++] = d; }
            }
        }
    }
    free(queue);
    return 0;
}

/* ------------------------------------------------------------------------
 * Morton key of a cell: centroid ((x0+x1)+x2)/3 in double, scaled by the
 * larger side S of the bounding box of all centroids, quantised to 16 bits
 * (floor((c - min)/S * 65536), clamped to 65535), x on the even bits.
 * ---------------------------------------------------------------------- */
static uint32_t interleave(uint32_t qx, uint32_t qy)
{
    uint32_t k = 0;
    for (int i = 0; i < 16; ++i) {
        k |= ((qx >> i) & 1u) << (2 * i);
        k |= ((qy >> i) & 1u) << (2 * i + 1);
    }
    return k;
}

int od_morton(int nn, const double *xy, int nc, const int *tri, uint32_t *key)
{
    (void)nn;
    double *cx = malloc(sizeof(double) * (size_t)nc), *cy = malloc(sizeof(double) * (size_t)nc);
    double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
    for (int c = 0; c < nc; ++c) {
        const int *t = tri + 3 * c;
        cx[c] = ((xy[2 * t[0]] + xy[2 * t[1]]) + xy[2 * t[2]]) / 3.0;
        cy[c] = ((xy[2 * t[0] + 1] + xy[2 * t[1] + 1]) + xy[2 * t[2] + 1]) / 3.0;
        if (cx[c] < mnx) mnx = cx[c];
        if (cy[c] < mny) mny = cy[c];
        if (cx[c] > mxx) mxx = cx[c];
        if (cy[c] > mxy) mxy = cy[c];
    }
    double S = (mxx - mnx) > (mxy - mny) ? (mxx - mnx) : (mxy - mny);
    if (!(S > 0.0)) S = 1.0;
    for (int c = 0; c < nc; ++c) {
        double fx = floor((cx[c] - mnx) / S * 65536.0), fy = floor((cy[c] - mny) / S * 65536.0);
        if (fx > 65535.0) fx = 65535.0;
        if (fy > 65535.0) fy = 65535.0;
        if (fx < 0.0) fx = 0.0;
        if (fy < 0.0) fy = 0.0;
        key[c] = interleave((uint32_t)fx, (uint32_t)fy);
    }
    free(cx); free(cy);
    return 0;
}

/* ------------------------------------------------------------------------
 * Ghost layers (Sec. 3.2) and renumbering (Sec. 3.3) of part p.
 *   layer 0 = owned cells; layer j = cells not yet included that share an
 *   edge with layer j-1 (breadth-first search on the global dual graph, so
 *   no ghost is ever missed).  Owner of a ghost = its part.  Peers = owners
 *   of the ghosts, ascending.  send(p -> q) = cells of p that are ghosts of q.
 * Local order:
 *   owned send cells by (ascending tuple of destination parts, Morton, gid),
 *   then owned interior cells by (Morton, gid),
 *   then one ghost block per peer (ascending), inside it (layer, Morton, gid).
 *   The send list to q is sorted by (layer seen from q, Morton, gid): the
 *   same key as q's receive block, so a receive lands in place.
 * ---------------------------------------------------------------------- */
typedef struct {
    int n_owned, n_total, n_peers, n_send;
    int *l2g, *layer, *owner, *nbr, *peers, *recv_off, *send_off, *send_idx;
} od_sub;

void od_sub_free(od_sub *S)
{
    if (!S) return;
    free(S->l2g); free(S->layer); free(S->owner); free(S->nbr); free(S->peers);
    free(S->recv_off); free(S->send_off); free(S->send_idx); free(S);
}

/* breadth-first layers from the cells of part q, up to depth k.  dist[] must
 * be -1 on entry; cells reached are appended to list (returns count). */
static int bfs_layers(int nc, const int *nbr, const int *part, int q, int k, int *dist, int *list)
{
    int n = 0;
    for (int c = 0; c < nc; ++c)
        if (part[c] == q) { dist[c] = 0; list[n++] = c; }
    int begin = 0;
    for (int d = 1; d <= k; ++d) {
        int end = n;
        for (int i = begin; i < end; ++i) {
            int c = list[i];
            for (int m = 0; m < 3; ++m) {
                int e = nbr[3 * c + m];
                if (e >= 0 && dist[e] < 0) { dist[e] = d; list[n++] = e; }
            }
        }
        begin = end;
    }
    return n;
}

static const uint32_t *g_key;
static const int *g_lay, *g_own;
static const int *g_dst_off, *g_dst;   /* destination tuples of owned cells */

static int cmp_morton_gid(int a, int b)
{
    if (g_key[a] != g_key[b]) return g_key[a] < g_key[b] ? -1 : 1;
    return a < b ? -1 : (a > b);
}

static int cmp_interior(const void *pa, const void *pb)
{
    return cmp_morton_gid(*(const int *)pa, *(const int *)pb);
}

static int cmp_ghost(const void *pa, const void *pb)
{
    int a = *(const int *)pa, b = *(const int *)pb;
    if (g_own[a] != g_own[b]) return g_own[a] < g_own[b] ? -1 : 1;
    if (g_lay[a] != g_lay[b]) return g_lay[a] < g_lay[b] ? -1 : 1;
    return cmp_morton_gid(a, b);
}

static int cmp_layer(const void *pa, const void *pb)
{
    int a = *(const int *)pa, b = *(const int *)pb;
    if (g_lay[a] != g_lay[b]) return g_lay[a] < g_lay[b] ? -1 : 1;
    return cmp_morton_gid(a, b);
}

/* sort entries are (local slot index into tuple arrays, gid) pairs */
typedef struct { int slot, gid; } sendent;

static int cmp_send(const void *pa, const void *pb)
{
    const sendent *a = pa, *b = pb;
    int na = g_dst_off[a->slot + 1] - g_dst_off[a->slot];
    int nb = g_dst_off[b->slot + 1] - g_dst_off[b->slot];
    const int *ta = g_dst + g_dst_off[a->slot], *tb = g_dst + g_dst_off[b->slot];
    for (int i = 0; i < na && i < nb; ++i)
        if (ta[i] != tb[i]) return ta[i] < tb[i] ? -1 : 1;
    if (na != nb) return na < nb ? -1 : 1;
    return cmp_morton_gid(a->gid, b->gid);
}

od_sub *od_subdomain(int nn, const double *xy, int nc, const int *tri, const int *nbr,
                     const signed char *bc, const int *part, int P, int p, int k)
{
    od_sub *S = calloc(1, sizeof(od_sub));
    uint32_t *key = malloc(sizeof(uint32_t) * (size_t)nc);
    od_morton(nn, xy, nc, tri, key);
    int *dist = malloc(sizeof(int) * (size_t)nc), *list = malloc(sizeof(int) * (size_t)nc);
    for (int c = 0; c < nc; ++c) dist[c] = -1;
    int n_in = bfs_layers(nc, nbr, part, p, k, dist, list);

    /* peers */
    char *is_peer = calloc((size_t)P, 1);
    int n_owned = 0;
    for (int i = 0; i < n_in; ++i) {
        int c = list[i];
        if (dist[c] == 0) ++n_owned;
        else is_peer[part[c]] = 1;
    }
    int n_peers = 0;
    for (int q = 0; q < P; ++q) n_peers += is_peer[q];
    S->n_peers = n_peers;
    S->peers = malloc(sizeof(int) * (size_t)(n_peers + 1));
    int *peer_slot = malloc(sizeof(int) * (size_t)P);
    for (int q = 0, j = 0; q < P; ++q) {
        peer_slot[q] = -1;
        if (is_peer[q]) { S->peers[j] = q; peer_slot[q] = j++; }
    }

    /* for every peer q: cells of p within distance k of q's cells */
    int *distq = malloc(sizeof(int) * (size_t)nc), *listq = malloc(sizeof(int) * (size_t)nc);
    for (int c = 0; c < nc; ++c) distq[c] = -1;
    int *owned_slot = malloc(sizeof(int) * (size_t)nc);
    for (int c = 0; c < nc; ++c) owned_slot[c] = -1;
    int *owned = malloc(sizeof(int) * (size_t)(n_owned + 1));
    int no = 0;
    for (int c = 0; c < nc; ++c)
        if (part[c] == p) { owned_slot[c] = no; owned[no++] = c; }
    /* destination tuples: count, then fill (peers visited ascending) */
    int *dcount = calloc((size_t)n_owned + 1, sizeof(int));
    int **sendsets = malloc(sizeof(int *) * (size_t)(n_peers + 1));
    int **sendlay = malloc(sizeof(int *) * (size_t)(n_peers + 1));
    int *sendn = calloc((size_t)n_peers + 1, sizeof(int));
    for (int j = 0; j < n_peers; ++j) {
        int q = S->peers[j];
        int nq = bfs_layers(nc, nbr, part, q, k, distq, listq);
        sendsets[j] = malloc(sizeof(int) * (size_t)(nq + 1));
        sendlay[j] = malloc(sizeof(int) * (size_t)(nq + 1));
        for (int i = 0; i < nq; ++i) {
            int c = listq[i];
            if (distq[c] > 0 && part[c] == p) {
                sendsets[j][sendn[j]] = c;
                sendlay[j][sendn[j]] = distq[c];
                sendn[j]++;
                dcount[owned_slot[c]]++;
            }
        }
        for (int i = 0; i < nq; ++i) distq[listq[i]] = -1;
    }
    int *doff = malloc(sizeof(int) * ((size_t)n_owned + 1));
    doff[0] = 0;
    for (int i = 0; i < n_owned; ++i) doff[i + 1] = doff[i] + dcount[i];
    int *dst = malloc(sizeof(int) * (size_t)(doff[n_owned] + 1));
    int *fill = calloc((size_t)n_owned + 1, sizeof(int));
    for (int j = 0; j < n_peers; ++j)
        for (int i = 0; i < sendn[j]; ++i) {
            int s = owned_slot[sendsets[j][i]];
            dst[doff[s] + fill[s]++] = S->peers[j];
        }

    /* order owned cells */
    g_key = key; g_dst_off = doff; g_dst = dst;
    int n_sendcells = 0;
    for (int i = 0; i < n_owned; ++i) n_sendcells += dcount[i] > 0;
    sendent *se = malloc(sizeof(sendent) * (size_t)(n_sendcells + 1));
    int *interior = malloc(sizeof(int) * (size_t)(n_owned + 1));
    int ns = 0, ni = 0;
    for (int i = 0; i < n_owned; ++i) {
        if (dcount[i] > 0) { se[ns].slot = i; se[ns].gid = owned[i]; ++ns; }
        else interior[ni++] = owned[i];
    }
    qsort(se, (size_t)ns, sizeof(sendent), cmp_send);
    qsort(interior, (size_t)ni, sizeof(int), cmp_interior);

    /* ghosts */
    int n_ghost = n_in - n_owned;
    int *ghost = malloc(sizeof(int) * (size_t)(n_ghost + 1));
    int ng = 0;
    for (int i = 0; i < n_in; ++i)
        if (dist[list[i]] > 0) ghost[ng++] = list[i];
    g_lay = dist; g_own = part;
    qsort(ghost, (size_t)ng, sizeof(int), cmp_ghost);

    int n_total = n_in;
    S->n_owned = n_owned; S->n_total = n_total;
    S->l2g = malloc(sizeof(int) * (size_t)(n_total + 1));
    S->layer = malloc(sizeof(int) * (size_t)(n_total + 1));
    S->owner = malloc(sizeof(int) * (size_t)(n_total + 1));
    int L = 0;
    for (int i = 0; i < ns; ++i) S->l2g[L++] = se[i].gid;
    for (int i = 0; i < ni; ++i) S->l2g[L++] = interior[i];
    for (int i = 0; i < ng; ++i) S->l2g[L++] = ghost[i];
    int *g2l = malloc(sizeof(int) * (size_t)nc);
    for (int c = 0; c < nc; ++c) g2l[c] = -1;
    for (int i = 0; i < n_total; ++i) {
        int c = S->l2g[i];
        g2l[c] = i; S->layer[i] = dist[c]; S->owner[i] = part[c];
    }
    S->recv_off = malloc(sizeof(int) * (size_t)(n_peers + 1));
    S->recv_off[0] = 0;
    for (int j = 0; j < n_peers; ++j) {
        int cntq = 0;
        for (int i = 0; i < ng; ++i) cntq += (part[ghost[i]] == S->peers[j]);
        S->recv_off[j + 1] = S->recv_off[j] + cntq;
    }
    /* local neighbour table */
    S->nbr = malloc(sizeof(int) * 3 * (size_t)(n_total + 1));
    for (int i = 0; i < n_total; ++i)
        for (int m = 0; m < 3; ++m) {
            int gnb = nbr[3 * S->l2g[i] + m];
            int v;
            if (gnb >= 0) v = g2l[gnb] >= 0 ? g2l[gnb] : BC_HALO;
            else v = bc[3 * S->l2g[i] + m] < 0 ? bc[3 * S->l2g[i] + m] : -1;
            S->nbr[3 * i + m] = v;
        }
    /* send lists */
    S->send_off = malloc(sizeof(int) * (size_t)(n_peers + 1));
    S->send_off[0] = 0;
    for (int j = 0; j < n_peers; ++j) S->send_off[j + 1] = S->send_off[j] + sendn[j];
    S->n_send = S->send_off[n_peers];
    S->send_idx = malloc(sizeof(int) * (size_t)(S->n_send + 1));
    int *laybuf = malloc(sizeof(int) * (size_t)nc);
    for (int j = 0; j < n_peers; ++j) {
        int *cells = sendsets[j];
        for (int i = 0; i < sendn[j]; ++i) laybuf[cells[i]] = sendlay[j][i];
        g_lay = laybuf;
        qsort(cells, (size_t)sendn[j], sizeof(int), cmp_layer);
        for (int i = 0; i < sendn[j]; ++i) S->send_idx[S->send_off[j] + i] = g2l[cells[i]];
    }
    (void)peer_slot;
    free(laybuf); free(g2l); free(ghost); free(interior); free(se); free(fill); free(dst);
    free(doff);
    for (int j = 0; j < n_peers; ++j) { free(sendsets[j]); free(sendlay[j]); }
    free(sendsets); free(sendlay); free(sendn); free(dcount); free(owned); free(owned_slot);
    free(distq); free(listq); free(peer_slot); free(is_peer); free(dist); free(list); free(key);
    return S;
}
