// Host-side renumbering of sets: Cuthill-McKee level ordering of points,
// lexicographic element order, first-touch ordering of secondary point sets
// (paper Section 2.3.1), partition-based element blocks and block-signature
// point grouping (Section 2.3.2).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.hpp"

namespace um {

namespace {

// Point graph of a map: the points of each element form a clique.
struct Graph {
    std::vector<int64_t> off;
    std::vector<int32_t> adj;
    int32_t degree(int32_t p) const { return int32_t(off[p + 1] - off[p]); }
};

Graph point_graph(const Map &m, int64_t n) {
    const int k = m.arity;
    const int64_t ne = k ? int64_t(m.table.size()) / k : 0;
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t *r = &m.table[e * k];
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j)
                if (r[i] != r[j]) cnt[r[i] + 1]++;
    }
    for (int64_t p = 0; p < n; ++p) cnt[p + 1] += cnt[p];
    std::vector<int32_t> raw(cnt[n]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t *r = &m.table[e * k];
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j)
                if (r[i] != r[j]) raw[fill[r[i]]++] = r[j];
    }
    Graph g;
    g.off.assign(n + 1, 0);
    g.adj.reserve(raw.size());
    for (int64_t p = 0; p < n; ++p) {
        auto b = raw.begin() + cnt[p], e = raw.begin() + cnt[p + 1];
        std::sort(b, e);
        auto u = std::unique(b, e);
        g.adj.insert(g.adj.end(), b, u);
        g.off[p + 1] = int64_t(g.adj.size());
    }
    return g;
}

// Breadth-first search from `root`.  Fills dist for reached points (others
// must be -1 on entry), appends reached points to `seen` in visit order and
// returns the eccentricity of root.  The caller resets dist via `seen`.
int32_t bfs(const Graph &g, int32_t root, std::vector<int32_t> &dist, std::vector<int32_t> &seen) {
    size_t head = seen.size();
    dist[root] = 0;
    seen.push_back(root);
    int32_t ecc = 0;
    while (head < seen.size()) {
        int32_t p = seen[head++];
        int32_t d = dist[p];
        ecc = std::max(ecc, d);
        for (int64_t i = g.off[p]; i < g.off[p + 1]; ++i) {
            int32_t q = g.adj[i];
            if (dist[q] < 0) {
                dist[q] = d + 1;
                seen.push_back(q);
            }
        }
    }
    return ecc;
}

void reset(std::vector<int32_t> &dist, std::vector<int32_t> &seen) {
    for (int32_t p : seen) dist[p] = -1;
    seen.clear();
}

// (degree, id) ordering used for every tie-break in the traversal.
struct DegLess {
    const Graph *g;
    bool operator()(int32_t a, int32_t b) const {
        int32_t da = g->degree(a), db = g->degree(b);
        return da != db ? da < db : a < b;
    }
};

// George & Liu pseudo-peripheral point of the component of `seed`.
int32_t pseudo_peripheral(const Graph &g, int32_t seed, std::vector<int32_t> &dist,
                          std::vector<int32_t> &seen) {
    DegLess less{&g};
    bfs(g, seed, dist, seen);
    int32_t r = *std::min_element(seen.begin(), seen.end(), less);
    reset(dist, seen);
    for (;;) {
        int32_t ecc_r = bfs(g, r, dist, seen);
        int32_t x = -1;
        for (int32_t p : seen)
            if (dist[p] == ecc_r && (x < 0 || less(p, x))) x = p;
        reset(dist, seen);
        int32_t ecc_x = bfs(g, x, dist, seen);
        reset(dist, seen);
        if (ecc_x > ecc_r) {
            r = x;
            continue;
        }
        return r;
    }
}

std::vector<int32_t> inverse(const std::vector<int32_t> &p) {
    std::vector<int32_t> inv(p.size());
    for (size_t k = 0; k < p.size(); ++k) inv[p[k]] = int32_t(k);
    return inv;
}

}  // namespace

std::vector<int32_t> cuthill_mckee(const Map &m, int64_t n, bool reverse) {
    Graph g = point_graph(m, n);
    DegLess less{&g};
    std::vector<int32_t> dist(n, -1), seen, order;
    std::vector<char> visited(n, 0);
    order.reserve(n);
    std::vector<int32_t> nb;
    for (int64_t s = 0; s < n; ++s) {
        if (visited[s]) continue;
        int32_t r = pseudo_peripheral(g, int32_t(s), dist, seen);
        size_t head = order.size();
        visited[r] = 1;
        order.push_back(r);
        while (head < order.size()) {
            int32_t p = order[head++];
            nb.clear();
            for (int64_t i = g.off[p]; i < g.off[p + 1]; ++i)
                if (!visited[g.adj[i]]) nb.push_back(g.adj[i]);
            std::sort(nb.begin(), nb.end(), less);
            for (int32_t q : nb) {
                visited[q] = 1;
                order.push_back(q);
            }
        }
    }
    if (reverse) std::reverse(order.begin(), order.end());
    return order;
}

std::vector<int32_t> lexicographic_elements(const Map &m) {
    const int k = m.arity;
    const int64_t ne = int64_t(m.table.size()) / k;
    std::vector<int32_t> keys(m.table);
    for (int64_t e = 0; e < ne; ++e) std::sort(keys.begin() + e * k, keys.begin() + (e + 1) * k);
    std::vector<int32_t> order(ne);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const int32_t *ka = &keys[int64_t(a) * k], *kb = &keys[int64_t(b) * k];
        for (int i = 0; i < k; ++i)
            if (ka[i] != kb[i]) return ka[i] < kb[i];
        return a < b;
    });
    return order;
}

std::vector<int32_t> first_touch(const Map &m, int64_t n) {
    std::vector<char> seen(n, 0);
    std::vector<int32_t> order;
    order.reserve(n);
    for (int32_t p : m.table)
        if (!seen[p]) {
            seen[p] = 1;
            order.push_back(p);
        }
    for (int64_t p = 0; p < n; ++p)
        if (!seen[p]) order.push_back(int32_t(p));
    return order;
}

void apply_set_perm(Ctx &ctx, int32_t set, const std::vector<int32_t> &perm) {
    Set &s = ctx.sets[set];
    std::vector<int32_t> inv = inverse(perm);
    for (Map &m : ctx.maps) {
        if (m.to == set)
            for (int32_t &v : m.table) v = inv[v];
        if (m.from == set) {
            std::vector<int32_t> t(m.table.size());
            for (int64_t k = 0; k < s.size; ++k)
                std::memcpy(&t[k * m.arity], &m.table[int64_t(perm[k]) * m.arity],
                            sizeof(int32_t) * m.arity);
            m.table.swap(t);
        }
    }
    std::vector<int32_t> n2o(s.size);
    for (int64_t k = 0; k < s.size; ++k) n2o[k] = s.new2orig[perm[k]];
    s.new2orig.swap(n2o);
    s.part_block_size = 0;
    s.part_off.clear();
    s.part_code.clear();
}

// ------------------------------------------------------------ partitioning
namespace {

struct Bisector {
    const std::vector<double> *coord;  // [n_elem][dim]
    int dim;
    int32_t max_block;
    std::vector<int32_t> out;          // element order, block by block
    std::vector<int32_t> off;          // block offsets
    std::vector<int32_t> code;         // per block: last cut side along each axis

    void run(int32_t *first, int64_t n, int64_t nb, int32_t sides) {
        if (nb <= 1 || n <= max_block) {
            // one block (nb >= 1 and n <= nb*max_block guarantee n <= max_block)
            std::sort(first, first + n);
            out.insert(out.end(), first, first + n);
            off.push_back(int32_t(out.size()));
            code.push_back(sides);
            return;
        }
        // cut across the longest extent; extents within 5 % of each other
        // count as equal and the lowest axis wins, so that equal subtrees of
        // a perturbed structured mesh are cut alike and their blocks stay on
        // a regular grid
        const std::vector<double> &c = *coord;
        int axis = 0;
        double best = -1.0;
        for (int a = 0; a < dim; ++a) {
            double lo = INFINITY, hi = -INFINITY;
            for (int64_t i = 0; i < n; ++i) {
                double v = c[int64_t(first[i]) * dim + a];
                lo = std::min(lo, v);
                hi = std::max(hi, v);
            }
            if (hi - lo > 1.05 * best) {
                best = hi - lo;
                axis = a;
            }
        }
        int64_t nl = nb / 2;
        int64_t n1 = (n * nl) / nb;  // floor keeps both sides within their share
        std::nth_element(first, first + n1, first + n, [&](int32_t x, int32_t y) {
            double vx = c[int64_t(x) * dim + axis], vy = c[int64_t(y) * dim + axis];
            return vx != vy ? vx < vy : x < y;
        });
        run(first, n1, nl, sides & ~(1 << axis));
        run(first + n1, n - n1, nb - nl, sides | (1 << axis));
    }
};

// Graph-distance coordinates of points when no geometry is given: BFS
// distances from landmarks found by repeated farthest-point sweeps; the
// coordinates are (d0 - d1, d2 - d3).
std::vector<double> landmark_coords(const Map &m, int64_t n) {
    Graph g = point_graph(m, n);
    std::vector<double> xy(2 * n, 0.0);
    std::vector<int32_t> dist(n, -1), seen;
    std::vector<char> done(n, 0);
    std::vector<std::vector<int32_t>> F(5, std::vector<int32_t>(n, 0));
    for (int64_t s = 0; s < n; ++s) {
        if (done[s]) continue;
        bfs(g, int32_t(s), dist, seen);
        std::vector<int32_t> comp(seen);
        reset(dist, seen);
        for (int32_t p : comp) done[p] = 1;
        auto farthest_from = [&](const std::vector<std::vector<int32_t> *> &fields) {
            int32_t best = comp[0];
            int64_t bv = -1;
            for (int32_t p : comp) {
                int64_t v = INT64_MAX;
                for (auto *f : fields) v = std::min<int64_t>(v, (*f)[p]);
                if (v > bv || (v == bv && p < best)) {
                    bv = v;
                    best = p;
                }
            }
            return best;
        };
        auto field = [&](int32_t root, std::vector<int32_t> &f) {
            bfs(g, root, dist, seen);
            for (int32_t p : comp) f[p] = dist[p];
            reset(dist, seen);
        };
        field(comp[0], F[4]);
        int32_t l0 = farthest_from({&F[4]});
        field(l0, F[0]);
        int32_t l1 = farthest_from({&F[0]});
        field(l1, F[1]);
        int32_t l2 = farthest_from({&F[0], &F[1]});
        field(l2, F[2]);
        int32_t l3 = farthest_from({&F[0], &F[1], &F[2]});
        field(l3, F[3]);
        for (int32_t p : comp) {
            xy[2 * p] = double(F[0][p] - F[1][p]);
            xy[2 * p + 1] = double(F[2][p] - F[3][p]);
        }
    }
    return xy;
}

}  // namespace

std::vector<int32_t> partition_elements(const Ctx &ctx, int32_t drv, int32_t block_size,
                                        int32_t coord_map, int32_t coord_dim,
                                        const double *coords, std::vector<int32_t> &block_off,
                                        std::vector<int32_t> &block_code) {
    const Map &m = ctx.maps[drv];
    const int64_t ne = ctx.sets[m.from].size;
    block_off.assign(1, 0);
    block_code.clear();
    if (ne == 0) return {};
    // element coordinates: mean of their points' coordinates
    std::vector<double> pc;
    int dim = 2;
    const Map *cm = &m;
    if (coords && coord_map >= 0) {
        cm = &ctx.maps[coord_map];
        dim = coord_dim;
        pc.assign(coords, coords + ctx.sets[cm->to].size * dim);
    } else {
        pc = landmark_coords(m, ctx.sets[m.to].size);
    }
    std::vector<double> ec(ne * dim, 0.0);
    const int k = cm->arity;
    for (int64_t e = 0; e < ne; ++e)
        for (int i = 0; i < k; ++i) {
            int32_t p = cm->table[e * k + i];
            for (int a = 0; a < dim; ++a) ec[e * dim + a] += pc[int64_t(p) * dim + a];
        }
    for (double &v : ec) v /= k;
    // connected components of the elements (elements sharing a point of the
    // driving map): each with at least block_size elements is bisected on
    // its own into ceil(n_c / block_size) blocks, so such a component never
    // shares a block (a count-based cut through a union of separate meshes
    // would otherwise leave slivers and blocks straddling two meshes, whose
    // staged sets are several times larger); smaller components are packed
    // whole, in order, into blocks of at most block_size elements
    const int64_t np = ctx.sets[m.to].size;
    std::vector<int32_t> parent(np);
    std::iota(parent.begin(), parent.end(), 0);
    auto find = [&](int32_t x) {
        while (parent[x] != x) {
            parent[x] = parent[parent[x]];
            x = parent[x];
        }
        return x;
    };
    for (int64_t e = 0; e < ne; ++e)
        for (int i = 1; i < m.arity; ++i) {
            const int32_t a = find(m.table[e * m.arity]), c = find(m.table[e * m.arity + i]);
            if (a != c) parent[std::max(a, c)] = std::min(a, c);
        }
    // components numbered by their first element; elements listed per
    // component in increasing order
    std::vector<int32_t> comp_of_root(np, -1), comp(ne);
    int32_t ncomp = 0;
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t r = find(m.table[e * m.arity]);
        if (comp_of_root[r] < 0) comp_of_root[r] = ncomp++;
        comp[e] = comp_of_root[r];
    }
    std::vector<int64_t> coff(int64_t(ncomp) + 1, 0);
    for (int64_t e = 0; e < ne; ++e) coff[comp[e] + 1]++;
    for (int32_t c = 0; c < ncomp; ++c) coff[c + 1] += coff[c];
    std::vector<int32_t> ids(ne);
    {
        std::vector<int64_t> fill(coff.begin(), coff.end() - 1);
        for (int64_t e = 0; e < ne; ++e) ids[fill[comp[e]]++] = int32_t(e);
    }
    Bisector b{&ec, dim, block_size, {}, {0}, {}};
    b.out.reserve(ne);
    int64_t pack = 0;  // elements of small components in the open block
    auto close_pack = [&]() {
        if (pack == 0) return;
        // previous relative order inside the block, as for bisected blocks
        std::sort(b.out.end() - pack, b.out.end());
        b.off.push_back(int32_t(b.out.size()));
        b.code.push_back(0);
        pack = 0;
    };
    for (int32_t c = 0; c < ncomp; ++c) {
        const int64_t n = coff[c + 1] - coff[c];
        if (n >= block_size) {
            close_pack();
            b.run(ids.data() + coff[c], n, (n + block_size - 1) / block_size, 0);
            continue;
        }
        if (pack + n > block_size) close_pack();
        b.out.insert(b.out.end(), ids.data() + coff[c], ids.data() + coff[c + 1]);
        pack += n;
    }
    close_pack();
    block_off.swap(b.off);
    block_code.swap(b.code);
    return b.out;
}

std::vector<int32_t> signature_order(const Ctx &ctx, int32_t from, int32_t set,
                                     const std::vector<int32_t> &block_of_elem, int32_t key) {
    const int64_t n = ctx.sets[set].size;
    const int64_t ne = ctx.sets[from].size;
    // accessing blocks per point; elements are visited in block order so each
    // point's list comes out sorted, duplicates adjacent
    std::vector<int64_t> cnt(n + 1, 0);
    std::vector<const Map *> maps;
    for (const Map &m : ctx.maps)
        if (m.from == from && m.to == set) maps.push_back(&m);
    for (const Map *m : maps)
        for (int32_t p : m->table) cnt[p + 1]++;
    for (int64_t p = 0; p < n; ++p) cnt[p + 1] += cnt[p];
    std::vector<int32_t> lst(cnt[n]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t e = 0; e < ne; ++e)
        for (const Map *m : maps)
            for (int i = 0; i < m->arity; ++i) {
                int32_t p = m->table[e * m->arity + i];
                lst[fill[p]++] = block_of_elem[e];
            }
    std::vector<int64_t> len(n);
    for (int64_t p = 0; p < n; ++p) {
        auto b = lst.begin() + cnt[p], e = lst.begin() + cnt[p + 1];
        std::sort(b, e);  // already sorted unless several maps interleave
        len[p] = std::unique(b, e) - b;
    }
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        if (key == 3) {
            // the accessing blocks from the largest down, element by element
            // (a prefix first); unaccessed points last
            if (!len[a] || !len[b]) return len[a] != 0 && len[b] == 0;
            const int64_t m = std::min(len[a], len[b]);
            for (int64_t i = 1; i <= m; ++i) {
                const int32_t x = lst[cnt[a] + len[a] - i], y = lst[cnt[b] + len[b] - i];
                if (x != y) return x < y;
            }
            return len[a] < len[b];
        }
        if (key == 2) {
            // smallest accessing block first; unaccessed points last
            const int64_t fa = len[a] ? lst[cnt[a]] : INT64_MAX;
            const int64_t fb = len[b] ? lst[cnt[b]] : INT64_MAX;
            if (fa != fb) return fa < fb;
        }
        int64_t la = len[a] ? len[a] : INT64_MAX, lb = len[b] ? len[b] : INT64_MAX;
        if (la != lb) return la < lb;
        for (int64_t i = 0; i < len[a]; ++i) {
            int32_t x = lst[cnt[a] + i], y = lst[cnt[b] + i];
            if (x != y) return x < y;
        }
        return false;
    });
    return order;
}

void reorder_mesh(Ctx &ctx, const um_reorder_opts &o) {
    if (o.mode == UM_REORDER_NONE) return;
    if (o.driving_map < 0 || o.driving_map >= int32_t(ctx.maps.size()))
        fail(UM_ERR_ARG, "reorder: driving_map %d is not a map id", o.driving_map);
    const int32_t F = ctx.maps[o.driving_map].from, T = ctx.maps[o.driving_map].to;
    if (o.mode == UM_REORDER_RCM || o.mode == UM_REORDER_GPS) {
        if (F == T) fail(UM_ERR_UNSUPPORTED, "reorder: map from a set into itself");
        apply_set_perm(ctx, T, cuthill_mckee(ctx.maps[o.driving_map], ctx.sets[T].size,
                                             o.mode == UM_REORDER_RCM));
        apply_set_perm(ctx, F, lexicographic_elements(ctx.maps[o.driving_map]));
        std::vector<int32_t> done{F, T};
        for (size_t i = 0; i < ctx.maps.size(); ++i) {
            const Map &m = ctx.maps[i];
            if (m.from != F || std::find(done.begin(), done.end(), m.to) != done.end()) continue;
            done.push_back(m.to);
            apply_set_perm(ctx, m.to, first_touch(m, ctx.sets[m.to].size));
        }
        return;
    }
    if (o.mode == UM_REORDER_LEXICOGRAPHIC) {
        apply_set_perm(ctx, F, lexicographic_elements(ctx.maps[o.driving_map]));
        return;
    }
    if (o.mode != UM_REORDER_PARTITION && o.mode != UM_REORDER_USER_BLOCKS)
        fail(UM_ERR_ARG, "reorder: unknown mode %d", o.mode);
    if (o.block_size < 1 || o.block_size > 1024)
        fail(UM_ERR_ARG, "reorder: block_size %d outside 1..1024", o.block_size);
    std::vector<int32_t> off, code;
    std::vector<int32_t> perm;
    if (o.mode == UM_REORDER_USER_BLOCKS) {
        if (!o.block_of) fail(UM_ERR_ARG, "reorder: USER_BLOCKS needs block_of");
        const int64_t n = ctx.sets[F].size;
        int32_t nbid = 0;
        for (int64_t e = 0; e < n; ++e) {
            if (o.block_of[e] < 0) fail(UM_ERR_ARG, "reorder: negative block id at %lld", (long long)e);
            nbid = std::max(nbid, o.block_of[e] + 1);
        }
        std::vector<int32_t> cnt(int64_t(nbid) + 1, 0);
        for (int64_t e = 0; e < n; ++e) cnt[o.block_of[e] + 1]++;
        for (int32_t b = 0; b < nbid; ++b)
            if (cnt[b + 1] > o.block_size)
                fail(UM_ERR_ARG, "reorder: block %d holds %d elements > block_size %d", b, cnt[b + 1],
                     o.block_size);
        for (int32_t b = 0; b < nbid; ++b) cnt[b + 1] += cnt[b];
        perm.resize(n);
        std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
        for (int64_t e = 0; e < n; ++e) perm[fill[o.block_of[e]]++] = int32_t(e);
        off.push_back(0);
        for (int32_t b = 0; b < nbid; ++b)
            if (cnt[b + 1] > cnt[b]) off.push_back(cnt[b + 1]);
    }
    if (o.mode == UM_REORDER_PARTITION && o.coord_map >= 0) {
        if (o.coord_map >= int32_t(ctx.maps.size()) || ctx.maps[o.coord_map].from != F)
            fail(UM_ERR_ARG, "reorder: coord_map must be a map from the partitioned set");
        if (!o.coords || o.coord_dim < 1 || o.coord_dim > 3)
            fail(UM_ERR_ARG, "reorder: coords missing or coord_dim outside 1..3");
    }
    if (o.mode == UM_REORDER_PARTITION)
        perm = partition_elements(ctx, o.driving_map, o.block_size, o.coord_map, o.coord_dim,
                                  o.coords, off, code);
    apply_set_perm(ctx, F, perm);
    ctx.sets[F].part_block_size = o.block_size;
    ctx.sets[F].part_off = off;
    ctx.sets[F].part_code = code;
    if (o.point_reorder < 0 || o.point_reorder > 3)
        fail(UM_ERR_ARG, "reorder: point_reorder %d not in 0..3", o.point_reorder);
    if (o.point_reorder) {
        std::vector<int32_t> blk(ctx.sets[F].size);
        for (size_t b = 0; b + 1 < off.size(); ++b)
            for (int32_t e = off[b]; e < off[b + 1]; ++e) blk[e] = int32_t(b);
        std::vector<int32_t> done{F};
        for (size_t i = 0; i < ctx.maps.size(); ++i) {
            const Map &m = ctx.maps[i];
            if (m.from != F || std::find(done.begin(), done.end(), m.to) != done.end()) continue;
            done.push_back(m.to);
            apply_set_perm(ctx, m.to, signature_order(ctx, F, m.to, blk, o.point_reorder));
        }
    }
}

}  // namespace um
