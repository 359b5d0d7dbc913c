// Host-side execution plans for the edge-flux loop: global colouring,
// two-layer (block + thread) colouring with staged point lists and local
// index maps (paper Section 2.1 and 2.2, Algorithm 1), LDS sizing.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <set>

#include "internal.hpp"

namespace um {

// x[3], v[3], force acc[3] and the staged node id
int64_t hex_lds_bytes(int64_t nn, bool dataflow) {
    // x, v, force accumulators (3 doubles each) and a staged id per node; the
    // dataflow kernel pads its accumulators to groups of 16 nodes
    return nn * (9 * 8 + 4) + (dataflow ? 3 * 8 * (((nn + 15) & ~int64_t(15)) - nn) : 0);
}

int64_t lf2d_lds_bytes(int32_t staging, int32_t dtype, int64_t nc, int64_t nn) {
    const int64_t inc = nc * 4 * 8;  // FP64 increments (res preloaded)
    if (staging == UM_STAGE_INC_ONLY) return inc;
    const int64_t w = dtype == UM_F64 ? 8 : 4;
    return inc + nc * 5 * w + nn * 2 * w;  // q[4], adt per cell; x[2] per node
}

// Stable counting sort of 0..n-1 by small integer keys; returns the order
// and fills offsets[key] (size nkeys + 1).
std::vector<int32_t> counting_order(const std::vector<int32_t> &key, int32_t nkeys,
                                    std::vector<int32_t> &offsets) {
    offsets.assign(nkeys + 1, 0);
    for (int32_t k : key) offsets[k + 1]++;
    for (int32_t c = 0; c < nkeys; ++c) offsets[c + 1] += offsets[c];
    std::vector<int32_t> fill(offsets.begin(), offsets.end() - 1), order(key.size());
    for (size_t i = 0; i < key.size(); ++i) order[fill[key[i]]++] = int32_t(i);
    return order;
}

// Global first-fit colouring of elements writing the points of their map
// row: every point keeps a bit set of the colours already written there.
int32_t global_colours(const Map &mc, int64_t C, std::vector<int32_t> &colour) {
    const int k = mc.arity;
    const int64_t E = int64_t(mc.table.size()) / k;
    colour.assign(E, 0);
    int32_t words = 1;
    std::vector<uint64_t> used(C, 0);
    int32_t ncol = 0;
    for (int64_t e = 0; e < E; ++e) {
        const int32_t *pts = &mc.table[k * e];
        int32_t c = 0;
        for (int32_t w = 0;; ++w) {
            if (w == words) {  // grow the bit sets by one word per point
                std::vector<uint64_t> grown(C * (words + 1), 0);
                for (int64_t p = 0; p < C; ++p)
                    std::memcpy(&grown[p * (words + 1)], &used[p * words], 8 * words);
                used.swap(grown);
                ++words;
            }
            uint64_t taken = 0;
            for (int i = 0; i < k; ++i) taken |= used[int64_t(pts[i]) * words + w];
            if (~taken) {
                c = w * 64 + __builtin_ctzll(~taken);
                break;
            }
        }
        colour[e] = c;
        for (int i = 0; i < k; ++i) used[int64_t(pts[i]) * words + c / 64] |= 1ull << (c % 64);
        ncol = std::max(ncol, c + 1);
    }
    return ncol;
}

// DSatur (Brelaz): repeatedly colour, with its smallest free colour, the
// uncoloured block whose neighbours hold the most distinct colours (ties:
// more uncoloured neighbours, then the smaller id).  Returns the number of
// colours, or 0 if it would need more than 64.
static int32_t dsatur(const std::vector<int64_t> &adj_off, const std::vector<int32_t> &adj,
                      std::vector<int32_t> &col) {
    const int32_t nb = int32_t(adj_off.size()) - 1;
    col.assign(nb, -1);
    std::vector<uint64_t> seen(nb, 0);
    std::vector<int32_t> sat(nb, 0), deg(nb);
    for (int32_t b = 0; b < nb; ++b) deg[b] = int32_t(adj_off[b + 1] - adj_off[b]);
    struct Key {
        int32_t sat, deg, id;
        bool operator<(const Key &o) const {
            if (sat != o.sat) return sat > o.sat;
            if (deg != o.deg) return deg > o.deg;
            return id < o.id;
        }
    };
    std::set<Key> q;
    for (int32_t b = 0; b < nb; ++b) q.insert(Key{0, deg[b], b});
    int32_t ncol = 0;
    while (!q.empty()) {
        const int32_t b = q.begin()->id;
        q.erase(q.begin());
        if (~seen[b] == 0) return 0;
        const int32_t c = __builtin_ctzll(~seen[b]);
        col[b] = c;
        ncol = std::max(ncol, c + 1);
        for (int64_t i = adj_off[b]; i < adj_off[b + 1]; ++i) {
            const int32_t n = adj[i];
            if (col[n] >= 0) continue;
            q.erase(Key{sat[n], deg[n], n});
            if (!(seen[n] >> c & 1)) {
                seen[n] |= 1ull << c;
                sat[n]++;
            }
            deg[n]--;
            q.insert(Key{sat[n], deg[n], n});
        }
    }
    return ncol;
}

// Tabu search for a proper k-colouring of the block graph (Hertz and de
// Werra's TabuCol), starting from `col` with colour x folded onto x mod k:
// each step moves one conflicting block (among at most 40 sampled) to the
// colour that removes the most conflicts (ties broken at random), never back
// to a colour it left in the last 10-15 steps.  Deterministic (fixed-seed SplitMix64).  On success
// `col` holds the k-colouring; otherwise it is unchanged.
static bool tabu_colouring(const std::vector<int64_t> &adj_off, const std::vector<int32_t> &adj,
                           int32_t k, int64_t max_iter, std::vector<int32_t> &col) {
    const int32_t nb = int32_t(col.size());
    uint64_t rng = 0x243F6A8885A308D3ull;
    auto next = [&rng]() {
        uint64_t z = (rng += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    std::vector<int32_t> c(nb);
    for (int32_t b = 0; b < nb; ++b) c[b] = col[b] % k;
    std::vector<int32_t> g(int64_t(nb) * k, 0);  // neighbours of b holding colour x
    for (int32_t b = 0; b < nb; ++b)
        for (int64_t i = adj_off[b]; i < adj_off[b + 1]; ++i) g[int64_t(b) * k + c[adj[i]]]++;
    std::vector<int32_t> cl, where(nb, -1);   // conflicting blocks
    auto refresh = [&](int32_t b) {
        const bool in = g[int64_t(b) * k + c[b]] > 0;
        if (in && where[b] < 0) {
            where[b] = int32_t(cl.size());
            cl.push_back(b);
        } else if (!in && where[b] >= 0) {
            const int32_t last = cl.back();
            cl[where[b]] = last;
            where[last] = where[b];
            cl.pop_back();
            where[b] = -1;
        }
    };
    int64_t conf = 0;
    for (int32_t b = 0; b < nb; ++b) {
        conf += g[int64_t(b) * k + c[b]];
        refresh(b);
    }
    conf /= 2;
    std::vector<int64_t> tabu(int64_t(nb) * k, 0);
    for (int64_t it = 1; conf > 0 && it <= max_iter; ++it) {
        int32_t mb = -1, mc = -1;
        int64_t md = 0;
        uint64_t ties = 0;  // equal best moves seen: one is kept uniformly
        const size_t ns = std::min<size_t>(cl.size(), 40);
        for (size_t j = 0; j < ns; ++j) {
            const int32_t b = cl.size() <= 40 ? cl[j] : cl[next() % cl.size()];
            for (int32_t x = 0; x < k; ++x) {
                if (x == c[b] || tabu[int64_t(b) * k + x] > it) continue;
                const int64_t d = int64_t(g[int64_t(b) * k + x]) - g[int64_t(b) * k + c[b]];
                if (mb < 0 || d < md) {
                    mb = b;
                    mc = x;
                    md = d;
                    ties = 1;
                } else if (d == md && next() % ++ties == 0) {
                    mb = b;
                    mc = x;
                }
            }
        }
        if (mb < 0) continue;
        const int32_t old = c[mb];
        tabu[int64_t(mb) * k + old] = it + 10 + int64_t(next() % 6);
        c[mb] = mc;
        for (int64_t i = adj_off[mb]; i < adj_off[mb + 1]; ++i) {
            g[int64_t(adj[i]) * k + old]--;
            g[int64_t(adj[i]) * k + mc]++;
        }
        conf += md;
        refresh(mb);
        for (int64_t i = adj_off[mb]; i < adj_off[mb + 1]; ++i) refresh(adj[i]);
    }
    if (conf != 0) return false;
    col = c;
    return true;
}

// Blocks, layer-1 colouring, launch order and dataflow predecessors: the
// part of a hierarchical plan that only depends on which points each
// element writes (wt: [E][arity] into 0..C-1).  Returns the colour count.
int32_t plan_blocks(const Ctx &ctx, int32_t iter_set, const int32_t *wt, int arity, int64_t C,
                    const um_plan_opts &o, HostPlan &hp) {
    const int64_t E = ctx.sets[iter_set].size;
    // ---- blocks: the set's partition if built for this size; groups of k
    // consecutive partition blocks if built for block_size / k (bisection
    // order keeps consecutive blocks adjacent in space); else chunks
    const Set &is = ctx.sets[iter_set];
    const int32_t pbs = is.part_block_size;
    bool partition_blocks = false;  // plan blocks are the partition's own blocks
    if (pbs > 0 && !is.part_off.empty() && o.block_size % pbs == 0) {
        const int32_t k = o.block_size / pbs;
        partition_blocks = k == 1;
        const int32_t npb = int32_t(is.part_off.size()) - 1;
        hp.blk_off.clear();
        for (int32_t b = 0; b < npb; b += k) hp.blk_off.push_back(is.part_off[b]);
        hp.blk_off.push_back(is.part_off[npb]);
    } else {
        hp.blk_off.clear();
        for (int64_t s = 0; s < E; s += o.block_size) hp.blk_off.push_back(int32_t(s));
        hp.blk_off.push_back(int32_t(E));
        if (E == 0) hp.blk_off.assign(1, 0);
    }
    const int32_t nb = int32_t(hp.blk_off.size()) - 1;

    // ---- layer 1: block colouring.  For every cell, the blocks that write
    // it (in block order); a block's forbidden colours are those of the
    // earlier blocks sharing one of its cells.
    std::vector<int64_t> cb_off(C + 1, 0);
    std::vector<int32_t> last(C, -1);
    for (int32_t b = 0; b < nb; ++b)
        for (int32_t e = hp.blk_off[b]; e < hp.blk_off[b + 1]; ++e)
            for (int s = 0; s < arity; ++s) {
                int32_t c = wt[int64_t(arity) * e + s];
                if (last[c] != b) {
                    last[c] = b;
                    cb_off[c + 1]++;
                }
            }
    for (int64_t c = 0; c < C; ++c) cb_off[c + 1] += cb_off[c];
    std::vector<int32_t> cb(cb_off[C]);
    {
        std::vector<int64_t> fill(cb_off.begin(), cb_off.end() - 1);
        std::fill(last.begin(), last.end(), -1);
        for (int32_t b = 0; b < nb; ++b)
            for (int32_t e = hp.blk_off[b]; e < hp.blk_off[b + 1]; ++e)
                for (int s = 0; s < arity; ++s) {
                    int32_t c = wt[int64_t(arity) * e + s];
                    if (last[c] != b) {
                        last[c] = b;
                        cb[fill[c]++] = b;
                    }
                }
    }
    // block adjacency: blocks sharing a written cell
    std::vector<int64_t> adj_off(nb + 1, 0);
    std::vector<int32_t> adj;
    {
        std::vector<int32_t> nbrs;
        for (int32_t b = 0; b < nb; ++b) {
            nbrs.clear();
            for (int32_t e = hp.blk_off[b]; e < hp.blk_off[b + 1]; ++e)
                for (int s = 0; s < arity; ++s) {
                    const int32_t c = wt[int64_t(arity) * e + s];
                    for (int64_t i = cb_off[c]; i < cb_off[c + 1]; ++i)
                        if (cb[i] != b) nbrs.push_back(cb[i]);
                }
            std::sort(nbrs.begin(), nbrs.end());
            nbrs.erase(std::unique(nbrs.begin(), nbrs.end()), nbrs.end());
            adj.insert(adj.end(), nbrs.begin(), nbrs.end());
            adj_off[b + 1] = int64_t(adj.size());
        }
    }
    const int32_t maxcol = o.max_block_colours > 0 ? o.max_block_colours : 256;
    std::vector<int32_t> stamp(maxcol + 1, -1);
    // first-fit over blocks visited in `order`
    auto first_fit = [&](const std::vector<int32_t> &order, std::vector<int32_t> &col) {
        col.assign(nb, -1);
        std::fill(stamp.begin(), stamp.end(), -1);
        int32_t ncol = 0;
        for (int32_t b : order) {
            for (int64_t i = adj_off[b]; i < adj_off[b + 1]; ++i)
                if (col[adj[i]] >= 0) stamp[col[adj[i]]] = b;
            int32_t c = 0;
            while (c < maxcol && stamp[c] == b) ++c;
            if (c >= maxcol)
                fail(UM_ERR_COLOURS, "block colouring needs more than %d colours (block %d of %d)",
                     maxcol, b, nb);
            col[b] = c;
            ncol = std::max(ncol, c + 1);
        }
        return ncol;
    };
    std::vector<int32_t> order(nb);
    std::iota(order.begin(), order.end(), 0);
    int32_t nbcol = first_fit(order, hp.blk_colour);
    if ((o.block_colouring == UM_BCOL_RECOLOUR || o.block_colouring == UM_BCOL_MIN) && nb > 0) {
        // one iterated-greedy pass: colour classes revisited from the last to
        // the first (ties by block id) never need more colours
        std::vector<int32_t> prev = hp.blk_colour;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t x, int32_t y) { return prev[x] > prev[y]; });
        nbcol = first_fit(order, hp.blk_colour);
        if (o.block_colouring == UM_BCOL_MIN) {
            // DSatur, then tabu search for one colour fewer at a time
            std::vector<int32_t> ds;
            const int32_t nds = dsatur(adj_off, adj, ds);
            if (nds > 0 && nds < nbcol) {
                hp.blk_colour = ds;
                nbcol = nds;
            }
            // the bisection's parity code (2^dim colours when the blocks form
            // a regular grid: neighbours differ by one along some axis), its
            // conflicts repaired first-fit in block order
            bool code_won = false;
            if (partition_blocks && is.part_code.size() == size_t(nb)) {
                std::vector<int32_t> pc(is.part_code);
                int32_t npc = 0;
                std::fill(stamp.begin(), stamp.end(), -1);
                for (int32_t b = 0; b < nb; ++b) {
                    bool clash = false;
                    for (int64_t i = adj_off[b]; i < adj_off[b + 1]; ++i)
                        if (adj[i] < b && pc[adj[i]] == pc[b]) clash = true;
                    if (clash) {
                        // every neighbour's colour (repaired or still the code)
                        for (int64_t i = adj_off[b]; i < adj_off[b + 1]; ++i)
                            if (pc[adj[i]] < maxcol) stamp[pc[adj[i]]] = b;
                        int32_t c = 0;
                        while (c < maxcol && stamp[c] == b) ++c;
                        if (c >= maxcol) {
                            npc = maxcol + 1;
                            break;
                        }
                        pc[b] = c;
                    }
                    npc = std::max(npc, pc[b] + 1);
                }
                std::fill(stamp.begin(), stamp.end(), -1);
                if (npc < nbcol) {
                    hp.blk_colour = pc;
                    nbcol = npc;
                    code_won = true;
                }
            }
            std::vector<int32_t> cur = code_won || nds <= 0 ? hp.blk_colour : ds;
            while (nbcol > 1 &&
                   tabu_colouring(adj_off, adj, nbcol - 1, 100 * int64_t(nb) + 100000, cur)) {
                hp.blk_colour = cur;
                --nbcol;
            }
        }
        // balancing: in block order, move a block to the least used colour
        // none of its neighbours holds, if that class is smaller by two or more
        std::vector<int64_t> count(nbcol, 0);
        for (int32_t c : hp.blk_colour) count[c]++;
        for (int32_t b = 0; b < nb; ++b) {
            for (int64_t i = adj_off[b]; i < adj_off[b + 1]; ++i) stamp[hp.blk_colour[adj[i]]] = nb + b;
            const int32_t c = hp.blk_colour[b];
            int32_t best = c;
            for (int32_t k = 0; k < nbcol; ++k)
                if (stamp[k] != nb + b && count[k] < count[best]) best = k;
            if (best != c && count[best] + 1 < count[c]) {
                count[c]--;
                count[best]++;
                hp.blk_colour[b] = best;
            }
        }
        std::fill(stamp.begin(), stamp.end(), -1);
    }
    hp.blk_order = counting_order(hp.blk_colour, nbcol, hp.bcol_off);
    hp.schedule = o.schedule;
    // XCD groups: the blocks are split into G equal ranges of block ids
    // (regions of space, since partition blocks are numbered in bisection
    // order); inside each colour the k-th workgroup of its launch (k = the
    // launch position for the one-launch dataflow schedule, the position
    // within the colour for colour launches) takes the next block of group
    // k mod G, or, once that group has none left in the colour, the next
    // block of the group with most left.  A device that hands consecutive
    // workgroups to its G last-level-cache domains in turn then runs each
    // region on one domain, where a block finds halo lines its neighbours
    // have read.
    const int32_t G = o.xcd_groups;
    std::vector<std::vector<int32_t>> glist(G > 1 ? G : 0);
    std::vector<size_t> gnext(glist.size());
    auto group_interleave = [&](int32_t c) {
        const int32_t p0 = hp.bcol_off[c], p1 = hp.bcol_off[c + 1];
        for (auto &l : glist) l.clear();
        std::fill(gnext.begin(), gnext.end(), 0);
        for (int32_t pos = p0; pos < p1; ++pos) {
            const int32_t b = hp.blk_order[pos];
            glist[int64_t(b) * G / nb].push_back(b);
        }
        const int32_t base = o.schedule == UM_SCHED_DATAFLOW ? 0 : p0;
        for (int32_t pos = p0; pos < p1; ++pos) {
            int32_t g = (pos - base) % G;
            if (gnext[g] == glist[g].size()) {
                size_t most = 0;
                for (int32_t h = 0; h < G; ++h)
                    if (glist[h].size() - gnext[h] > most) {
                        most = glist[h].size() - gnext[h];
                        g = h;
                    }
            }
            hp.blk_order[pos] = glist[g][gnext[g]++];
        }
    };
    if (G > 1 && o.schedule != UM_SCHED_DATAFLOW)
        for (int32_t c = 0; c < nbcol; ++c) group_interleave(c);
    if (o.schedule == UM_SCHED_DATAFLOW) {
        // inside each colour after the first, launch first the blocks whose
        // earlier-coloured neighbours were launched earliest (stable sort by
        // the latest such neighbour's position), so that the blocks the
        // dispatcher starts first rarely find a neighbour still running;
        // XCD groups are interleaved after that sort, colour by colour
        if (G > 1 && nbcol > 0) group_interleave(0);
        std::vector<int32_t> pos_of(nb);
        for (int32_t pos = 0; pos < nb; ++pos) pos_of[hp.blk_order[pos]] = pos;
        std::vector<int32_t> key(nb, -1);
        for (int32_t c = 1; c < nbcol; ++c) {
            const int32_t p0 = hp.bcol_off[c], p1 = hp.bcol_off[c + 1];
            for (int32_t pos = p0; pos < p1; ++pos) {
                const int32_t b = hp.blk_order[pos];
                for (int64_t i = adj_off[b]; i < adj_off[b + 1]; ++i)
                    if (hp.blk_colour[adj[i]] < c) key[b] = std::max(key[b], pos_of[adj[i]]);
            }
            std::stable_sort(hp.blk_order.begin() + p0, hp.blk_order.begin() + p1,
                             [&](int32_t x, int32_t y) { return key[x] < key[y]; });
            if (G > 1) group_interleave(c);
            for (int32_t pos = p0; pos < p1; ++pos) pos_of[hp.blk_order[pos]] = pos;
        }
        // predecessors of a launch position: its neighbours launched earlier,
        // which are exactly its neighbours of smaller colour
        hp.pred_off.assign(nb + 1, 0);
        hp.preds.clear();
        for (int32_t pos = 0; pos < nb; ++pos) {
            const int32_t b = hp.blk_order[pos];
            for (int64_t i = adj_off[b]; i < adj_off[b + 1]; ++i)
                if (pos_of[adj[i]] < pos) hp.preds.push_back(pos_of[adj[i]]);
            hp.pred_off[pos + 1] = int32_t(hp.preds.size());
            if (hp.pred_off[pos + 1] - hp.pred_off[pos] > 64)
                fail(UM_ERR_UNSUPPORTED, "dataflow schedule: block %d waits on more than 64 blocks", b);
        }

    }

    return nbcol;
}

void build_host_plan(const Ctx &ctx, const EdgeArgs &ea, int32_t iter_set,
                     const um_plan_opts &o, HostPlan &hp) {
    const Map &mc = ctx.maps[ea.map_c];
    const Map &mn = ctx.maps[ea.map_n];
    const int64_t E = ctx.sets[iter_set].size;
    const int64_t C = ctx.sets[mc.to].size;
    hp.strategy = o.strategy;
    hp.block_size = o.block_size;
    hp.n_elem = E;
    hp.staging = o.staging;
    hp.tcmode = o.tcmode;
    hp.ept = o.elems_per_thread > 0 ? o.elems_per_thread : 1;
    hp.threads = ((o.block_size + hp.ept - 1) / hp.ept + 63) / 64 * 64;
    hp.n_slots = E;
    auto pack = [&](int64_t e, int32_t *dst) {
        dst[0] = mc.table[2 * e];
        dst[1] = mc.table[2 * e + 1];
        dst[2] = mn.table[2 * e];
        dst[3] = mn.table[2 * e + 1];
    };

    if (o.strategy == UM_STRAT_ATOMIC) {
        hp.emap.resize(4 * E);
        for (int64_t e = 0; e < E; ++e) pack(e, &hp.emap[4 * e]);
        return;
    }
    if (o.strategy == UM_STRAT_GLOBAL_COLOUR) {
        int32_t ncol = global_colours(mc, C, hp.elem_colour);
        std::vector<int32_t> order = counting_order(hp.elem_colour, ncol, hp.colour_off);
        hp.emap.resize(4 * E);
        hp.slot_elem = order;
        for (int64_t s = 0; s < E; ++s) pack(order[s], &hp.emap[4 * s]);
        return;
    }
    if (o.strategy != UM_STRAT_HIER) fail(UM_ERR_ARG, "unknown strategy %d", o.strategy);

    const int32_t nbcol = plan_blocks(ctx, iter_set, mc.table.data(), 2, C, o, hp);
    const int32_t nb = int32_t(hp.blk_off.size()) - 1;

    // ---- per block in launch order: staged lists, layer 2 colouring, slots
    std::vector<int32_t> cloc(C, -1), nloc(ctx.sets[mn.to].size, -1);
    hp.binfo.resize(nb + 1);
    // local index words: one 32-bit word per slot (lL | lR << 11 |
    // nA[0:10) << 22), then one 16-bit half per slot (nA >> 10 | nB << 1 |
    // colour << 12), packed two per 32-bit word: 6 bytes per edge.  Colour
    // code 15 marks an empty slot (padding of wave-pure colour groups), so a
    // block may use at most 15 thread colours.
    std::vector<uint32_t> words;
    std::vector<uint16_t> halves;
    words.reserve(E);
    halves.reserve(E);
    hp.slot_elem.clear();
    hp.slot_elem.reserve(E);
    const bool wave_groups = o.wave_colour_groups != 0;
    hp.wave_groups = wave_groups ? 1 : 0;
    int32_t max_slots = 0;
    hp.tcol.assign(E, 0);
    hp.stg_c.clear();
    hp.stg_n.clear();
    hp.crun.clear();
    hp.nrun.clear();
    hp.use_runs = o.explicit_lists == 0;
    hp.lds_per_colour.assign(nbcol, 0);
    std::vector<int64_t> lds_all(nb);
    std::vector<int32_t> mask, ecol, goff, order;
    int64_t slot = 0, tcol_sum = 0;
    hp.max_tcol = 0;
    for (int32_t pos = 0; pos < nb; ++pos) {
        const int32_t b = hp.blk_order[pos];
        const int32_t e0 = hp.blk_off[b], e1 = hp.blk_off[b + 1], ne = e1 - e0;
        BlockInfo &bi = hp.binfo[pos];
        bi.slot_off = int32_t(slot);
        bi.cell_off = int32_t(hp.stg_c.size());
        bi.node_off = int32_t(hp.stg_n.size());
        const size_t c0 = hp.stg_c.size(), n0 = hp.stg_n.size();
        for (int32_t e = e0; e < e1; ++e) {
            hp.stg_c.push_back(mc.table[2 * int64_t(e)]);
            hp.stg_c.push_back(mc.table[2 * int64_t(e) + 1]);
            hp.stg_n.push_back(mn.table[2 * int64_t(e)]);
            hp.stg_n.push_back(mn.table[2 * int64_t(e) + 1]);
        }
        std::sort(hp.stg_c.begin() + c0, hp.stg_c.end());
        hp.stg_c.erase(std::unique(hp.stg_c.begin() + c0, hp.stg_c.end()), hp.stg_c.end());
        std::sort(hp.stg_n.begin() + n0, hp.stg_n.end());
        hp.stg_n.erase(std::unique(hp.stg_n.begin() + n0, hp.stg_n.end()), hp.stg_n.end());
        const int32_t nc = int32_t(hp.stg_c.size() - c0), nn = int32_t(hp.stg_n.size() - n0);
        for (int32_t i = 0; i < nc; ++i) cloc[hp.stg_c[c0 + i]] = i;
        for (int32_t i = 0; i < nn; ++i) nloc[hp.stg_n[n0 + i]] = i;
        if (nc > 2048 || nn > 2048)
            fail(UM_ERR_UNSUPPORTED, "block %d stages %d cells / %d nodes", b, nc, nn);

        // layer 2: first-fit over the block's edges with per-cell bit masks
        mask.assign(nc, 0);
        ecol.assign(ne, 0);
        int32_t ncol = 0;
        for (int32_t i = 0; i < ne; ++i) {
            const int64_t e = e0 + i;
            const int32_t lL = cloc[mc.table[2 * e]], lR = cloc[mc.table[2 * e + 1]];
            uint32_t taken = uint32_t(mask[lL]) | uint32_t(mask[lR]);
            if ((taken & 0x7FFFu) == 0x7FFFu)
                fail(UM_ERR_UNSUPPORTED, "block %d needs more than 15 thread colours", b);
            int32_t c = __builtin_ctz(~taken);
            ecol[i] = c;
            mask[lL] |= 1 << c;
            mask[lR] |= 1 << c;
            ncol = std::max(ncol, c + 1);
        }
        bi.ncol = ncol;
        // run encoding of the staged lists (sorted, so runs are maximal)
        auto encode = [&](const std::vector<int32_t> &lst, size_t first, size_t n,
                          std::vector<Run> &runs, int32_t &off) {
            off = int32_t(runs.size());
            if (!hp.use_runs) return;
            int32_t nr = 0;
            for (size_t i = 0; i < n; ++i)
                if (i == 0 || lst[first + i] != lst[first + i - 1] + 1) ++nr;
            if (nr > MAX_RUNS) return;
            for (size_t i = 0; i < n; ++i)
                if (i == 0 || lst[first + i] != lst[first + i - 1] + 1)
                    runs.push_back(Run{lst[first + i], int32_t(i)});
        };
        encode(hp.stg_c, c0, nc, hp.crun, bi.crun_off);
        encode(hp.stg_n, n0, nn, hp.nrun, bi.nrun_off);
        tcol_sum += ncol;
        hp.max_tcol = std::max(hp.max_tcol, ncol);
        // slots: the block's edges sorted by colour, stable; with wave-pure
        // groups every colour's run of slots is padded with empty slots to a
        // multiple of 64, so that each wavefront's slots hold one colour
        order = counting_order(ecol, ncol, goff);
        const int64_t slot0 = slot;
        for (int32_t c = 0; c < ncol; ++c) {
            for (int32_t i = goff[c]; i < goff[c + 1]; ++i) {
                const int64_t e = e0 + order[i];
                const uint32_t lL = cloc[mc.table[2 * e]], lR = cloc[mc.table[2 * e + 1]];
                const uint32_t nA = nloc[mn.table[2 * e]], nB = nloc[mn.table[2 * e + 1]];
                words.push_back(lL | (lR << 11) | ((nA & 0x3FFu) << 22));
                halves.push_back(uint16_t((nA >> 10) | (nB << 1) | (uint32_t(c) << 12)));
                hp.slot_elem.push_back(int32_t(e));
                hp.tcol[e] = c;
                ++slot;
            }
            if (wave_groups)
                for (; (slot - slot0) % 64 != 0; ++slot) {
                    words.push_back(0u);
                    halves.push_back(uint16_t(15u << 12));
                    hp.slot_elem.push_back(-1);
                }
        }
        max_slots = std::max(max_slots, int32_t(slot - slot0));
        for (int32_t i = 0; i < nc; ++i) cloc[hp.stg_c[c0 + i]] = -1;
        for (int32_t i = 0; i < nn; ++i) nloc[hp.stg_n[n0 + i]] = -1;
        lds_all[pos] = lf2d_lds_bytes(UM_STAGE_ALL, ea.dtype, nc, nn);
    }
    hp.binfo[nb] = BlockInfo{int32_t(slot), int32_t(hp.stg_c.size()), int32_t(hp.stg_n.size()), 0,
                             int32_t(hp.crun.size()), int32_t(hp.nrun.size()), 0, 0};
    hp.n_slots = slot;
    if (slot > int64_t(INT32_MAX)) fail(UM_ERR_UNSUPPORTED, "too many slots");
    hp.loc.assign(size_t(slot) + size_t(slot + 1) / 2, 0u);
    std::copy(words.begin(), words.end(), hp.loc.begin());
    for (int64_t i = 0; i < slot; ++i)
        hp.loc[size_t(slot) + size_t(i / 2)] |= uint32_t(halves[i]) << (16 * (i & 1));
    if (wave_groups) {
        // lanes: enough for the largest padded block
        hp.threads = ((max_slots + hp.ept - 1) / hp.ept + 63) / 64 * 64;
        if (hp.threads > 1024)
            fail(UM_ERR_ARG, "wave-pure colour groups need %d slots in a block: more than "
                 "1024 lanes at %d elements per lane", max_slots, hp.ept);
        hp.threads = std::max(hp.threads, 64);
    }

    // ---- LDS sizing, with the increments-only fallback
    const int64_t limit = o.lds_limit_bytes > 0 ? o.lds_limit_bytes : ctx.lds_limit;
    int64_t need_all = 0, need_inc = 0;
    for (int32_t pos = 0; pos < nb; ++pos) {
        need_all = std::max(need_all, lds_all[pos]);
        const int64_t nc = hp.binfo[pos + 1].cell_off - hp.binfo[pos].cell_off;
        need_inc = std::max(need_inc, lf2d_lds_bytes(UM_STAGE_INC_ONLY, ea.dtype, nc, 0));
    }
    if (hp.staging == UM_STAGE_ALL && need_all > limit) {
        if (!o.allow_fallback)
            fail(UM_ERR_LDS, "staging all data needs %lld bytes of LDS per block, limit %lld",
                 (long long)need_all, (long long)limit);
        hp.staging = UM_STAGE_INC_ONLY;
    }
    if (hp.schedule == UM_SCHED_DATAFLOW && hp.staging != UM_STAGE_ALL)
        fail(UM_ERR_UNSUPPORTED, "dataflow schedule needs STAGE_ALL staging");
    if (hp.schedule == UM_SCHED_DATAFLOW && 32 * C > int64_t(INT32_MAX))
        fail(UM_ERR_UNSUPPORTED, "dataflow schedule addresses res with 32-bit byte offsets: "
             "at most %lld cells", (long long)(int64_t(INT32_MAX) / 32));
    if (o.gather == UM_GATHER_LDS_DMA && hp.staging != UM_STAGE_ALL)
        fail(UM_ERR_UNSUPPORTED, "LDS-DMA gather needs STAGE_ALL staging");
    if (o.gather == UM_GATHER_LDS_DMA && 16 * ctx.sets[mn.to].size > int64_t(INT32_MAX))
        fail(UM_ERR_UNSUPPORTED, "LDS-DMA gather addresses x with 32-bit byte offsets");
    if (hp.staging == UM_STAGE_INC_ONLY && need_inc > limit)
        fail(UM_ERR_LDS, "staging increments needs %lld bytes of LDS per block, limit %lld",
             (long long)need_inc, (long long)limit);
    hp.lds_max = 0;
    for (int32_t c = 0; c < nbcol; ++c) {
        int64_t m = 0;
        for (int32_t pos = hp.bcol_off[c]; pos < hp.bcol_off[c + 1]; ++pos) {
            const int64_t nc = hp.binfo[pos + 1].cell_off - hp.binfo[pos].cell_off;
            const int64_t nn = hp.binfo[pos + 1].node_off - hp.binfo[pos].node_off;
            m = std::max(m, lf2d_lds_bytes(hp.staging, ea.dtype, nc, nn));
        }
        hp.lds_per_colour[c] = m;
        hp.lds_max = std::max(hp.lds_max, m);
    }
    hp.staged_total = int64_t(hp.stg_c.size() + hp.stg_n.size());
    hp.reuse = hp.stg_c.empty() ? 0.0 : double(2 * E) / double(hp.stg_c.size());
    hp.avg_tcol = nb ? double(tcol_sum) / nb : 0.0;
    if (hp.schedule == UM_SCHED_DATAFLOW) {
        // Blocks the device holds at once, by LDS per compute unit and by its
        // 2048 lanes.  A block whose latest awaited neighbour was launched
        // fewer than 3/4 of that many positions earlier is likely to find it
        // still running; it sums its fluxes in LDS before the wait (sum_first)
        // and afterwards only adds the sums to its cells' residuals, so that
        // a chain of waiting blocks carries only that read-add-write.  The
        // other blocks load their residuals early and accumulate onto them
        // (blocks closer to the whole resident count measured faster so).
        const int64_t per_cu = std::max<int64_t>(
            1, std::min<int64_t>(ctx.lds_per_cu / std::max<int64_t>(hp.lds_max, 1),
                                 2048 / std::max(hp.threads, 64)));
        const int64_t resident = int64_t(ctx.n_cu) * per_cu;
        hp.n_sum_first = 0;
        hp.frec.assign(nb, FlowRec{});
        for (int32_t pos = 0; pos < nb; ++pos) {
            const BlockInfo &a = hp.binfo[pos], &z = hp.binfo[pos + 1];
            FlowRec &r = hp.frec[pos];
            r.slot_off = a.slot_off;
            r.cell_off = a.cell_off;
            r.node_off = a.node_off;
            r.ncol = a.ncol;
            r.ne = z.slot_off - a.slot_off;
            r.nc = z.cell_off - a.cell_off;
            r.nn = z.node_off - a.node_off;
            r.p0 = hp.pred_off[pos];
            r.np = hp.pred_off[pos + 1] - hp.pred_off[pos];
            for (int32_t k = 0; k < r.np && k < 8; ++k) r.preds[k] = hp.preds[r.p0 + k];
            int32_t latest = -1;
            for (int32_t k = 0; k < r.np; ++k) latest = std::max(latest, hp.preds[r.p0 + k]);
            r.sum_first = latest >= 0 && o.sum_first >= 0 &&
                          (o.sum_first == 1 || 4 * (int64_t(pos) - latest) < 3 * resident);
            hp.binfo[pos].sum_first = r.sum_first;
            hp.n_sum_first += r.sum_first;
            r.ncr = z.crun_off - a.crun_off;
            r.nnr = z.nrun_off - a.nrun_off;
            for (int32_t k = 0; k < r.ncr; ++k) r.cruns[k] = hp.crun[a.crun_off + k];
            for (int32_t k = 0; k < r.nnr; ++k) r.nruns[k] = hp.nrun[a.nrun_off + k];
        }
    }
}

}  // namespace um

namespace um {

void build_host_plan_hex(const Ctx &ctx, const HexArgs &ha, int32_t iter_set,
                         const um_plan_opts &o, HostPlan &hp) {
    const Map &m = ctx.maps[ha.map];
    const int64_t E = ctx.sets[iter_set].size;
    const int64_t N = ctx.sets[m.to].size;
    hp.strategy = o.strategy;
    hp.block_size = o.block_size;
    hp.n_elem = E;
    hp.staging = o.staging;
    hp.tcmode = o.tcmode;
    hp.ept = 1;
    hp.threads = (o.block_size + 63) / 64 * 64;
    if (o.strategy == UM_STRAT_ATOMIC) {
        hp.emap = m.table;
        return;
    }
    if (o.strategy == UM_STRAT_GLOBAL_COLOUR) {
        int32_t ncol = global_colours(m, N, hp.elem_colour);
        std::vector<int32_t> order = counting_order(hp.elem_colour, ncol, hp.colour_off);
        hp.emap.resize(8 * E);
        hp.slot_elem = order;
        for (int64_t s = 0; s < E; ++s)
            std::copy(&m.table[8 * int64_t(order[s])], &m.table[8 * int64_t(order[s]) + 8],
                      &hp.emap[8 * s]);
        return;
    }
    if (o.strategy != UM_STRAT_HIER) fail(UM_ERR_ARG, "unknown strategy %d", o.strategy);
    if (o.staging != UM_STAGE_ALL || (o.elems_per_thread > 1))
        fail(UM_ERR_UNSUPPORTED, "hex loop: only STAGE_ALL with one element per lane");
    const int32_t nbcol = plan_blocks(ctx, iter_set, m.table.data(), 8, N, o, hp);
    const int32_t nb = int32_t(hp.blk_off.size()) - 1;
    if (hp.schedule == UM_SCHED_DATAFLOW && 24 * N > int64_t(INT32_MAX))
        fail(UM_ERR_UNSUPPORTED, "dataflow schedule addresses force with 32-bit byte offsets: "
             "at most %lld nodes", (long long)(int64_t(INT32_MAX) / 24));

    // per block in launch order: staged nodes, layer-2 colouring, slots.
    // Local index word: 4 x uint32 per slot holding 8 x 16-bit node indices
    // (< 2048), the thread colour in bits 11..15 of the first one.
    std::vector<int32_t> nloc(N, -1), mask, ecol, goff, order;
    hp.binfo.resize(nb + 1);
    hp.loc.resize(4 * E);
    hp.slot_elem.resize(E);
    hp.tcol.assign(E, 0);
    hp.stg_c.clear(); hp.stg_n.clear(); hp.crun.clear(); hp.nrun.clear();
    hp.use_runs = o.explicit_lists == 0;
    hp.lds_per_colour.assign(nbcol, 0);
    int64_t slot = 0, tcol_sum = 0;
    hp.max_tcol = 0;
    const int64_t limit = o.lds_limit_bytes > 0 ? o.lds_limit_bytes : ctx.lds_limit;
    for (int32_t pos = 0; pos < nb; ++pos) {
        const int32_t b = hp.blk_order[pos];
        const int32_t e0 = hp.blk_off[b], e1 = hp.blk_off[b + 1], ne = e1 - e0;
        BlockInfo &bi = hp.binfo[pos];
        bi = BlockInfo{int32_t(slot), int32_t(hp.stg_c.size()), 0, 0, 0, 0, 0, 0};
        const size_t n0 = hp.stg_c.size();
        hp.stg_c.insert(hp.stg_c.end(), &m.table[8 * int64_t(e0)], &m.table[8 * int64_t(e1)]);
        std::sort(hp.stg_c.begin() + n0, hp.stg_c.end());
        hp.stg_c.erase(std::unique(hp.stg_c.begin() + n0, hp.stg_c.end()), hp.stg_c.end());
        const int32_t nn = int32_t(hp.stg_c.size() - n0);
        if (nn > 2048) fail(UM_ERR_UNSUPPORTED, "hex block %d stages %d nodes (> 2048)", b, nn);
        for (int32_t i = 0; i < nn; ++i) nloc[hp.stg_c[n0 + i]] = i;
        mask.assign(nn, 0);
        ecol.assign(ne, 0);
        int32_t ncol = 0;
        for (int32_t i = 0; i < ne; ++i) {
            const int32_t *row = &m.table[8 * int64_t(e0 + i)];
            uint32_t taken = 0;
            for (int a = 0; a < 8; ++a) taken |= uint32_t(mask[nloc[row[a]]]);
            if (taken == 0xFFFFFFFFu)
                fail(UM_ERR_UNSUPPORTED, "hex block %d needs more than 32 thread colours", b);
            const int32_t c = __builtin_ctz(~taken);
            ecol[i] = c;
            for (int a = 0; a < 8; ++a) mask[nloc[row[a]]] |= 1 << c;
            ncol = std::max(ncol, c + 1);
        }
        bi.ncol = ncol;
        tcol_sum += ncol;
        hp.max_tcol = std::max(hp.max_tcol, ncol);
        order = counting_order(ecol, ncol, goff);
        for (int32_t i = 0; i < ne; ++i) {
            const int64_t e = e0 + order[i];
            const int32_t *row = &m.table[8 * e];
            uint32_t l[8];
            for (int a = 0; a < 8; ++a) l[a] = uint32_t(nloc[row[a]]);
            l[0] |= uint32_t(ecol[order[i]]) << 11;
            for (int w = 0; w < 4; ++w) hp.loc[4 * slot + w] = l[2 * w] | (l[2 * w + 1] << 16);
            hp.slot_elem[slot] = int32_t(e);
            hp.tcol[e] = ecol[order[i]];
            ++slot;
        }
        // run encoding of the staged nodes
        bi.crun_off = int32_t(hp.crun.size());
        if (hp.use_runs) {
            int32_t nr = 0;
            for (int32_t i = 0; i < nn; ++i)
                if (i == 0 || hp.stg_c[n0 + i] != hp.stg_c[n0 + i - 1] + 1) ++nr;
            if (nr <= MAX_RUNS)
                for (int32_t i = 0; i < nn; ++i)
                    if (i == 0 || hp.stg_c[n0 + i] != hp.stg_c[n0 + i - 1] + 1)
                        hp.crun.push_back(Run{hp.stg_c[n0 + i], i});
        }
        for (int32_t i = 0; i < nn; ++i) nloc[hp.stg_c[n0 + i]] = -1;
        const int64_t lds = hex_lds_bytes(nn, hp.schedule == UM_SCHED_DATAFLOW);
        if (lds > limit)
            fail(UM_ERR_LDS, "hex block %d needs %lld bytes of LDS, limit %lld", b,
                 (long long)lds, (long long)limit);
        hp.lds_per_colour[hp.blk_colour[b]] = std::max(hp.lds_per_colour[hp.blk_colour[b]], lds);
    }
    hp.binfo[nb] = BlockInfo{int32_t(slot), int32_t(hp.stg_c.size()), 0, 0,
                             int32_t(hp.crun.size()), 0, 0, 0};
    hp.lds_max = 0;
    for (int64_t v : hp.lds_per_colour) hp.lds_max = std::max(hp.lds_max, v);
    hp.staged_total = int64_t(hp.stg_c.size());
    hp.reuse = hp.stg_c.empty() ? 0.0 : double(8 * E) / double(hp.stg_c.size());
    hp.avg_tcol = nb ? double(tcol_sum) / nb : 0.0;
}

}  // namespace um
