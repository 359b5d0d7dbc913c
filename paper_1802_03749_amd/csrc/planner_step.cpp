// Argument checks and host plans of the other loops of one explicit time
// step of the 2D solver: cell time-step scalar, far-field boundary flux and
// the update with its sum-of-squares reduction (argument patterns in
// umesh.h).  The cell loops need no colouring; the boundary flux increments
// cells that may own several boundary edges, so it is coloured globally or
// run with atomics (Section 2.1).
#include <algorithm>

#include "internal.hpp"

namespace um {

namespace {

struct Want {
    int dim;
    int arity;  // 0: direct; -2: global
    int slot;
    int acc;
    const char *name;
    bool real;  // UM_F64 or UM_F32 (one type for all such args); else UM_F64 only
};

void check_pattern(const Ctx &ctx, const um_arg *args, int32_t nargs, int32_t iter,
                   const Want *want, int n, const char *kname) {
    if (nargs != n || !args) fail(UM_ERR_ARITY, "%s kernel takes %d args, got %d", kname, n, nargs);
    for (int i = 0; i < n; ++i) {
        const um_arg &a = args[i];
        const Want &w = want[i];
        if (a.dat < 0 || a.dat >= int32_t(ctx.dats.size()))
            fail(UM_ERR_RANGE, "arg %d: dat %d does not exist", i, a.dat);
        const Dat &d = ctx.dats[a.dat];
        if (d.dim != w.dim)
            fail(UM_ERR_ARITY, "arg %d: %s needs dim %d, dat has %d", i, w.name, w.dim, d.dim);
        if (!w.real && d.dtype != UM_F64)
            fail(UM_ERR_UNSUPPORTED, "%s kernel: %s must be UM_F64", kname, w.name);
        if (w.real && d.dtype != UM_F64 && d.dtype != UM_F32)
            fail(UM_ERR_UNSUPPORTED, "%s kernel: %s must be UM_F64 or UM_F32", kname, w.name);
        if (a.acc != w.acc) fail(UM_ERR_ARITY, "arg %d: wrong access mode for %s", i, w.name);
        if (w.arity == 0) {
            if (a.map != -1) fail(UM_ERR_ARITY, "arg %d: %s is accessed directly (map -1)", i, w.name);
            if (d.set != iter) fail(UM_ERR_ARITY, "arg %d: %s is not on the iteration set", i, w.name);
            continue;
        }
        if (w.arity == UM_GLOBAL) {
            if (a.map != UM_GLOBAL) fail(UM_ERR_ARITY, "arg %d: %s needs map UM_GLOBAL", i, w.name);
            if (ctx.sets[d.set].size != 1)
                fail(UM_ERR_ARITY, "arg %d: global %s must be on a set of size 1", i, w.name);
            continue;
        }
        if (a.map < 0 || a.map >= int32_t(ctx.maps.size()))
            fail(UM_ERR_ARITY, "arg %d: %s must be accessed through a map", i, w.name);
        const Map &m = ctx.maps[a.map];
        if (m.from != iter) fail(UM_ERR_ARITY, "arg %d: map does not start at the iteration set", i);
        if (m.arity != w.arity)
            fail(UM_ERR_ARITY, "arg %d: map arity %d, need %d", i, m.arity, w.arity);
        if (m.to != d.set) fail(UM_ERR_ARITY, "arg %d: %s is not on the map's to-set", i, w.name);
        if (a.idx != w.slot) fail(UM_ERR_ARITY, "arg %d: %s needs map slot %d", i, w.name, w.slot);
    }
}

void check_layouts(const Ctx &ctx, std::initializer_list<int32_t> ids, const char *kname) {
    const int32_t l = ctx.dats[*ids.begin()].layout;
    for (int32_t id : ids)
        if (ctx.dats[id].layout != l)
            fail(UM_ERR_UNSUPPORTED, "%s kernel: all set dats must share one layout", kname);
}

// x, q and adt share one real type (UM_F64, or UM_F32 for binary32 storage).
int32_t check_real(const Ctx &ctx, std::initializer_list<int32_t> ids, const char *kname) {
    const int32_t t = ctx.dats[*ids.begin()].dtype;
    for (int32_t id : ids)
        if (ctx.dats[id].dtype != t)
            fail(UM_ERR_UNSUPPORTED, "%s kernel: x, q and adt must share one dtype", kname);
    return t;
}

}  // namespace

StepArgs check_step_args(const Ctx &ctx, int32_t kernel, const um_arg *args, int32_t nargs,
                         int32_t iter) {
    StepArgs sa;
    if (kernel == UM_K_CELL_ADT_2D) {
        const Want w[3] = {{2, 4, UM_ALL_SLOTS, UM_READ, "x", true},
                           {4, 0, 0, UM_READ, "q", true},
                           {1, 0, 0, UM_WRITE, "adt", true}};
        check_pattern(ctx, args, nargs, iter, w, 3, "cell adt");
        sa.map_n = args[0].map;
        sa.dat_x = args[0].dat;
        sa.dat_q = args[1].dat;
        sa.dat_adt = args[2].dat;
        check_layouts(ctx, {sa.dat_x, sa.dat_q, sa.dat_adt}, "cell adt");
        sa.dtype = check_real(ctx, {sa.dat_x, sa.dat_q, sa.dat_adt}, "cell adt");
    } else if (kernel == UM_K_BOUNDARY_FLUX_2D) {
        const Want w[5] = {{2, 2, 0, UM_READ, "x", true},
                           {2, 2, 1, UM_READ, "x", true},
                           {4, 1, 0, UM_READ, "q", true},
                           {1, 1, 0, UM_READ, "adt", true},
                           {4, 1, 0, UM_INC, "res", false}};
        check_pattern(ctx, args, nargs, iter, w, 5, "boundary flux");
        if (args[1].dat != args[0].dat || args[1].map != args[0].map)
            fail(UM_ERR_ARITY, "args 0 and 1 must use the same dat and map");
        if (args[3].map != args[2].map || args[4].map != args[2].map)
            fail(UM_ERR_ARITY, "q, adt and res must use the same boundary-edge->cell map");
        sa.map_n = args[0].map;
        sa.map_c = args[2].map;
        sa.dat_x = args[0].dat;
        sa.dat_q = args[2].dat;
        sa.dat_adt = args[3].dat;
        sa.dat_res = args[4].dat;
        check_layouts(ctx, {sa.dat_x, sa.dat_q, sa.dat_adt, sa.dat_res}, "boundary flux");
        sa.dtype = check_real(ctx, {sa.dat_x, sa.dat_q, sa.dat_adt}, "boundary flux");
    } else if (kernel == UM_K_UPDATE_2D) {
        const Want w[4] = {{4, 0, 0, UM_RW, "q", true},
                           {4, 0, 0, UM_RW, "res", false},
                           {1, 0, 0, UM_READ, "adt", true},
                           {1, UM_GLOBAL, 0, UM_INC, "rms", false}};
        check_pattern(ctx, args, nargs, iter, w, 4, "update");
        sa.dat_q = args[0].dat;
        sa.dat_res = args[1].dat;
        sa.dat_adt = args[2].dat;
        sa.dat_rms = args[3].dat;
        if (sa.dat_q == sa.dat_res) fail(UM_ERR_ARITY, "update kernel: q and res must differ");
        check_layouts(ctx, {sa.dat_q, sa.dat_res, sa.dat_adt}, "update");
        sa.dtype = check_real(ctx, {sa.dat_q, sa.dat_adt}, "update");
    } else if (kernel == UM_K_UPDATE_ADT_2D) {
        const Want w[5] = {{4, 0, 0, UM_RW, "q", true},
                           {4, 0, 0, UM_RW, "res", false},
                           {1, 0, 0, UM_RW, "adt", true},
                           {1, UM_GLOBAL, 0, UM_INC, "rms", false},
                           {2, 4, UM_ALL_SLOTS, UM_READ, "x", true}};
        check_pattern(ctx, args, nargs, iter, w, 5, "update + adt");
        sa.dat_q = args[0].dat;
        sa.dat_res = args[1].dat;
        sa.dat_adt = args[2].dat;
        sa.dat_rms = args[3].dat;
        sa.map_n = args[4].map;
        sa.dat_x = args[4].dat;
        if (sa.dat_q == sa.dat_res) fail(UM_ERR_ARITY, "update + adt kernel: q and res must differ");
        check_layouts(ctx, {sa.dat_x, sa.dat_q, sa.dat_res, sa.dat_adt}, "update + adt");
        sa.dtype = check_real(ctx, {sa.dat_x, sa.dat_q, sa.dat_adt}, "update + adt");
    } else {
        fail(UM_ERR_UNSUPPORTED, "unknown kernel %d", kernel);
    }
    sa.layout = ctx.dats[sa.dat_q].layout;
    return sa;
}

void build_host_plan_step(const Ctx &ctx, int32_t kernel, const StepArgs &sa, int32_t iter,
                          const um_plan_opts &o, HostPlan &hp) {
    hp = HostPlan{};
    hp.strategy = o.strategy;
    hp.block_size = o.block_size;
    hp.threads = o.block_size;
    const int64_t n = ctx.sets[iter].size;
    hp.n_elem = n;
    if (kernel == UM_K_CELL_ADT_2D) {
        hp.emap = ctx.maps[sa.map_n].table;  // [C][4] node ids
        return;
    }
    if (kernel == UM_K_UPDATE_2D || kernel == UM_K_UPDATE_ADT_2D) {
        if (o.block_size % 64) fail(UM_ERR_ARG, "update kernel: block_size must be a multiple of 64");
        hp.n_partials = int32_t((n + o.block_size - 1) / o.block_size);
        if (kernel == UM_K_UPDATE_ADT_2D) hp.emap = ctx.maps[sa.map_n].table;  // [C][4] node ids
        return;
    }
    // boundary flux: (cell, a, b, 0) per slot
    if (o.strategy == UM_STRAT_HIER)
        fail(UM_ERR_UNSUPPORTED, "boundary flux kernel: use UM_STRAT_ATOMIC or UM_STRAT_GLOBAL_COLOUR");
    const Map &mc = ctx.maps[sa.map_c], &mn = ctx.maps[sa.map_n];
    auto pack = [&](int64_t e, int32_t *dst) {
        dst[0] = mc.table[e];
        dst[1] = mn.table[2 * e];
        dst[2] = mn.table[2 * e + 1];
        dst[3] = 0;
    };
    hp.emap.resize(4 * n);
    if (o.strategy == UM_STRAT_GLOBAL_COLOUR) {
        const int32_t ncol = global_colours(mc, ctx.sets[mc.to].size, hp.elem_colour);
        hp.slot_elem = counting_order(hp.elem_colour, ncol, hp.colour_off);
        for (int64_t s = 0; s < n; ++s) pack(hp.slot_elem[s], &hp.emap[4 * s]);
    } else {
        for (int64_t e = 0; e < n; ++e) pack(e, &hp.emap[4 * e]);
    }
}

}  // namespace um
