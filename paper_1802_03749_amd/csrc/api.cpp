// C ABI of libumesh: contexts, declarations, reordering, plans, execution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.hpp"
#include "launch.hpp"

struct um_ctx_s : um::Ctx {};
struct um_plan_s : um::Plan {};
struct um_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace um {

// Device memory of um_loop_exec_static: a file-scope array that every GPU the
// library runs on holds until the process ends.  Host code never uses the
// array's name as an address; it uses the device address looked up once per
// device (scratch_address) with that device current.
constexpr int64_t STATIC_SCRATCH_BYTES = 256 * 1024;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {
thread_local std::string g_err;

#define UM_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) fail(UM_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Makes the context's device current for the scope, restoring the previous.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (dev < 0) return;
        UM_HIP(hipGetDevice(&prev));
        if (prev != dev) UM_HIP(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        if (prev >= 0) hipSetDevice(prev);
    }
};

template <typename F>
um_status guarded(F &&f) {
    try {
        f();
        return UM_OK;
    } catch (const Error &e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return UM_ERR_NOMEM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return UM_ERR_ARG;
    }
}

// Device address of `scratch` on `device` (which must be current), looked
// up on the first call for that device and kept.
void *scratch_address(int device) {
    static std::mutex mu;
    static std::vector<void *> addr;
    std::lock_guard<std::mutex> lock(mu);
    if (device >= int(addr.size())) addr.resize(size_t(device) + 1, nullptr);
    if (!addr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            fail(UM_ERR_HIP, "hipGetSymbolAddress of the static scratch on device %d: %s", device,
                 hipGetErrorString(e));
        addr[device] = ptr;
    }
    return addr[device];
}

Ctx &need(um_ctx c) {
    if (!c) fail(UM_ERR_ARG, "null context");
    return *c;
}
Plan &need(um_plan p) {
    if (!p) fail(UM_ERR_ARG, "null plan");
    return *p;
}

template <typename T>
T *upload(const std::vector<T> &v, int64_t &bytes) {
    if (v.empty()) return nullptr;
    T *d = nullptr;
    if (hipMalloc(&d, sizeof(T) * v.size()) != hipSuccess)
        fail(UM_ERR_NOMEM, "device allocation of %zu bytes failed", sizeof(T) * v.size());
    bytes += int64_t(sizeof(T) * v.size());
    UM_HIP(hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return d;
}

void free_device_plan(Plan &p) {
    void *bufs[13] = {p.dp.emap,  p.dp.binfo, p.dp.stg_c,    p.dp.stg_n, p.dp.loc,
                      p.dp.crun,  p.dp.nrun,  p.dp.pred_off, p.dp.preds, p.dp.frec,
                      p.dp.flags, p.dp.err,   p.dp.partials};
    for (void *b : bufs)
        if (b) hipFree(b);
    p.dp = DevicePlan{};
    for (void *e : p.events) hipEventDestroy(static_cast<hipEvent_t>(e));
    p.events.clear();
}

// The kernels move a dat's elements with vector accesses: an AoS element of
// dim * size bytes with 16-byte (or, for 8-byte records, 8-byte) loads, an SoA
// component one value at a time.  A pointer must be aligned to that width.
void check_dat_alignment(const Dat &d, const void *ptr) {
    const int64_t esize = d.dtype == UM_F64 ? 8 : 4;
    int64_t align = esize;
    if (d.layout == UM_AOS) {
        const int64_t rec = esize * d.dim;
        align = rec % 16 == 0 ? 16 : rec % 8 == 0 ? 8 : esize;
    }
    if (reinterpret_cast<uintptr_t>(ptr) % uintptr_t(align) != 0)
        fail(UM_ERR_ARG, "dat pointer %p is not aligned to %lld bytes (dim %d, %s, %s)", ptr,
             (long long)align, d.dim, d.dtype == UM_F64 ? "f64" : "f32",
             d.layout == UM_AOS ? "AoS" : "SoA");
}

int64_t dat_bytes(const Ctx &c, const Dat &d) {
    return c.sets[d.set].size * d.dim * (d.dtype == UM_F64 ? 8 : 4);
}

// An incremented dat must not share memory with a dat the loop reads: the
// kernels read those through non-aliasing (restrict) pointers.
void check_no_overlap(const Ctx &c, int32_t inc, const int32_t *reads, int n, const char *what) {
    const Dat &w = c.dats[inc];
    for (int i = 0; i < n; ++i) {
        if (reads[i] == inc) fail(UM_ERR_ARG, "%s: the incremented dat is also read", what);
        const Dat &r = c.dats[reads[i]];
        if (!w.ptr || !r.ptr) continue;
        const char *a = static_cast<const char *>(w.ptr), *b = static_cast<const char *>(r.ptr);
        if (a < b + dat_bytes(c, r) && b < a + dat_bytes(c, w))
            fail(UM_ERR_ARG, "%s: the incremented dat overlaps a dat the loop reads", what);
    }
}

// LF2D argument pattern (umesh.h, UM_K_EDGE_FLUX_LF2D).
EdgeArgs check_lf2d_args(const Ctx &ctx, const um_arg *args, int32_t nargs, int32_t iter) {
    if (nargs != 8 || !args) fail(UM_ERR_ARITY, "edge flux kernel takes 8 args, got %d", nargs);
    struct Want { int dim, slot, acc; const char *name; };
    const Want want[8] = {{2, 0, UM_READ, "x"},   {2, 1, UM_READ, "x"},  {4, 0, UM_READ, "q"},
                          {4, 1, UM_READ, "q"},   {1, 0, UM_READ, "adt"}, {1, 1, UM_READ, "adt"},
                          {4, 0, UM_INC, "res"},  {4, 1, UM_INC, "res"}};
    for (int i = 0; i < 8; ++i) {
        const um_arg &a = args[i];
        if (a.dat < 0 || a.dat >= int32_t(ctx.dats.size()))
            fail(UM_ERR_RANGE, "arg %d: dat %d does not exist", i, a.dat);
        if (a.map < 0 || a.map >= int32_t(ctx.maps.size()))
            fail(UM_ERR_ARITY, "arg %d: must be accessed through a map", i);
        const Dat &d = ctx.dats[a.dat];
        const Map &m = ctx.maps[a.map];
        if (m.from != iter) fail(UM_ERR_ARITY, "arg %d: map does not start at the iteration set", i);
        if (m.arity != 2) fail(UM_ERR_ARITY, "arg %d: map arity %d, need 2", i, m.arity);
        if (m.to != d.set) fail(UM_ERR_ARITY, "arg %d: dat %s is not on the map's to-set", i, want[i].name);
        if (d.dim != want[i].dim)
            fail(UM_ERR_ARITY, "arg %d: %s needs dim %d, dat has %d", i, want[i].name, want[i].dim, d.dim);
        if (a.idx != want[i].slot) fail(UM_ERR_ARITY, "arg %d: needs map slot %d", i, want[i].slot);
        if (a.acc != want[i].acc) fail(UM_ERR_ARITY, "arg %d: wrong access mode for %s", i, want[i].name);
    }
    EdgeArgs ea;
    ea.map_n = args[0].map;
    ea.map_c = args[2].map;
    ea.dat_x = args[0].dat;
    ea.dat_q = args[2].dat;
    ea.dat_adt = args[4].dat;
    ea.dat_res = args[6].dat;
    for (int i = 0; i < 8; i += 2)
        if (args[i + 1].dat != args[i].dat || args[i + 1].map != args[i].map)
            fail(UM_ERR_ARITY, "args %d and %d must use the same dat and map", i, i + 1);
    if (args[4].map != ea.map_c || args[6].map != ea.map_c)
        fail(UM_ERR_ARITY, "q, adt and res must use the same edge->cell map");
    if (ea.map_n == ea.map_c) fail(UM_ERR_ARITY, "x must use the edge->node map");
    const int ids[4] = {ea.dat_x, ea.dat_q, ea.dat_adt, ea.dat_res};
    ea.layout = ctx.dats[ea.dat_q].layout;
    ea.dtype = ctx.dats[ea.dat_q].dtype;
    for (int id : ids)
        if (ctx.dats[id].layout != ea.layout)
            fail(UM_ERR_UNSUPPORTED, "edge flux kernel: x, q, adt and res must share one layout");
    if (ctx.dats[ea.dat_x].dtype != ea.dtype || ctx.dats[ea.dat_adt].dtype != ea.dtype)
        fail(UM_ERR_UNSUPPORTED, "edge flux kernel: x, q and adt must share one dtype");
    if (ctx.dats[ea.dat_res].dtype != UM_F64)
        fail(UM_ERR_UNSUPPORTED, "edge flux kernel: res must be UM_F64");
    const int32_t reads[3] = {ea.dat_x, ea.dat_q, ea.dat_adt};
    check_no_overlap(ctx, ea.dat_res, reads, 3, "edge flux kernel");
    return ea;
}

// Hex loop argument pattern (umesh.h, UM_K_HEX_HOURGLASS_3D).
HexArgs check_hex_args(const Ctx &ctx, const um_arg *args, int32_t nargs, int32_t iter) {
    if (nargs != 3 || !args) fail(UM_ERR_ARITY, "hex kernel takes 3 args, got %d", nargs);
    const int acc[3] = {UM_READ, UM_READ, UM_INC};
    const char *name[3] = {"x", "v", "force"};
    for (int i = 0; i < 3; ++i) {
        const um_arg &a = args[i];
        if (a.dat < 0 || a.dat >= int32_t(ctx.dats.size()))
            fail(UM_ERR_RANGE, "arg %d: dat %d does not exist", i, a.dat);
        if (a.map < 0 || a.map >= int32_t(ctx.maps.size()))
            fail(UM_ERR_ARITY, "arg %d: must be accessed through a map", i);
        const Dat &d = ctx.dats[a.dat];
        const Map &m = ctx.maps[a.map];
        if (m.from != iter || m.arity != 8)
            fail(UM_ERR_ARITY, "arg %d: needs an arity-8 map from the iteration set", i);
        if (m.to != d.set) fail(UM_ERR_ARITY, "arg %d: %s is not on the map's to-set", i, name[i]);
        if (d.dim != 3) fail(UM_ERR_ARITY, "arg %d: %s needs dim 3", i, name[i]);
        if (a.idx != UM_ALL_SLOTS) fail(UM_ERR_ARITY, "arg %d: needs idx UM_ALL_SLOTS", i);
        if (a.acc != acc[i]) fail(UM_ERR_ARITY, "arg %d: wrong access mode for %s", i, name[i]);
        if (d.dtype != UM_F64) fail(UM_ERR_UNSUPPORTED, "hex kernel: only UM_F64 dats");
        if (a.map != args[0].map) fail(UM_ERR_ARITY, "hex kernel: one map for all args");
        if (d.layout != ctx.dats[args[0].dat].layout)
            fail(UM_ERR_UNSUPPORTED, "hex kernel: x, v and force must share one layout");
    }
    HexArgs ha;
    ha.map = args[0].map;
    ha.dat_x = args[0].dat;
    ha.dat_v = args[1].dat;
    ha.dat_f = args[2].dat;
    ha.layout = ctx.dats[ha.dat_x].layout;
    const int32_t reads[2] = {ha.dat_x, ha.dat_v};
    check_no_overlap(ctx, ha.dat_f, reads, 2, "hex kernel");
    return ha;
}

LaunchArgs launch_args_hex(Plan &p, const double *params, int32_t nparams, void *stream) {
    const Ctx &ctx = *p.ctx;
    if (ctx.device < 0) fail(UM_ERR_STATE, "host-only context cannot execute");
    if (nparams != 1 || !params) fail(UM_ERR_ARG, "hex kernel takes params {kappa}");
    LaunchArgs la{};
    la.stream = static_cast<hipStream_t>(stream);
    la.layout = p.ha.layout;
    la.dtype = UM_F64;
    la.staging = p.hp.staging;
    la.tcmode = p.hp.tcmode;
    la.block_size = p.hp.strategy == UM_STRAT_HIER ? p.hp.threads : p.hp.block_size;
    la.ept = 1;
    la.binfo = p.dp.binfo;
    la.stg_c = p.dp.stg_c;
    la.crun = p.dp.crun;
    la.loc = p.dp.loc;
    la.emap = p.dp.emap;
    const Dat &x = ctx.dats[p.ha.dat_x], &v = ctx.dats[p.ha.dat_v], &f = ctx.dats[p.ha.dat_f];
    if (ctx.sets[p.iter_set].size > 0 && (!x.ptr || !v.ptr || !f.ptr))
        fail(UM_ERR_STATE, "a dat of the loop has no device memory");
    {
        const int32_t reads[2] = {p.ha.dat_x, p.ha.dat_v};
        check_no_overlap(ctx, p.ha.dat_f, reads, 2, "hex kernel");
    }
    la.x = x.ptr;
    la.q = v.ptr;
    la.res = static_cast<double *>(f.ptr);
    la.N = ctx.sets[x.set].size;
    la.gm1 = params[0];
    la.schedule = p.hp.schedule;
    la.pred_off = p.dp.pred_off;
    la.preds = p.dp.preds;
    la.frec = p.dp.frec;
    la.gather = p.hp.gather;
    la.flags = p.dp.flags;
    la.err = p.dp.err;
    la.wait_ticks = p.wait_ticks;
    return la;
}

bool is_step_kernel(int32_t k) {
    return k == UM_K_CELL_ADT_2D || k == UM_K_BOUNDARY_FLUX_2D || k == UM_K_UPDATE_2D ||
           k == UM_K_UPDATE_ADT_2D;
}

LaunchArgs launch_args_step(Plan &p, const double *params, int32_t nparams, void *stream) {
    const Ctx &ctx = *p.ctx;
    if (ctx.device < 0) fail(UM_ERR_STATE, "host-only context cannot execute");
    const int want = (p.kernel == UM_K_CELL_ADT_2D || p.kernel == UM_K_UPDATE_ADT_2D) ? 1
                     : p.kernel == UM_K_BOUNDARY_FLUX_2D                              ? 6
                                                                                      : 0;
    if (nparams != want || (want && !params))
        fail(UM_ERR_ARG, "kernel %d takes %d params, got %d", p.kernel, want, nparams);
    LaunchArgs la{};
    la.stream = static_cast<hipStream_t>(stream);
    la.layout = p.sa.layout;
    la.dtype = p.sa.dtype;
    la.block_size = p.hp.block_size;
    la.emap = p.dp.emap;
    const StepArgs &sa = p.sa;
    const int ids[5] = {sa.dat_x, sa.dat_q, sa.dat_adt, sa.dat_res, sa.dat_rms};
    if (ctx.sets[p.iter_set].size > 0)
        for (int id : ids)
            if (id >= 0 && !ctx.dats[id].ptr) fail(UM_ERR_STATE, "a dat of the loop has no device memory");
    if (sa.dat_x >= 0) {
        la.x = ctx.dats[sa.dat_x].ptr;
        la.N = ctx.sets[ctx.dats[sa.dat_x].set].size;
    }
    la.q = ctx.dats[sa.dat_q].ptr;
    la.C = ctx.sets[ctx.dats[sa.dat_q].set].size;
    la.adt = ctx.dats[sa.dat_adt].ptr;
    if (sa.dat_res >= 0) la.res = static_cast<double *>(ctx.dats[sa.dat_res].ptr);
    if (sa.dat_rms >= 0) la.gbl = static_cast<double *>(ctx.dats[sa.dat_rms].ptr);
    la.partials = p.dp.partials;
    la.n_partials = p.hp.n_partials;
    if (want >= 1) la.gm1 = params[0];
    if (want == 6) {
        la.eps = params[1];
        for (int k = 0; k < 4; ++k) la.qinf[k] = params[2 + k];
    }
    return la;
}

LaunchArgs launch_args(Plan &p, const double *params, int32_t nparams, void *stream) {
    if (p.kernel == UM_K_HEX_HOURGLASS_3D) return launch_args_hex(p, params, nparams, stream);
    if (is_step_kernel(p.kernel)) return launch_args_step(p, params, nparams, stream);
    const Ctx &ctx = *p.ctx;
    if (ctx.device < 0) fail(UM_ERR_STATE, "host-only context cannot execute");
    if (nparams != 2 || !params) fail(UM_ERR_ARG, "edge flux kernel takes params {gm1, eps}");
    LaunchArgs la{};
    la.stream = static_cast<hipStream_t>(stream);
    la.layout = p.ea.layout;
    la.staging = p.hp.staging;
    la.tcmode = p.hp.tcmode;
    la.block_size = p.hp.strategy == UM_STRAT_HIER ? p.hp.threads : p.hp.block_size;
    la.ept = p.hp.ept;
    la.binfo = p.dp.binfo;
    la.stg_c = p.dp.stg_c;
    la.stg_n = p.dp.stg_n;
    la.crun = p.dp.crun;
    la.nrun = p.dp.nrun;
    la.loc = p.dp.loc;
    la.n_slots = p.hp.n_slots;
    la.emap = p.dp.emap;
    const Dat &x = ctx.dats[p.ea.dat_x], &q = ctx.dats[p.ea.dat_q];
    const Dat &adt = ctx.dats[p.ea.dat_adt], &res = ctx.dats[p.ea.dat_res];
    const int64_t E = ctx.sets[p.iter_set].size;
    if (E > 0 && (!x.ptr || !q.ptr || !adt.ptr || !res.ptr))
        fail(UM_ERR_STATE, "a dat of the loop has no device memory");
    {
        const int32_t reads[3] = {p.ea.dat_x, p.ea.dat_q, p.ea.dat_adt};
        check_no_overlap(ctx, p.ea.dat_res, reads, 3, "edge flux kernel");
    }
    la.dtype = p.ea.dtype;
    la.x = x.ptr;
    la.q = q.ptr;
    la.adt = adt.ptr;
    la.res = static_cast<double *>(res.ptr);
    la.N = ctx.sets[x.set].size;
    la.C = ctx.sets[q.set].size;
    la.gm1 = params[0];
    la.eps = params[1];
    la.schedule = p.hp.schedule;
    la.pred_off = p.dp.pred_off;
    la.preds = p.dp.preds;
    la.frec = p.dp.frec;
    la.gather = p.hp.gather;
    la.sum_first = p.hp.n_sum_first > 0;
    la.flags = p.dp.flags;
    la.err = p.dp.err;
    la.wait_ticks = p.wait_ticks;
    return la;
}

}  // namespace

void fail(um_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error{code, buf};
}

}  // namespace um

using namespace um;

extern "C" {

int32_t um_abi_version(void) { return UMESH_ABI_VERSION; }

const char *um_last_error(void) { return g_err.c_str(); }

um_status um_create(int32_t device, um_ctx *out) {
    return guarded([&] {
        if (!out) fail(UM_ERR_ARG, "null output handle");
        *out = nullptr;
        if (device < -1) fail(UM_ERR_ARG, "device %d", device);
        auto *c = new um_ctx_s();
        c->device = device;
        if (device >= 0) {
            int n = 0;
            if (hipGetDeviceCount(&n) != hipSuccess || device >= n) {
                delete c;
                fail(UM_ERR_HIP, "HIP device %d not available (%d devices)", device, n);
            }
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
                delete c;
                fail(UM_ERR_HIP, "cannot query HIP device %d", device);
            }
            c->lds_limit = int32_t(prop.sharedMemPerBlock);
            c->n_cu = prop.multiProcessorCount;
            c->lds_per_cu = int64_t(prop.maxSharedMemoryPerMultiProcessor);
            try {
                DeviceGuard g(device);
                (void)scratch_address(device);
            } catch (...) {
                delete c;
                throw;
            }
        }
        *out = c;
    });
}

um_status um_destroy(um_ctx ctx) {
    return guarded([&] {
        if (!ctx) return;
        DeviceGuard g(ctx->device);
        if (ctx->device >= 0) hipDeviceSynchronize();
        for (Plan *p : ctx->plans) {
            free_device_plan(*p);
            delete static_cast<um_plan_s *>(p);
        }
        for (int32_t *d : ctx->d_new2orig)
            if (d) hipFree(d);
        for (int32_t *d : ctx->d_orig2new)
            if (d) hipFree(d);
        delete ctx;
    });
}

um_status um_decl_set(um_ctx ctx, int64_t size, const char *name, int32_t *set_id) {
    return guarded([&] {
        Ctx &c = need(ctx);
        if (!set_id) fail(UM_ERR_ARG, "null set_id");
        if (size < 0 || size > INT32_MAX) fail(UM_ERR_ARG, "set size %lld", (long long)size);
        Set s;
        s.size = size;
        s.name = name ? name : "";
        s.new2orig.resize(size);
        for (int64_t k = 0; k < size; ++k) s.new2orig[k] = int32_t(k);
        c.sets.push_back(std::move(s));
        c.d_new2orig.push_back(nullptr);
        c.d_orig2new.push_back(nullptr);
        *set_id = int32_t(c.sets.size()) - 1;
    });
}

um_status um_decl_map(um_ctx ctx, int32_t from_set, int32_t to_set, int32_t arity,
                      const int32_t *host_table, int32_t *map_id) {
    return guarded([&] {
        Ctx &c = need(ctx);
        if (!map_id) fail(UM_ERR_ARG, "null map_id");
        const int32_t ns = int32_t(c.sets.size());
        if (from_set < 0 || from_set >= ns || to_set < 0 || to_set >= ns)
            fail(UM_ERR_ARG, "bad set id (%d, %d)", from_set, to_set);
        if (arity < 1 || arity > 16) fail(UM_ERR_ARG, "arity %d outside 1..16", arity);
        const int64_t n = c.sets[from_set].size * arity, to_n = c.sets[to_set].size;
        if (n > 0 && !host_table) fail(UM_ERR_ARG, "null map table");
        for (int64_t i = 0; i < n; ++i)
            if (host_table[i] < 0 || host_table[i] >= to_n)
                fail(UM_ERR_RANGE, "map entry %lld (element %lld, slot %lld) = %d outside 0..%lld",
                     (long long)i, (long long)(i / arity), (long long)(i % arity), host_table[i],
                     (long long)to_n - 1);
        Map m;
        m.from = from_set;
        m.to = to_set;
        m.arity = arity;
        m.table.assign(host_table, host_table + n);
        c.maps.push_back(std::move(m));
        *map_id = int32_t(c.maps.size()) - 1;
    });
}

um_status um_decl_dat(um_ctx ctx, int32_t set, int32_t dim, int32_t dtype, int32_t layout,
                      void *device_ptr, int32_t *dat_id) {
    return guarded([&] {
        Ctx &c = need(ctx);
        if (!dat_id) fail(UM_ERR_ARG, "null dat_id");
        if (set < 0 || set >= int32_t(c.sets.size())) fail(UM_ERR_ARG, "bad set id %d", set);
        if (dim < 1 || dim > 16) fail(UM_ERR_ARG, "dim %d outside 1..16", dim);
        if (dtype != UM_F64 && dtype != UM_F32) fail(UM_ERR_ARG, "bad dtype %d", dtype);
        if (layout != UM_AOS && layout != UM_SOA) fail(UM_ERR_ARG, "bad layout %d", layout);
        Dat d;
        d.set = set;
        d.dim = dim;
        d.dtype = dtype;
        d.layout = layout;
        check_dat_alignment(d, device_ptr);
        d.ptr = device_ptr;
        c.dats.push_back(d);
        *dat_id = int32_t(c.dats.size()) - 1;
    });
}

um_status um_set_dat_ptr(um_ctx ctx, int32_t dat, void *device_ptr) {
    return guarded([&] {
        Ctx &c = need(ctx);
        if (dat < 0 || dat >= int32_t(c.dats.size())) fail(UM_ERR_ARG, "bad dat id %d", dat);
        check_dat_alignment(c.dats[dat], device_ptr);
        c.dats[dat].ptr = device_ptr;
    });
}

um_status um_reorder_mesh(um_ctx ctx, const um_reorder_opts *opts) {
    return guarded([&] {
        Ctx &c = need(ctx);
        if (!opts) fail(UM_ERR_ARG, "null options");
        if (!c.dats.empty() || !c.plans.empty())
            fail(UM_ERR_STATE, "reorder before declaring dats or building plans");
        reorder_mesh(c, *opts);
        // device copies of permutations are stale now
        DeviceGuard g(c.device);
        for (size_t s = 0; s < c.sets.size(); ++s) {
            if (c.d_new2orig[s]) hipFree(c.d_new2orig[s]);
            if (c.d_orig2new[s]) hipFree(c.d_orig2new[s]);
            c.d_new2orig[s] = c.d_orig2new[s] = nullptr;
        }
    });
}

um_status um_get_perm(um_ctx ctx, int32_t set, int32_t *out) {
    return guarded([&] {
        Ctx &c = need(ctx);
        if (set < 0 || set >= int32_t(c.sets.size()) || !out) fail(UM_ERR_ARG, "bad set or output");
        std::copy(c.sets[set].new2orig.begin(), c.sets[set].new2orig.end(), out);
    });
}

um_status um_get_map(um_ctx ctx, int32_t map, int32_t *out) {
    return guarded([&] {
        Ctx &c = need(ctx);
        if (map < 0 || map >= int32_t(c.maps.size()) || !out) fail(UM_ERR_ARG, "bad map or output");
        std::copy(c.maps[map].table.begin(), c.maps[map].table.end(), out);
    });
}

um_status um_get_blocks(um_ctx ctx, int32_t set, int32_t *block_size, int32_t *n_blocks,
                        int32_t *host_off, int64_t capacity) {
    return guarded([&] {
        Ctx &c = need(ctx);
        if (set < 0 || set >= int32_t(c.sets.size()) || !n_blocks || !block_size)
            fail(UM_ERR_ARG, "bad set or output");
        const Set &s = c.sets[set];
        *block_size = s.part_block_size;
        *n_blocks = s.part_off.empty() ? 0 : int32_t(s.part_off.size()) - 1;
        if (host_off) {
            if (capacity < int64_t(s.part_off.size())) fail(UM_ERR_ARG, "capacity too small");
            std::copy(s.part_off.begin(), s.part_off.end(), host_off);
        }
    });
}

um_status um_permute_dat(um_ctx ctx, int32_t set, int32_t direction, const void *src, void *dst,
                         int32_t dim, int32_t dtype, int32_t layout, void *stream) {
    return guarded([&] {
        Ctx &c = need(ctx);
        if (c.device < 0) fail(UM_ERR_STATE, "host-only context has no device");
        if (set < 0 || set >= int32_t(c.sets.size())) fail(UM_ERR_ARG, "bad set id %d", set);
        if (direction != 0 && direction != 1) fail(UM_ERR_ARG, "direction must be 0 or 1");
        if (dim < 1 || dim > 16 || (dtype != UM_F64 && dtype != UM_F32) ||
            (layout != UM_AOS && layout != UM_SOA))
            fail(UM_ERR_ARG, "bad dim/dtype/layout");
        const Set &s = c.sets[set];
        if (s.size == 0) return;
        if (!src || !dst || src == dst) fail(UM_ERR_ARG, "src and dst must be distinct buffers");
        DeviceGuard g(c.device);
        int32_t *&d_n2o = c.d_new2orig[set];
        int32_t *&d_o2n = c.d_orig2new[set];
        if (!d_n2o) {
            std::vector<int32_t> inv(s.size);
            for (int64_t k = 0; k < s.size; ++k) inv[s.new2orig[k]] = int32_t(k);
            int64_t bytes = 0;
            d_n2o = upload(s.new2orig, bytes);
            d_o2n = upload(inv, bytes);
        }
        // direction 0: dst[k] = src[new2orig[k]]; 1: dst[j] = src[orig2new[j]]
        UM_HIP(permute_gather(src, dst, direction == 0 ? d_n2o : d_o2n, s.size, dim, dtype, layout,
                              static_cast<hipStream_t>(stream)));
    });
}

um_status um_plan_build(um_ctx ctx, int32_t kernel, const um_arg *args, int32_t nargs,
                        int32_t iter_set, const um_plan_opts *opts, um_plan *out) {
    return guarded([&] {
        Ctx &c = need(ctx);
        if (!out || !opts) fail(UM_ERR_ARG, "null options or output");
        *out = nullptr;
        if (kernel != UM_K_EDGE_FLUX_LF2D && kernel != UM_K_HEX_HOURGLASS_3D &&
            !is_step_kernel(kernel))
            fail(UM_ERR_UNSUPPORTED, "unknown kernel %d", kernel);
        if (iter_set < 0 || iter_set >= int32_t(c.sets.size())) fail(UM_ERR_ARG, "bad iteration set");
        const um_plan_opts &o = *opts;
        if (o.strategy < UM_STRAT_ATOMIC || o.strategy > UM_STRAT_HIER)
            fail(UM_ERR_ARG, "bad strategy %d", o.strategy);
        if (o.block_size < 64 || o.block_size > 1024)
            fail(UM_ERR_ARG, "block_size %d outside 64..1024", o.block_size);
        if (o.staging != UM_STAGE_ALL && o.staging != UM_STAGE_INC_ONLY)
            fail(UM_ERR_ARG, "bad staging %d", o.staging);
        if (o.tcmode != UM_TC_BARRIER && o.tcmode != UM_TC_LDS_ATOMIC)
            fail(UM_ERR_ARG, "bad tcmode %d", o.tcmode);
        if (o.max_block_colours < 0 || o.lds_limit_bytes < 0) fail(UM_ERR_ARG, "negative limit");
        if (o.elems_per_thread != 0 && o.elems_per_thread != 1 && o.elems_per_thread != 2)
            fail(UM_ERR_ARG, "elems_per_thread %d not in {1, 2}", o.elems_per_thread);
        if (o.block_colouring != UM_BCOL_FIRST_FIT && o.block_colouring != UM_BCOL_RECOLOUR &&
            o.block_colouring != UM_BCOL_MIN)
            fail(UM_ERR_ARG, "bad block_colouring %d", o.block_colouring);
        if (o.schedule != UM_SCHED_COLOUR_LAUNCHES && o.schedule != UM_SCHED_DATAFLOW)
            fail(UM_ERR_ARG, "bad schedule %d", o.schedule);
        if (o.gather != UM_GATHER_REGISTERS && o.gather != UM_GATHER_LDS_DMA)
            fail(UM_ERR_ARG, "bad gather %d", o.gather);
        if (o.wave_colour_groups != 0 && o.wave_colour_groups != 1)
            fail(UM_ERR_ARG, "wave_colour_groups must be 0 or 1");
        if (o.wave_colour_groups != 0 &&
            (kernel != UM_K_EDGE_FLUX_LF2D || o.strategy != UM_STRAT_HIER))
            fail(UM_ERR_UNSUPPORTED, "wave-pure colour groups: HIER plans of the edge loop only");
        if (o.xcd_groups < 0 || o.xcd_groups > 64)
            fail(UM_ERR_ARG, "xcd_groups %d outside 0..64", o.xcd_groups);
        if (o.sum_first < -1 || o.sum_first > 1)
            fail(UM_ERR_ARG, "sum_first %d not in {-1, 0, 1}", o.sum_first);
        if (o.xcd_groups > 1 && (is_step_kernel(kernel) || o.strategy != UM_STRAT_HIER))
            fail(UM_ERR_UNSUPPORTED, "XCD groups: HIER plans of the edge and hex loops only");
        const auto t0 = std::chrono::steady_clock::now();
        auto *p = new um_plan_s();
        p->ctx = &c;
        p->kernel = kernel;
        p->iter_set = iter_set;
        try {
            if (kernel == UM_K_EDGE_FLUX_LF2D) {
                p->ea = check_lf2d_args(c, args, nargs, iter_set);
                if (o.gather == UM_GATHER_LDS_DMA &&
                    (o.strategy != UM_STRAT_HIER || o.schedule != UM_SCHED_DATAFLOW ||
                     p->ea.layout != UM_AOS))
                    fail(UM_ERR_UNSUPPORTED,
                         "LDS-DMA gather: HIER plans with the DATAFLOW schedule on AoS data only");
                build_host_plan(c, p->ea, iter_set, o, p->hp);
                p->hp.gather = o.gather;
            } else if (is_step_kernel(kernel)) {
                if (o.gather != UM_GATHER_REGISTERS)
                    fail(UM_ERR_UNSUPPORTED, "LDS-DMA gather: edge flux loop only");
                p->sa = check_step_args(c, kernel, args, nargs, iter_set);
                build_host_plan_step(c, kernel, p->sa, iter_set, o, p->hp);
            } else {
                if (o.gather != UM_GATHER_REGISTERS)
                    fail(UM_ERR_UNSUPPORTED, "LDS-DMA gather: edge flux loop only");
                p->ha = check_hex_args(c, args, nargs, iter_set);
                build_host_plan_hex(c, p->ha, iter_set, o, p->hp);
            }
            if (c.device >= 0) {
                DeviceGuard g(c.device);
                int64_t bytes = 0;
                p->dp.emap = upload(p->hp.emap, bytes);
                p->dp.binfo = upload(p->hp.binfo, bytes);
                p->dp.stg_c = upload(p->hp.stg_c, bytes);
                p->dp.stg_n = upload(p->hp.stg_n, bytes);
                p->dp.crun = upload(p->hp.crun, bytes);
                p->dp.nrun = upload(p->hp.nrun, bytes);
                p->dp.loc = upload(p->hp.loc, bytes);
                if (p->hp.schedule == UM_SCHED_DATAFLOW && !p->hp.binfo.empty()) {
                    p->dp.pred_off = upload(p->hp.pred_off, bytes);
                    p->dp.preds = upload(p->hp.preds, bytes);
                    p->dp.frec = upload(p->hp.frec, bytes);
                    std::vector<int32_t> zeros(p->hp.binfo.size(), 0);
                    p->dp.flags = upload(zeros, bytes);
                    std::vector<int32_t> ctl(4, 0);
                    p->dp.err = upload(ctl, bytes);
                }
                if (p->hp.n_partials > 0) {
                    std::vector<double> zeros(p->hp.n_partials, 0.0);
                    p->dp.partials = upload(zeros, bytes);
                }
                p->dp.bytes = bytes;
                UM_HIP(hipDeviceSynchronize());
            }
        } catch (...) {
            DeviceGuard g(c.device);
            free_device_plan(*p);
            delete p;
            throw;
        }
        p->build_seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        c.plans.push_back(p);
        *out = p;
    });
}

um_status um_plan_stats_get(um_plan plan, um_plan_stats *out) {
    return guarded([&] {
        Plan &p = need(plan);
        if (!out) fail(UM_ERR_ARG, "null output");
        std::memset(out, 0, sizeof *out);
        const HostPlan &hp = p.hp;
        out->strategy = hp.strategy;
        out->staging = hp.staging;
        out->block_size = hp.block_size;
        out->n_elements = hp.n_elem;
        out->plan_device_bytes = p.dp.bytes;
        out->build_seconds = p.build_seconds;
        if (is_step_kernel(p.kernel)) {
            if (p.kernel == UM_K_BOUNDARY_FLUX_2D && hp.strategy == UM_STRAT_GLOBAL_COLOUR) {
                out->n_global_colours = int32_t(hp.colour_off.size()) - 1;
                out->n_launches = out->n_global_colours;
            } else {
                const bool two = p.kernel == UM_K_UPDATE_2D || p.kernel == UM_K_UPDATE_ADT_2D;
                out->n_launches = hp.n_elem > 0 ? (two ? 2 : 1) : 0;
            }
        } else if (hp.strategy == UM_STRAT_HIER) {
            out->n_blocks = int32_t(hp.blk_colour.size());
            out->n_block_colours = int32_t(hp.bcol_off.size()) - 1;
            out->max_thread_colours = hp.max_tcol;
            out->avg_thread_colours = hp.avg_tcol;
            out->reuse_factor = hp.reuse;
            out->staged_points = hp.staged_total;
            out->lds_bytes_max = hp.lds_max;
            out->n_sum_first_blocks = hp.n_sum_first;
            out->n_launches = 0;
            for (int32_t c = 0; c + 1 < int32_t(hp.bcol_off.size()); ++c)
                out->n_launches += hp.bcol_off[c + 1] > hp.bcol_off[c];
            if (hp.schedule == UM_SCHED_DATAFLOW) out->n_launches = out->n_launches > 0;
        } else if (hp.strategy == UM_STRAT_GLOBAL_COLOUR) {
            out->n_global_colours = int32_t(hp.colour_off.size()) - 1;
            out->n_launches = out->n_global_colours;
        } else {
            out->n_launches = hp.n_elem > 0;
        }
    });
}

um_status um_plan_export(um_plan plan, int32_t field, int32_t *host_out, int64_t capacity,
                         int64_t *n_out) {
    return guarded([&] {
        Plan &p = need(plan);
        if (!n_out) fail(UM_ERR_ARG, "null n_out");
        const HostPlan &hp = p.hp;
        const Ctx &c = *p.ctx;
        std::vector<int32_t> tmp;
        const std::vector<int32_t> *v = &tmp;
        const bool hier = hp.strategy == UM_STRAT_HIER && !is_step_kernel(p.kernel);
        if (is_step_kernel(p.kernel) &&
            !(p.kernel == UM_K_BOUNDARY_FLUX_2D && hp.strategy == UM_STRAT_GLOBAL_COLOUR &&
              (field == UM_EXP_SLOT_ELEMENTS || field == UM_EXP_GLOBAL_COLOURS)))
            fail(UM_ERR_STATE, "field %d is not defined for kernel %d", field, p.kernel);
        auto staged = [&](bool cells, bool offsets) {
            // block id order
            const int32_t nb = int32_t(hp.blk_order.size());
            std::vector<int32_t> pos_of(nb);
            for (int32_t pos = 0; pos < nb; ++pos) pos_of[hp.blk_order[pos]] = pos;
            tmp.clear();
            if (offsets) tmp.push_back(0);
            for (int32_t b = 0; b < nb; ++b) {
                const int32_t pos = pos_of[b];
                const int32_t s0 = cells ? hp.binfo[pos].cell_off : hp.binfo[pos].node_off;
                const int32_t s1 = cells ? hp.binfo[pos + 1].cell_off : hp.binfo[pos + 1].node_off;
                if (offsets)
                    tmp.push_back(tmp.back() + (s1 - s0));
                else
                    for (int32_t i = s0; i < s1; ++i)
                        tmp.push_back(cells ? hp.stg_c[i] : hp.stg_n[i]);
            }
        };
        auto runs = [&](bool cells, bool offsets) {
            const int32_t nb = int32_t(hp.blk_order.size());
            std::vector<int32_t> pos_of(nb);
            for (int32_t pos = 0; pos < nb; ++pos) pos_of[hp.blk_order[pos]] = pos;
            const std::vector<Run> &rv = cells ? hp.crun : hp.nrun;
            tmp.clear();
            if (offsets) tmp.push_back(0);
            for (int32_t b = 0; b < nb; ++b) {
                const BlockInfo &a = hp.binfo[pos_of[b]], &z = hp.binfo[pos_of[b] + 1];
                const int32_t r0 = cells ? a.crun_off : a.nrun_off;
                const int32_t r1 = cells ? z.crun_off : z.nrun_off;
                if (offsets)
                    tmp.push_back(tmp.back() + (r1 - r0));
                else
                    for (int32_t r = r0; r < r1; ++r) {
                        tmp.push_back(rv[r].start);
                        tmp.push_back(rv[r].local);
                    }
            }
        };
        switch (field) {
        case UM_EXP_RUN_OFFSETS_A: if (!hier) fail(UM_ERR_STATE, "not a HIER plan"); runs(false, true); break;
        case UM_EXP_RUNS_A: if (!hier) fail(UM_ERR_STATE, "not a HIER plan"); runs(false, false); break;
        case UM_EXP_RUN_OFFSETS_B: if (!hier) fail(UM_ERR_STATE, "not a HIER plan"); runs(true, true); break;
        case UM_EXP_RUNS_B: if (!hier) fail(UM_ERR_STATE, "not a HIER plan"); runs(true, false); break;
        case UM_EXP_BLOCK_OFFSETS: if (!hier) fail(UM_ERR_STATE, "not a HIER plan"); v = &hp.blk_off; break;
        case UM_EXP_BLOCK_COLOURS: if (!hier) fail(UM_ERR_STATE, "not a HIER plan"); v = &hp.blk_colour; break;
        case UM_EXP_THREAD_COLOURS: if (!hier) fail(UM_ERR_STATE, "not a HIER plan"); v = &hp.tcol; break;
        case UM_EXP_BLOCK_ORDER: if (!hier) fail(UM_ERR_STATE, "not a HIER plan"); v = &hp.blk_order; break;
        case UM_EXP_PRED_OFFSETS:
        case UM_EXP_PREDS:
            if (!hier || hp.schedule != UM_SCHED_DATAFLOW) fail(UM_ERR_STATE, "not a DATAFLOW plan");
            v = field == UM_EXP_PREDS ? &hp.preds : &hp.pred_off;
            break;
        case UM_EXP_SLOT_ELEMENTS:
            if (hp.strategy == UM_STRAT_ATOMIC) fail(UM_ERR_STATE, "atomic plans run elements in order");
            v = &hp.slot_elem;
            break;
        case UM_EXP_GLOBAL_COLOURS:
            if (hp.strategy != UM_STRAT_GLOBAL_COLOUR) fail(UM_ERR_STATE, "not a GLOBAL_COLOUR plan");
            v = &hp.elem_colour;
            break;
        case UM_EXP_STAGED_OFFSETS_A: if (!hier) fail(UM_ERR_STATE, "not a HIER plan"); staged(false, true); break;
        case UM_EXP_STAGED_POINTS_A: if (!hier) fail(UM_ERR_STATE, "not a HIER plan"); staged(false, false); break;
        case UM_EXP_STAGED_OFFSETS_B: if (!hier) fail(UM_ERR_STATE, "not a HIER plan"); staged(true, true); break;
        case UM_EXP_STAGED_POINTS_B: if (!hier) fail(UM_ERR_STATE, "not a HIER plan"); staged(true, false); break;
        case UM_EXP_LOCAL_INDEX:
            if (!hier) fail(UM_ERR_STATE, "not a HIER plan");
            if (p.kernel == UM_K_HEX_HOURGLASS_3D) {
                tmp.resize(8 * hp.n_elem);
                for (int64_t s = 0; s < hp.n_elem; ++s)
                    for (int w = 0; w < 4; ++w) {
                        const uint32_t v = hp.loc[4 * s + w];
                        tmp[8 * s + 2 * w] = int32_t(w == 0 ? (v & 0x7FFu) : (v & 0xFFFFu));
                        tmp[8 * s + 2 * w + 1] = int32_t(v >> 16);
                    }
                break;
            }
            tmp.resize(4 * hp.n_slots);
            for (int64_t s = 0; s < hp.n_slots; ++s) {
                const uint32_t a = hp.loc[s];
                const uint32_t h = (hp.loc[hp.n_slots + s / 2] >> (16 * (s & 1))) & 0xFFFFu;
                tmp[4 * s] = int32_t(a & 0x7FFu);
                tmp[4 * s + 1] = int32_t((a >> 11) & 0x7FFu);
                tmp[4 * s + 2] = int32_t(((a >> 22) & 0x3FFu) | ((h & 1u) << 10));
                tmp[4 * s + 3] = int32_t((h >> 1) & 0x7FFu);
            }
            break;
        default: fail(UM_ERR_ARG, "unknown export field %d", field);
        }
        (void)c;
        *n_out = int64_t(v->size());
        if (host_out) {
            if (capacity < *n_out) fail(UM_ERR_ARG, "capacity %lld < %lld", (long long)capacity, (long long)*n_out);
            std::copy(v->begin(), v->end(), host_out);
        }
    });
}

um_status um_plan_destroy(um_plan plan) {
    return guarded([&] {
        if (!plan) return;
        Ctx &c = *plan->ctx;
        DeviceGuard g(c.device);
        if (c.device >= 0) hipDeviceSynchronize();
        free_device_plan(*plan);
        c.plans.erase(std::remove(c.plans.begin(), c.plans.end(), static_cast<Plan *>(plan)),
                      c.plans.end());
        delete plan;
    });
}

}  // extern "C"

namespace um {
namespace {

// Executes the plan once.  With use_static, the plan's scratch buffers (the
// DATAFLOW completion flags and control words, the UPDATE partial sums) are
// replaced by the static scratch array of the plan's device: the flags and
// control words are cleared by a kernel first (every execution then has
// epoch 1) and a give-up count is added to the plan's own count afterwards.
void exec_plan(Plan &p, const double *params, int32_t nparams, void *stream, bool use_static) {
        LaunchArgs la = launch_args(p, params, nparams, stream);
        const HostPlan &hp = p.hp;
        if (hp.n_elem == 0) return;
        DeviceGuard g(p.ctx->device);
        const bool flow = hp.strategy == UM_STRAT_HIER && hp.schedule == UM_SCHED_DATAFLOW &&
                          !is_step_kernel(p.kernel);
        int32_t *static_ctl = nullptr;
        if (use_static) {
            char *base = static_cast<char *>(scratch_address(p.ctx->device));
            if (flow) {
                // [control words: 256 bytes][flags: one word per launch position]
                const int64_t words = int64_t(hp.binfo.size());
                if (256 + 4 * words > STATIC_SCRATCH_BYTES)
                    fail(UM_ERR_ARG, "static scratch: %lld dataflow blocks need %lld bytes, "
                         "limit %lld", (long long)(words - 1), (long long)(256 + 4 * words),
                         (long long)STATIC_SCRATCH_BYTES);
                static_ctl = reinterpret_cast<int32_t *>(base);
                la.err = static_ctl;
                la.flags = reinterpret_cast<int32_t *>(base + 256);
                const hipError_t e1 = zero_words(static_ctl, 4, la.stream);
                const hipError_t e2 = zero_words(la.flags, words, la.stream);
                if (e1 != hipSuccess || e2 != hipSuccess)
                    fail(UM_ERR_HIP, "clearing the static scratch: %s",
                         hipGetErrorString(e1 != hipSuccess ? e1 : e2));
            } else if (la.n_partials > 0) {
                if (8 * int64_t(la.n_partials) > STATIC_SCRATCH_BYTES)
                    fail(UM_ERR_ARG, "static scratch: %d partial sums need %lld bytes, limit %lld",
                         la.n_partials, (long long)(8 * int64_t(la.n_partials)),
                         (long long)STATIC_SCRATCH_BYTES);
                la.partials = reinterpret_cast<double *>(base);
            }
        }
        auto one = [&](int which, int32_t b, int32_t e, int64_t lds) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (p.timing) {
                const size_t need_ev = 2 * size_t(p.pending_pairs + 1);
                while (p.events.size() < need_ev) {
                    hipEvent_t h;
                    UM_HIP(hipEventCreate(&h));
                    p.events.push_back(h);
                }
                e0 = static_cast<hipEvent_t>(p.events[2 * p.pending_pairs]);
                e1 = static_cast<hipEvent_t>(p.events[2 * p.pending_pairs + 1]);
                UM_HIP(hipEventRecord(e0, la.stream));
            }
            const hipError_t le = p.kernel == UM_K_HEX_HOURGLASS_3D
                                      ? hex_launch_one(la, which, b, e, lds)
                                      : lf2d_launch_one(la, which, b, e, lds);
            if (le != hipSuccess)
                fail(UM_ERR_HIP,
                     "launch %d of kernel %d (range [%d, %d), %d lanes per workgroup, %lld bytes "
                     "of LDS, dtype %d, layout %d, staging %d, schedule %d) failed: %s",
                     which, p.kernel, b, e, la.block_size, (long long)lds, la.dtype, la.layout,
                     la.staging, la.schedule, hipGetErrorString(le));
            if (p.timing) {
                UM_HIP(hipEventRecord(e1, la.stream));
                ++p.pending_pairs;
            }
        };
        if (is_step_kernel(p.kernel)) {
            auto step = [&](int which, int32_t b, int32_t e) {
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (p.timing) {
                    const size_t need_ev = 2 * size_t(p.pending_pairs + 1);
                    while (p.events.size() < need_ev) {
                        hipEvent_t h;
                        UM_HIP(hipEventCreate(&h));
                        p.events.push_back(h);
                    }
                    e0 = static_cast<hipEvent_t>(p.events[2 * p.pending_pairs]);
                    e1 = static_cast<hipEvent_t>(p.events[2 * p.pending_pairs + 1]);
                    UM_HIP(hipEventRecord(e0, la.stream));
                }
                const hipError_t le = step_launch_one(la, p.kernel, which, b, e);
                if (le != hipSuccess)
                    fail(UM_ERR_HIP, "launch %d of kernel %d (range [%d, %d), %d lanes per "
                         "workgroup, dtype %d) failed: %s", which, p.kernel, b, e, la.block_size,
                         la.dtype, hipGetErrorString(le));
                if (p.timing) {
                    UM_HIP(hipEventRecord(e1, la.stream));
                    ++p.pending_pairs;
                }
            };
            const int32_t n = int32_t(hp.n_elem);
            if (p.kernel == UM_K_CELL_ADT_2D) {
                step(LAUNCH_DIRECT, 0, n);
            } else if (p.kernel == UM_K_UPDATE_2D || p.kernel == UM_K_UPDATE_ADT_2D) {
                step(LAUNCH_DIRECT, 0, n);
                step(LAUNCH_REDUCE, 0, 1);
            } else if (hp.strategy == UM_STRAT_GLOBAL_COLOUR) {
                for (int32_t c = 0; c + 1 < int32_t(hp.colour_off.size()); ++c)
                    if (hp.colour_off[c + 1] > hp.colour_off[c])
                        step(LAUNCH_GCOL, hp.colour_off[c], hp.colour_off[c + 1]);
            } else {
                step(LAUNCH_ATOMIC, 0, n);
            }
        } else if (hp.strategy == UM_STRAT_HIER && hp.schedule == UM_SCHED_DATAFLOW) {
            // the execution number is kept and advanced on the device
            one(LAUNCH_HIER_FLOW, 0, int32_t(hp.blk_order.size()), hp.lds_max);
        } else if (hp.strategy == UM_STRAT_HIER) {
            for (int32_t c = 0; c + 1 < int32_t(hp.bcol_off.size()); ++c)
                if (hp.bcol_off[c + 1] > hp.bcol_off[c])
                    one(LAUNCH_HIER, hp.bcol_off[c], hp.bcol_off[c + 1], hp.lds_per_colour[c]);
        } else if (hp.strategy == UM_STRAT_GLOBAL_COLOUR) {
            for (int32_t c = 0; c + 1 < int32_t(hp.colour_off.size()); ++c)
                if (hp.colour_off[c + 1] > hp.colour_off[c])
                    one(LAUNCH_GCOL, hp.colour_off[c], hp.colour_off[c + 1], 0);
        } else {
            one(LAUNCH_ATOMIC, 0, int32_t(hp.n_elem), 0);
        }
        if (static_ctl) {
            const hipError_t e = add_count(p.dp.err, static_ctl, la.stream);
            if (e != hipSuccess)
                fail(UM_ERR_HIP, "adding the give-up count: %s", hipGetErrorString(e));
        }
}

}  // namespace
}  // namespace um

extern "C" {

um_status um_loop_exec(um_plan plan, const double *params, int32_t nparams, void *stream) {
    return guarded([&] { exec_plan(need(plan), params, nparams, stream, false); });
}

um_status um_loop_exec_static(um_plan plan, const double *params, int32_t nparams,
                              void *stream) {
    return guarded([&] { exec_plan(need(plan), params, nparams, stream, true); });
}

um_status um_plan_autotune(um_ctx ctx, int32_t kernel, const um_arg *args, int32_t nargs,
                           int32_t iter_set, const um_plan_opts *candidates,
                           int32_t n_candidates, const double *params, int32_t nparams,
                           void *stream, int32_t reps, int32_t *best_index, double *ms_out,
                           um_plan *out) {
    return guarded([&] {
        Ctx &c = need(ctx);
        if (!candidates || n_candidates < 1 || reps < 1 || !best_index || !out)
            fail(UM_ERR_ARG, "autotune: null output, no candidates or reps < 1");
        if (c.device < 0) fail(UM_ERR_STATE, "host-only context cannot execute");
        *out = nullptr;
        *best_index = -1;
        DeviceGuard g(c.device);
        struct Events {
            hipEvent_t e[2] = {nullptr, nullptr};
            ~Events() {
                for (hipEvent_t h : e)
                    if (h) hipEventDestroy(h);
            }
        } ev;
        UM_HIP(hipEventCreate(&ev.e[0]));
        UM_HIP(hipEventCreate(&ev.e[1]));
        const hipStream_t s = static_cast<hipStream_t>(stream);
        um_plan best = nullptr;
        double best_ms = 0.0;
        auto check = [](um_status st) {
            if (st != UM_OK) throw Error{st, g_err};
        };
        try {
            for (int32_t i = 0; i < n_candidates; ++i) {
                if (ms_out) ms_out[i] = -1.0;
                um_plan p = nullptr;
                const um_status st =
                    um_plan_build(ctx, kernel, args, nargs, iter_set, &candidates[i], &p);
                if (st != UM_OK && st != UM_ERR_LDS && st != UM_ERR_COLOURS &&
                    st != UM_ERR_UNSUPPORTED && st != UM_ERR_ARG)
                    g_err = "candidate " + std::to_string(i) + ": " + g_err;
                if (st == UM_ERR_LDS || st == UM_ERR_COLOURS || st == UM_ERR_UNSUPPORTED ||
                    st == UM_ERR_ARG)
                    continue;
                check(st);
                try {
                    const um_status st0 = um_loop_exec(p, params, nparams, stream);
                    if (st0 != UM_OK) g_err = "candidate " + std::to_string(i) + ": " + g_err;
                    check(st0);
                    UM_HIP(hipEventRecord(ev.e[0], s));
                    for (int32_t r = 0; r < reps; ++r) check(um_loop_exec(p, params, nparams, stream));
                    UM_HIP(hipEventRecord(ev.e[1], s));
                    UM_HIP(hipEventSynchronize(ev.e[1]));
                    int32_t nerr = 0;
                    check(um_plan_errors(p, &nerr));
                    float ms = 0.f;
                    UM_HIP(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
                    const double per = double(ms) / reps;
                    if (nerr != 0) {
                        um_plan_destroy(p);
                        continue;
                    }
                    if (ms_out) ms_out[i] = per;
                    if (!best || per < best_ms) {
                        if (best) um_plan_destroy(best);
                        best = p;
                        best_ms = per;
                        *best_index = i;
                    } else {
                        um_plan_destroy(p);
                    }
                } catch (...) {
                    um_plan_destroy(p);
                    throw;
                }
            }
        } catch (...) {
            if (best) um_plan_destroy(best);
            *best_index = -1;
            throw;
        }
        if (!best) fail(UM_ERR_UNSUPPORTED, "autotune: no candidate could be built");
        *out = best;
    });
}

um_status um_plan_set_timing(um_plan plan, int32_t enable) {
    return guarded([&] { need(plan).timing = enable != 0; });
}

um_status um_plan_timing(um_plan plan, double *ms_total, int64_t *n_launches) {
    return guarded([&] {
        Plan &p = need(plan);
        if (!ms_total || !n_launches) fail(UM_ERR_ARG, "null output");
        DeviceGuard g(p.ctx->device);
        double ms = 0.0;
        for (int64_t i = 0; i < p.pending_pairs; ++i) {
            hipEvent_t e0 = static_cast<hipEvent_t>(p.events[2 * i]);
            hipEvent_t e1 = static_cast<hipEvent_t>(p.events[2 * i + 1]);
            UM_HIP(hipEventSynchronize(e1));
            float t = 0.f;
            UM_HIP(hipEventElapsedTime(&t, e0, e1));
            ms += t;
        }
        *ms_total = ms;
        *n_launches = p.pending_pairs;
        p.pending_pairs = 0;
    });
}

um_status um_plan_errors(um_plan plan, int32_t *n_errors) {
    return guarded([&] {
        Plan &p = need(plan);
        if (!n_errors) fail(UM_ERR_ARG, "null output");
        *n_errors = 0;
        if (!p.dp.err) return;
        DeviceGuard g(p.ctx->device);
        UM_HIP(hipDeviceSynchronize());
        UM_HIP(hipMemcpy(n_errors, p.dp.err, sizeof(int32_t), hipMemcpyDeviceToHost));
    });
}

um_status um_plan_reset_errors(um_plan plan) {
    return guarded([&] {
        Plan &p = need(plan);
        if (!p.dp.err) return;
        DeviceGuard g(p.ctx->device);
        UM_HIP(hipDeviceSynchronize());
        const int32_t zero[2] = {0, 0};
        UM_HIP(hipMemcpy(p.dp.err, zero, sizeof zero, hipMemcpyHostToDevice));
    });
}

um_status um_plan_set_wait_limit(um_plan plan, int64_t ticks) {
    return guarded([&] {
        Plan &p = need(plan);
        if (ticks < 0) fail(UM_ERR_ARG, "negative wait limit");
        p.wait_ticks = ticks == 0 ? DEFAULT_WAIT_TICKS : uint64_t(ticks);
    });
}

um_status um_debug_fluxes(um_plan plan, const double *params, int32_t nparams, void *f_out,
                          void *stream) {
    return guarded([&] {
        Plan &p = need(plan);
        if (is_step_kernel(p.kernel))
            fail(UM_ERR_UNSUPPORTED, "per-element debug output exists for the edge and hex loops only");
        LaunchArgs la = launch_args(p, params, nparams, stream);
        const Ctx &c = *p.ctx;
        const int64_t E = c.sets[p.iter_set].size;
        if (E == 0) return;
        if (!f_out) fail(UM_ERR_ARG, "null output buffer");
        DeviceGuard g(c.device);
        std::vector<int32_t> em;
        if (p.kernel == UM_K_HEX_HOURGLASS_3D) {
            em = c.maps[p.ha.map].table;
        } else {
            em.resize(4 * E);
            const Map &mc = c.maps[p.ea.map_c], &mn = c.maps[p.ea.map_n];
            for (int64_t e = 0; e < E; ++e) {
                em[4 * e] = mc.table[2 * e];
                em[4 * e + 1] = mc.table[2 * e + 1];
                em[4 * e + 2] = mn.table[2 * e];
                em[4 * e + 3] = mn.table[2 * e + 1];
            }
        }
        int64_t bytes = 0;
        int32_t *d_em = upload(em, bytes);
        la.emap = d_em;
        la.out = static_cast<double *>(f_out);
        la.block_size = 256;
        hipError_t err = p.kernel == UM_K_HEX_HOURGLASS_3D
                             ? hex_launch_one(la, LAUNCH_DEBUG, 0, int32_t(E), 0)
                             : lf2d_launch_one(la, LAUNCH_DEBUG, 0, int32_t(E), 0);
        hipError_t err2 = hipStreamSynchronize(la.stream);
        hipFree(d_em);
        if (err != hipSuccess || err2 != hipSuccess)
            fail(UM_ERR_HIP, "debug flux launch: %s", hipGetErrorString(err != hipSuccess ? err : err2));
    });
}

um_status um_graph_begin(void *stream) {
    return guarded([&] {
        if (!stream) fail(UM_ERR_ARG, "the default (NULL) stream cannot be captured");
        UM_HIP(hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeRelaxed));
    });
}

um_status um_graph_end(void *stream, um_graph *out) {
    return guarded([&] {
        if (!stream || !out) fail(UM_ERR_ARG, "null stream or output");
        *out = nullptr;
        hipGraph_t g = nullptr;
        UM_HIP(hipStreamEndCapture(static_cast<hipStream_t>(stream), &g));
        if (!g) fail(UM_ERR_STATE, "capture produced no graph");
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(g);
            fail(UM_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
        um_graph h = new um_graph_s;
        h->graph = g;
        h->exec = ex;
        *out = h;
    });
}

um_status um_graph_launch(um_graph graph, void *stream) {
    return guarded([&] {
        if (!graph) fail(UM_ERR_ARG, "null graph");
        UM_HIP(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)));
    });
}

um_status um_graph_destroy(um_graph graph) {
    return guarded([&] {
        if (!graph) return;
        if (graph->exec) hipGraphExecDestroy(graph->exec);
        if (graph->graph) hipGraphDestroy(graph->graph);
        delete graph;
    });
}

}  // extern "C"
