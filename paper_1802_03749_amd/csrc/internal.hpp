// Library-internal declarations of libumesh (not part of the C ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "umesh.h"

namespace um {

// Thrown inside the library, converted to a um_status at the ABI boundary.
struct Error {
    um_status code;
    std::string msg;
};
[[noreturn]] void fail(um_status code, const char *fmt, ...);

struct Set {
    int64_t size = 0;
    std::string name;
    std::vector<int32_t> new2orig;   // cumulative renumbering
    int32_t part_block_size = 0;     // blocks from the last PARTITION reorder
    std::vector<int32_t> part_off;   // [n_blocks + 1]
    std::vector<int32_t> part_code;  // [n_blocks] bisection parity code (empty if none)
};

struct Map {
    int32_t from = 0, to = 0, arity = 0;
    std::vector<int32_t> table;      // [size(from)][arity]
};

struct Dat {
    int32_t set = 0, dim = 0, dtype = UM_F64, layout = UM_AOS;
    void *ptr = nullptr;
};

struct Plan;

struct Ctx {
    int32_t device = -1;             // -1: host-only
    int32_t lds_limit = 65536;       // per-workgroup LDS limit in bytes
    int32_t n_cu = 256;              // compute units (host-only: MI355X's)
    int64_t lds_per_cu = 163840;     // LDS bytes per compute unit
    std::vector<Set> sets;
    std::vector<Map> maps;
    std::vector<Dat> dats;
    std::vector<Plan *> plans;
    // device copies of the cumulative permutations, uploaded on demand
    std::vector<int32_t *> d_new2orig;
    std::vector<int32_t *> d_orig2new;
};

// ------------------------------------------------------------ reordering
// All return new->old permutations (new id k holds old id perm[k]).

// Cuthill-McKee numbering of the to-set of `m` over the graph in which the
// points of each element form a clique; reverse = RCM.
std::vector<int32_t> cuthill_mckee(const Map &m, int64_t n_points, bool reverse);
// Elements sorted by their sorted point ids (lexicographic), ties by old id.
std::vector<int32_t> lexicographic_elements(const Map &m);
// Points numbered in order of first appearance over the elements (in table
// order) and slots; untouched points follow in ascending id.
std::vector<int32_t> first_touch(const Map &m, int64_t n_points);
// Partition the from-set of `drv` into blocks of <= block_size elements;
// returns the element order (block by block) and fills block offsets.
// Recursive coordinate bisection into blocks of at most block_size
// elements; block_off gets the block offsets and block_code, per block, the
// side (0 or 1) of the last cut along each axis as bit `axis` (the parity of
// the block's index along that axis when the blocks form a regular grid).
std::vector<int32_t> partition_elements(const Ctx &ctx, int32_t drv, int32_t block_size,
                                        int32_t coord_map, int32_t coord_dim,
                                        const double *coords, std::vector<int32_t> &block_off,
                                        std::vector<int32_t> &block_code);
// Points of to-set `set` sorted, stably, by key 1: (number of accessing
// blocks, list of accessing blocks); key 2: (smallest accessing block,
// number, list); key 3: the accessing blocks from the largest down, element
// by element (a prefix first).  Unaccessed points last; elements of `from`
// are in block order.
std::vector<int32_t> signature_order(const Ctx &ctx, int32_t from, int32_t set,
                                     const std::vector<int32_t> &block_of_elem, int32_t key);
// Renumber `set` by new->old `perm`: rewrites every map from or into it.
void apply_set_perm(Ctx &ctx, int32_t set, const std::vector<int32_t> &perm);

void reorder_mesh(Ctx &ctx, const um_reorder_opts &o);

// --------------------------------------------------------------- planning
// Elements of the LF2D edge loop in packed form: L, R cells and a, b nodes.
struct EdgeArgs {
    int32_t map_n = -1, map_c = -1;              // edge->node, edge->cell
    int32_t dat_x = -1, dat_q = -1, dat_adt = -1, dat_res = -1;
    int32_t dtype = UM_F64, layout = UM_AOS;
};

// Arguments of the hex element loop: one arity-8 map, x and v read, force
// incremented, all through every slot.
struct HexArgs {
    int32_t map = -1;
    int32_t dat_x = -1, dat_v = -1, dat_f = -1;
    int32_t dtype = UM_F64, layout = UM_AOS;
};

// Arguments of the other time-step loops (UM_K_CELL_ADT_2D,
// UM_K_BOUNDARY_FLUX_2D, UM_K_UPDATE_2D); unused ids stay -1.
struct StepArgs {
    int32_t map_n = -1, map_c = -1;              // element->node, element->cell
    int32_t dat_x = -1, dat_q = -1, dat_adt = -1, dat_res = -1, dat_rms = -1;
    int32_t layout = UM_AOS;
    int32_t dtype = UM_F64;                      // of x, q and adt
};

// Per-block layout of a hierarchical plan, in launch order.
struct BlockInfo {
    int32_t slot_off;   // first slot of the block
    int32_t cell_off;   // first staged cell (into stg_c)
    int32_t node_off;   // first staged node (into stg_n)
    int32_t ncol;       // thread colours used by the block
    int32_t crun_off;   // first run of the staged cells (into crun); a block
    int32_t nrun_off;   // with no runs reads its explicit list instead
    int32_t sum_first;  // DATAFLOW edge loop: sums its fluxes before its wait
    int32_t pad1;
};

// A run of consecutive staged points: staged positions local, local+1, ...
// (up to the next run's `local`) hold point ids start, start+1, ...
struct Run {
    int32_t start;
    int32_t local;
};

// Blocks whose staged list splits into more runs than this read the
// explicit list.
constexpr int32_t MAX_RUNS = 8;

// Everything a DATAFLOW block of the edge loop's LDS-DMA kernel needs before
// its first memory round trip, one record per launch position, read with
// scalar loads: its ranges and counts, its (first 8) predecessors, whether
// it sums its fluxes before waiting (sum_first), and the run descriptors of
// its staged cell and node lists (ncr / nnr = 0: the block reads its
// explicit list instead).
struct FlowRec {
    int32_t slot_off, cell_off, node_off, ncol;
    int32_t ne, nc, nn, np;
    int32_t ncr, nnr, p0, sum_first;
    int32_t preds[8];
    Run cruns[MAX_RUNS];
    Run nruns[MAX_RUNS];
    int32_t pad1[12];
};
static_assert(sizeof(FlowRec) == 256, "FlowRec is 256 bytes");

struct HostPlan {
    int32_t strategy = 0, staging = 0, tcmode = 0, block_size = 0;
    int32_t ept = 1, threads = 0;              // HIER: elements per lane, lanes per block
    int32_t n_partials = 0;                    // UPDATE: workgroups of the first launch
    int32_t schedule = 0;                      // HIER: um_schedule
    int64_t n_elem = 0;
    int64_t n_slots = 0;                       // HIER edge loop: slots incl. wave padding
    // GLOBAL_COLOUR / ATOMIC: packed (L, R, a, b) per slot, slot order
    std::vector<int32_t> emap;                 // [n_slots][4]
    std::vector<int32_t> colour_off;           // GLOBAL: [ncol + 1] slot ranges
    std::vector<int32_t> elem_colour;          // GLOBAL: colour per element
    // HIER
    std::vector<int32_t> blk_off;              // block id order: element ranges
    std::vector<int32_t> blk_colour;           // block id order
    std::vector<int32_t> blk_order;            // launch position -> block id
    std::vector<int32_t> bcol_off;             // [nbcol + 1] launch position ranges
    std::vector<BlockInfo> binfo;              // [nb + 1] launch order (+ sentinel)
    std::vector<int32_t> stg_c, stg_n;         // launch order
    std::vector<Run> crun, nrun;               // run encoding of stg_c, stg_n
    int32_t use_runs = 1;
    std::vector<uint32_t> loc;                 // LF2D: [n_slots] words + [n_slots] halves; hex: [n_slots][4]
    std::vector<int32_t> slot_elem;            // slot -> element
    std::vector<int32_t> tcol;                 // element -> thread colour
    std::vector<int64_t> lds_per_colour;       // max LDS bytes per block colour
    std::vector<int32_t> pred_off, preds;      // DATAFLOW: earlier neighbours per position
    std::vector<FlowRec> frec;                 // DATAFLOW edge loop: per position
    int64_t n_sum_first = 0;                   // DATAFLOW edge loop: blocks with sum_first
    int32_t gather = 0;                        // HIER, DATAFLOW: um_gather
    int32_t wave_groups = 0;                   // HIER: colour groups padded to waves
    int32_t max_tcol = 0;
    double avg_tcol = 0.0, reuse = 0.0;
    int64_t lds_max = 0, staged_total = 0;
};

void build_host_plan(const Ctx &ctx, const EdgeArgs &ea, int32_t iter_set,
                     const um_plan_opts &o, HostPlan &hp);
void build_host_plan_hex(const Ctx &ctx, const HexArgs &ha, int32_t iter_set,
                         const um_plan_opts &o, HostPlan &hp);

// Stable counting sort of 0..n-1 by small integer keys; returns the order
// and fills offsets (size nkeys + 1).
std::vector<int32_t> counting_order(const std::vector<int32_t> &key, int32_t nkeys,
                                    std::vector<int32_t> &offsets);
// First-fit colouring of the elements of `mc` (any arity) so that no two
// elements of one colour share a point; returns the number of colours.
int32_t global_colours(const Map &mc, int64_t n_points, std::vector<int32_t> &colour);

StepArgs check_step_args(const Ctx &ctx, int32_t kernel, const um_arg *args, int32_t nargs,
                         int32_t iter_set);
void build_host_plan_step(const Ctx &ctx, int32_t kernel, const StepArgs &sa, int32_t iter_set,
                          const um_plan_opts &o, HostPlan &hp);

// LDS bytes a block needs for the given counts.
int64_t lf2d_lds_bytes(int32_t staging, int32_t dtype, int64_t n_cells, int64_t n_nodes);
int64_t hex_lds_bytes(int64_t n_nodes, bool dataflow);

// ----------------------------------------------------------------- device
struct DevicePlan {
    int32_t *emap = nullptr;                   // int4 per slot
    BlockInfo *binfo = nullptr;
    int32_t *stg_c = nullptr, *stg_n = nullptr;
    Run *crun = nullptr, *nrun = nullptr;
    uint32_t *loc = nullptr;
    int32_t *pred_off = nullptr, *preds = nullptr;  // DATAFLOW
    FlowRec *frec = nullptr;                        // DATAFLOW edge loop: per position
    int32_t *flags = nullptr;                       // DATAFLOW: completion epochs per block
    int32_t *err = nullptr;                         // DATAFLOW: [timeouts, epoch of the
                                                    //  last timeout, unused x2]
    double *partials = nullptr;                     // UPDATE: one sum per workgroup
    int64_t bytes = 0;
};

// Longest a dataflow block waits for one neighbour: 0.2 s of the 100 MHz
// s_memrealtime counter.
constexpr uint64_t DEFAULT_WAIT_TICKS = 20000000ull;

struct Plan {
    Ctx *ctx = nullptr;
    int32_t kernel = 0;
    int32_t iter_set = 0;
    EdgeArgs ea;
    HexArgs ha;
    StepArgs sa;
    HostPlan hp;
    DevicePlan dp;
    double build_seconds = 0.0;
    uint64_t wait_ticks = DEFAULT_WAIT_TICKS;  // DATAFLOW wait limit
    bool timing = false;
    std::vector<void *> events;                // hipEvent_t pairs
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
    int64_t pending_pairs = 0;
};

}  // namespace um
