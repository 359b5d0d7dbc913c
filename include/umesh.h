/*
 * umesh.h -- race-free indirect-increment mesh loops on AMD MI355X (gfx950).
 *
 * C ABI of libumesh.so.  Plain integers, host pointers and device pointers
 * only; no C++ or framework types cross it.  Every entry point returns a
 * um_status; no exception crosses the boundary.  On failure the message of
 * the failing call is available from um_last_error() on the same thread.
 *
 * Model (Sulyok et al., "Locality optimized unstructured mesh algorithms on
 * GPUs", Section 1.1.1 "Unstructured meshes"): a mesh is a collection of
 * sets (elements numbered 0..size-1), maps (fixed-arity tables from every
 * element of a from-set to elements of a to-set, one level of indirection)
 * and dats (dim values per element of a set).  A loop runs an elemental
 * kernel over every element of an iteration set, reading data directly or
 * through one map, and may increment data on the to-set of a map, so that
 * several iterations update the same point.  The result must not depend on
 * the processing order beyond rounding.
 *
 * Execution strategies (Section 2.1 and 2.2):
 *   UM_STRAT_ATOMIC        one launch, increments with device atomics;
 *   UM_STRAT_GLOBAL_COLOUR elements coloured so no two of one colour write
 *                          the same point, one launch per colour;
 *   UM_STRAT_HIER          two-layer (hierarchical) colouring: elements are
 *                          grouped in blocks, blocks coloured so concurrent
 *                          blocks never write the same point (one launch per
 *                          block colour), each block stages its indirect data
 *                          and its increments in LDS, and elements inside a
 *                          block are coloured so that increments into LDS are
 *                          applied one colour at a time (Algorithm 1).
 * Reordering (Section 2.3): Cuthill-McKee style renumbering of points and a
 * lexicographic sort of elements (Section 2.3.1), partition-based element
 * blocks (Section 2.3.2) and grouping of points by the set of blocks that
 * access them (Section 2.3.2, cache-line heuristic).
 *
 * Threading: a um_ctx and its plans are not thread-safe; use one context
 * per host thread.  Device work is enqueued on the caller's HIP stream and
 * never synchronised by the library except where stated.
 */
#ifndef UMESH_H
#define UMESH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UMESH_ABI_VERSION 2

typedef struct um_ctx_s *um_ctx;
typedef struct um_plan_s *um_plan;
typedef struct um_graph_s *um_graph;

typedef enum {
    UM_OK = 0,
    UM_ERR_ARG = -1,         /* null pointer, bad enum, bad size            */
    UM_ERR_RANGE = -2,       /* map entry outside its to-set, bad id        */
    UM_ERR_ARITY = -3,       /* argument pattern does not fit the kernel    */
    UM_ERR_COLOURS = -4,     /* block colours exceed max_block_colours      */
    UM_ERR_LDS = -5,         /* staging exceeds the LDS limit, no fallback  */
    UM_ERR_HIP = -6,         /* a HIP runtime call failed                   */
    UM_ERR_STATE = -7,       /* call not valid in the current state         */
    UM_ERR_NOMEM = -8,       /* host or device allocation failed            */
    UM_ERR_UNSUPPORTED = -9  /* valid request the library does not provide  */
} um_status;

typedef enum { UM_F64 = 0, UM_F32 = 1 } um_dtype;
/* AoS: element-major [n][dim].  SoA: component-major [dim][n]
 * (Section 2.1.1 "Array-of-Structures (AoS) vs Structure-of-Arrays"). */
typedef enum { UM_AOS = 0, UM_SOA = 1 } um_layout;
typedef enum { UM_READ = 0, UM_WRITE = 1, UM_RW = 2, UM_INC = 3 } um_access;
typedef enum {
    UM_STRAT_ATOMIC = 0,
    UM_STRAT_GLOBAL_COLOUR = 1,
    UM_STRAT_HIER = 2
} um_strategy;
typedef enum {
    UM_REORDER_NONE = 0,
    UM_REORDER_RCM = 1,       /* reverse Cuthill-McKee numbering of points   */
    UM_REORDER_GPS = 2,       /* forward Cuthill-McKee (level order) numbering */
    UM_REORDER_PARTITION = 3, /* partition elements into blocks, renumber    */
    UM_REORDER_LEXICOGRAPHIC = 4, /* renumber only the from-set of the map by
                                     its sorted point ids (secondary loops) */
    UM_REORDER_USER_BLOCKS = 5    /* blocks given by the caller (block_of)   */
} um_reorder;
/* What a hierarchical block stages in LDS (Section 2.2; increments-only
 * staging is the fallback the paper needed when the staged data did not fit
 * in on-chip memory, Section 3.1.5). */
typedef enum { UM_STAGE_ALL = 0, UM_STAGE_INC_ONLY = 1 } um_staging;
/* How increments inside a block are serialised: colour rounds separated by
 * workgroup barriers (Algorithm 1), or LDS floating-point atomics without
 * thread colours (an extension; order inside a block is not fixed). */
typedef enum { UM_TC_BARRIER = 0, UM_TC_LDS_ATOMIC = 1 } um_tcmode;
/* Block colouring (layer 1).  FIRST_FIT: first-fit greedy in block order.
 * RECOLOUR: after first-fit, one iterated-greedy pass (blocks revisited by
 * decreasing colour, first-fit again; never more colours) and one balancing
 * pass (in block order a block moves to the least used colour none of its
 * neighbours holds when that class is smaller by two or more); fewer and
 * more even launches.
 * MIN: as RECOLOUR, but before the balancing pass also a DSatur colouring
 * (Brelaz) and, when the plan's blocks are those of the last PARTITION
 * reorder, the bisection's parity code (per axis, the side of the block's
 * last cut along it: 2^dim colours on a regular grid of blocks; clashes
 * recoloured first-fit), then a tabu search (Hertz and de Werra's TabuCol,
 * deterministic, bounded to 100 moves per block) for one colour fewer at a
 * time; the plan keeps the fewest colours found.  Slower to build. */
typedef enum { UM_BCOL_FIRST_FIT = 0, UM_BCOL_RECOLOUR = 1, UM_BCOL_MIN = 2 } um_bcolouring;
/* How block colours are ordered in time (HIER).  COLOUR_LAUNCHES: one kernel
 * launch per block colour (the kernel boundary orders colours, Section 2.2).
 * DATAFLOW: one launch over all blocks in colour order; each block computes
 * its fluxes, then waits until every neighbouring block of an earlier colour
 * has published its write-back, then loads and updates its residuals.  The
 * schedule's residual loads and stores carry device-scope coherence (they
 * bypass the per-XCD L2 caches' stale lines), a block's completion flag is
 * stored once its residual stores have completed and polled with
 * device-scope loads.  Needs 32 * (cells) < 2^31.  The per-cell order of additions is the same as
 * with colour launches; results agree to rounding (the two kernels may pair
 * multiply-adds into FMAs differently) and each schedule is bitwise
 * reproducible from run to run.
 * A wait that exceeds a time limit counts an error of the plan instead of
 * hanging (um_plan_errors, um_plan_set_wait_limit).  Each block's flag counts the executions it has
 * completed (all flags advance together), so the launch needs no host-side
 * counter and may be captured in a HIP graph and replayed.  Supported for STAGE_ALL with one or two
 * elements per lane; a plan must not execute concurrently with itself. */
typedef enum { UM_SCHED_COLOUR_LAUNCHES = 0, UM_SCHED_DATAFLOW = 1 } um_schedule;
/* How a DATAFLOW block of the edge loop moves its staged data from HBM to
 * LDS (Section 2.2's gather step).  REGISTERS: each lane loads a staged
 * point's values into registers and stores them to LDS.  LDS_DMA: the loads
 * write LDS directly (gfx950 buffer/global loads with the LDS bit, 4- and
 * 16-byte per lane), no registers hold staged data, and the residuals are
 * fetched in the same round trip as q, adt and x whenever the block's
 * earlier-coloured neighbours have already published (their flags are read
 * at the block's start); AoS data only. */
typedef enum { UM_GATHER_REGISTERS = 0, UM_GATHER_LDS_DMA = 1 } um_gather;

/* Elemental kernels compiled into the library (no run-time code generation).
 *
 * UM_K_EDGE_FLUX_LF2D -- 2D finite-volume edge flux (the Airfoil res_calc
 * access pattern of Section 3.1.1: per edge, read 2 coordinates on each of 2
 * nodes, read 4 conserved values and 1 time-step value on each of 2 cells,
 * increment 4 residual values on both cells).  Required args, in order:
 *   0: x   dim 2 via edge->node map slot 0, UM_READ
 *   1: x   dim 2 via edge->node map slot 1, UM_READ
 *   2: q   dim 4 via edge->cell map slot 0, UM_READ
 *   3: q   dim 4 via edge->cell map slot 1, UM_READ
 *   4: adt dim 1 via edge->cell map slot 0, UM_READ
 *   5: adt dim 1 via edge->cell map slot 1, UM_READ
 *   6: res dim 4 via edge->cell map slot 0, UM_INC
 *   7: res dim 4 via edge->cell map slot 1, UM_INC
 * Both maps have arity 2 and the iteration set as from-set; res is UM_F64;
 * x, q and adt are all UM_F64, or all UM_F32 (the flux is then evaluated in
 * FP32 and each increment is accumulated into the FP64 residual without
 * further rounding of the FP32 value).  One layout for all four dats.
 * params = {gm1, eps}.  Per edge, with n = (y_b - y_a, x_a - x_b):
 *   per side s: ri = 1/q0, u = q1 ri, v = q2 ri,
 *               p = gm1 (q3 - 0.5 (q1 u + q2 v)), U = u n_x + v n_y,
 *               F = (q0 U, q1 U + p n_x, q2 U + p n_y, (q3 + p) U)
 *   mu = eps 0.5 (adt_L + adt_R)
 *   f  = 0.5 (F_L + F_R) + 0.5 mu (q_L - q_R)
 *   res[L] += f, res[R] -= f.
 *
 * UM_K_HEX_HOURGLASS_3D -- 3D element loop over hexahedra (the access
 * pattern of the LULESH stress/hourglass loop, Section 3.1.4: per element,
 * read 3 coordinates and 3 velocities on each of its 8 nodes, increment 3
 * force values on each of the 8 nodes).  Required args, in order, each
 * through all 8 slots of one element->node map (idx = UM_ALL_SLOTS):
 *   0: x     dim 3, UM_READ
 *   1: v     dim 3, UM_READ
 *   2: force dim 3, UM_INC
 * All UM_F64, one layout.  params = {kappa}.  Per element, with node order
 * 0-3 counter-clockwise on the bottom face and 4-7 above them, and the
 * hourglass base vectors
 *   G_1 = ( 1,  1, -1, -1, -1, -1,  1,  1)    G_2 = ( 1, -1, -1,  1, -1,  1,  1, -1)
 *   G_3 = ( 1, -1,  1, -1,  1, -1,  1, -1)    G_4 = (-1,  1, -1,  1,  1, -1,  1, -1)
 *   h = |x_6 - x_0|;  m_i,d = sum_b G_i,b v_b,d;  f_a,d = (-kappa h) sum_i G_i,a m_i,d
 *   force[node a] += f_a.
 *
 * The other loops of one explicit time step of the 2D solver (the Airfoil
 * loops of Section 3.1.1 besides the edge flux; their formulas are this
 * library's, the paper prints none):
 *
 * UM_K_CELL_ADT_2D -- cell loop, per cell the time-step scalar.  Args:
 *   0: x   dim 2 via a cell->node map of arity 4 (nodes counter-clockwise),
 *          idx UM_ALL_SLOTS, UM_READ
 *   1: q   dim 4 direct (map -1), UM_READ
 *   2: adt dim 1 direct, UM_WRITE
 * All UM_F64, one layout.  params = {gm1}.  Per cell, with side k from
 * node k to node k+1 (mod 4) and m = (y_k+1 - y_k, x_k - x_k+1):
 *   ri = 1/q0, u = q1 ri, v = q2 ri, p = gm1 (q3 - 0.5 (q1 u + q2 v)),
 *   c = sqrt((1 + gm1) p ri), adt = sum_k |u m_x + v m_y| + c |m|.
 * Any strategy; one launch of block_size lanes per workgroup.
 *
 * UM_K_BOUNDARY_FLUX_2D -- boundary-edge loop, the edge flux between the
 * edge's cell (left) and a far-field state (right).  Args:
 *   0: x   dim 2 via boundary-edge->node map (arity 2) slot 0, UM_READ
 *   1: x   dim 2 via the same map slot 1, UM_READ
 *   2: q   dim 4 via boundary-edge->cell map (arity 1) slot 0, UM_READ
 *   3: adt dim 1 via the same map slot 0, UM_READ
 *   4: res dim 4 via the same map slot 0, UM_INC
 * All UM_F64, one layout.  params = {gm1, eps, qinf0, qinf1, qinf2, qinf3}.
 * f = the UM_K_EDGE_FLUX_LF2D flux with q_L = q[cell], q_R = qinf and
 * adt_L = adt_R = adt[cell]; res[cell] += f.  A cell may have several
 * boundary edges, so the increment is race-prone: UM_STRAT_ATOMIC or
 * UM_STRAT_GLOBAL_COLOUR (UM_STRAT_HIER gives UM_ERR_UNSUPPORTED).
 *
 * UM_K_UPDATE_2D -- cell loop, explicit update and residual sum of squares.
 * Args:
 *   0: q   dim 4 direct, UM_RW
 *   1: res dim 4 direct, UM_RW
 *   2: adt dim 1 direct, UM_READ
 *   3: rms dim 1 global (map UM_GLOBAL, a dat on a set of size 1), UM_INC
 * All UM_F64, q/res/adt one layout.  No params (nparams 0).  Per cell and
 * component: d = res/adt, q -= d, res = 0; rms += sum of d^2 over all
 * cells.  The sum is reduced per workgroup in a fixed tree, the per-
 * workgroup partials are summed by a second launch in a fixed order and
 * added to rms, so the result is bitwise reproducible for a given
 * block_size.  Two launches; the plan owns the partials buffer.
 *
 * UM_K_UPDATE_ADT_2D -- UM_K_UPDATE_2D followed, in the same cell loop, by
 * UM_K_CELL_ADT_2D on the updated state: the time-step scalar the next step
 * needs, without reading q again.  Args:
 *   0: q   dim 4 direct, UM_RW
 *   1: res dim 4 direct, UM_RW
 *   2: adt dim 1 direct, UM_RW (read for the update, then overwritten)
 *   3: rms dim 1 global, UM_INC
 *   4: x   dim 2 via a cell->node map of arity 4, idx UM_ALL_SLOTS, UM_READ
 * Types and layouts as for the two loops.  params = {gm1}.  Per cell the
 * results equal bit for bit those of UM_K_UPDATE_2D then UM_K_CELL_ADT_2D
 * (same arithmetic in the same order; the sum of squares is reduced the
 * same way).  A time step then reads: edge flux, boundary flux, update +
 * adt, with adt computed once before the first step.  Two launches.
 */
typedef enum {
    UM_K_EDGE_FLUX_LF2D = 0,
    UM_K_HEX_HOURGLASS_3D = 1,
    UM_K_CELL_ADT_2D = 2,
    UM_K_BOUNDARY_FLUX_2D = 3,
    UM_K_UPDATE_2D = 4,
    UM_K_UPDATE_ADT_2D = 5
} um_kernel;

/* Map slot value meaning "every slot of the map" (a vector argument). */
#define UM_ALL_SLOTS (-1)

/* Map value of an argument that is a global reduction target: a dat
 * declared on a set of size 1, reduced into once per loop. */
#define UM_GLOBAL (-2)

/* One loop argument: dat `dat` accessed through slot `idx` of map `map`
 * (map = -1: direct access on the iteration set; idx = UM_ALL_SLOTS: every
 * slot) with access mode `acc`. */
typedef struct {
    int32_t dat;
    int32_t map;
    int32_t idx;
    int32_t acc; /* um_access */
} um_arg;

typedef struct {
    int32_t mode;          /* um_reorder                                     */
    int32_t driving_map;   /* map whose to-set is renumbered (RCM/GPS) and
                              whose from-set is partitioned (PARTITION)      */
    int32_t block_size;    /* PARTITION: maximum elements per block, 1..1024 */
    int32_t point_reorder; /* PARTITION / USER_BLOCKS: 0 = keep the order;
                              1 = group points of every to-set by accessing-
                              block signature (Section 2.3.2: number of
                              accessing blocks, then their list); 2 = by the
                              smallest accessing block first, then number
                              and list (an extension: each block's own
                              points and the halo it shares with later
                              blocks form one run); 3 = by the list of
                              accessing blocks taken from the largest down,
                              element by element, a prefix first (an
                              extension: halo groups whose last blocks
                              agree lie side by side, so fewer cache lines
                              hold points of unrelated blocks)              */
    int32_t coord_map;     /* PARTITION, optional: map from the partitioned set
                              whose to-set carries `coords`; -1 = none, then
                              a graph-distance embedding is used instead     */
    int32_t coord_dim;     /* 1..3                                           */
    const double *coords;  /* host [size(to-set of coord_map)][coord_dim],
                              current numbering; read during the call only   */
    const int32_t *block_of; /* USER_BLOCKS: host [size(from-set)], the block
                              id (>= 0) of every element in the current
                              numbering; read during the call only           */
    int32_t reserved[2];
} um_reorder_opts;

typedef struct {
    int32_t strategy;          /* um_strategy                                */
    int32_t block_size;        /* HIER: elements per block = workgroup size,
                                  64..1024; others: workgroup size, 64..1024 */
    int32_t staging;           /* um_staging (HIER)                          */
    int32_t tcmode;            /* um_tcmode (HIER)                           */
    int32_t max_block_colours; /* HIER: 0 means 256 (Section 3.1.5 limit)      */
    int32_t lds_limit_bytes;   /* HIER: 0 means the device's per-workgroup
                                  limit (163840 on gfx950; 65536 host-only)  */
    int32_t allow_fallback;    /* HIER: 1 = STAGE_ALL over the LDS limit falls
                                  back to STAGE_INC_ONLY instead of failing  */
    int32_t elems_per_thread;  /* HIER: elements each lane computes, 1 or 2
                                  (0 means 1); the workgroup has
                                  ceil(block_size / elems_per_thread) lanes
                                  rounded up to a multiple of 64             */
    int32_t explicit_lists;    /* HIER: 0 = a block whose staged points form
                                  at most 8 runs of consecutive ids finds
                                  them from the runs (no index loads); 1 =
                                  every block reads its explicit id list     */
    int32_t block_colouring;   /* HIER: um_bcolouring                        */
    int32_t schedule;          /* HIER: um_schedule                          */
    int32_t gather;            /* HIER, DATAFLOW: um_gather                  */
    int32_t wave_colour_groups;/* HIER: 1 = pad each thread-colour group of a
                                  block to whole 64-lane wavefronts, so that
                                  every wavefront holds one colour and takes
                                  part in one colour round only (more lanes
                                  per block: UM_ERR_ARG when the padded slots
                                  exceed 1024 * elems_per_thread)           */
    int32_t xcd_groups;        /* HIER, edge and hex loops: 0 or 1 = blocks
                                  launched in colour order as planned;
                                  G = 2..64: the blocks form G equal ranges
                                  of block ids (regions of space in
                                  partition order) and inside each block
                                  colour the k-th workgroup of its launch
                                  takes a block of range k mod G while that
                                  range has blocks left in the colour.  With
                                  G = 8 on MI355X, which hands consecutive
                                  workgroups of a launch to its 8 XCDs in
                                  turn, each region runs on one XCD and its
                                  blocks share that XCD's L2.  Launch order
                                  only: every block still follows the blocks
                                  of smaller colour around it, so barrier
                                  rounds give bitwise the same results where
                                  every block takes the same sum_first path */
    int32_t sum_first;         /* HIER, DATAFLOW, edge loop: which blocks
                                  sum their fluxes in LDS before waiting for
                                  their earlier-coloured neighbours and then
                                  only add the sums to the residuals, while
                                  the others load their residuals early and
                                  accumulate onto them.  0 = those whose
                                  latest such neighbour is launched fewer
                                  positions earlier than 3/4 of the blocks
                                  the device holds at once; 1 = every block
                                  with a neighbour to wait for; -1 = none.
                                  The results agree to rounding.  (The hex
                                  loop's dataflow blocks always sum first;
                                  other plans ignore the field.)            */
} um_plan_opts;

typedef struct {
    int32_t strategy;
    int32_t staging;             /* staging actually used (after fallback)   */
    int32_t block_size;
    int32_t n_blocks;            /* HIER                                     */
    int32_t n_block_colours;     /* HIER                                     */
    int32_t n_global_colours;    /* GLOBAL_COLOUR                            */
    int32_t max_thread_colours;  /* HIER                                     */
    int32_t n_launches;          /* kernel launches per um_loop_exec         */
    double avg_thread_colours;   /* HIER, mean over blocks                   */
    double reuse_factor;         /* HIER: sum over blocks of arity*|B| over
                                    sum of staged points, driving INC map    */
    int64_t n_elements;
    int64_t staged_points;       /* HIER: total staged points, all maps      */
    int64_t lds_bytes_max;       /* HIER: largest per-block LDS footprint    */
    int64_t plan_device_bytes;   /* device memory owned by the plan          */
    double build_seconds;        /* host wall time of um_plan_build          */
    int64_t n_sum_first_blocks;  /* HIER, DATAFLOW, edge loop: blocks that
                                    sum their fluxes before their wait
                                    (um_plan_opts.sum_first)                 */
    int64_t reserved[3];
} um_plan_stats;

/* Plan contents that can be copied out for verification (um_plan_export). */
typedef enum {
    UM_EXP_BLOCK_OFFSETS = 0,   /* int32[n_blocks+1]: element ranges, block id order */
    UM_EXP_BLOCK_COLOURS = 1,   /* int32[n_blocks]                                   */
    UM_EXP_THREAD_COLOURS = 2,  /* int32[n_elements]: thread colour per element     */
    UM_EXP_SLOT_ELEMENTS = 3,   /* int32[n_slots]: element executed at each slot,
                                   -1 for an empty slot (wave-pure colour groups);
                                   slots are grouped by block in launch order;
                                   n_slots = n_elements without padding          */
    UM_EXP_GLOBAL_COLOURS = 4,  /* int32[n_elements]: global colour per element      */
    UM_EXP_STAGED_OFFSETS_A = 5,/* int32[n_blocks+1]: staged points of the read-only
                                   indirect map (edge->node for LF2D; none for the
                                   hex loop), block id order                         */
    UM_EXP_STAGED_POINTS_A = 6, /* int32[...]: those points                          */
    UM_EXP_STAGED_OFFSETS_B = 7,/* as above for the INC map (edge->cell for LF2D,
                                   element->node for the hex loop)                   */
    UM_EXP_STAGED_POINTS_B = 8,
    UM_EXP_LOCAL_INDEX = 9,     /* int32[n_slots][k]: per slot, local staged index;
                                   LF2D k = 4: (B slot 0, B slot 1, A slot 0, A slot 1);
                                   hex k = 8: B slots 0..7                           */
    UM_EXP_BLOCK_ORDER = 10,    /* int32[n_blocks]: block id at each launch position  */
    UM_EXP_RUN_OFFSETS_A = 11,  /* int32[n_blocks+1]: run descriptors per block of the
                                   first indirect map's staged list, block id order;
                                   a block with none reads its explicit list        */
    UM_EXP_RUNS_A = 12,         /* int32[...][2]: (first point id, staged position)  */
    UM_EXP_RUN_OFFSETS_B = 13,  /* as above for the INC map                          */
    UM_EXP_RUNS_B = 14,
    UM_EXP_PRED_OFFSETS = 15,   /* DATAFLOW: int32[n_blocks+1], launch position order:
                                   the blocks each position waits for              */
    UM_EXP_PREDS = 16           /* DATAFLOW: int32[...]: their launch positions      */
} um_export_field;

/* ---------------------------------------------------------------- context */

/* ABI version compiled into the library (UMESH_ABI_VERSION). */
int32_t um_abi_version(void);

/* Message of the last failing call on this thread ("" if none).  The
 * pointer stays valid until the next failing call on this thread. */
const char *um_last_error(void);

/* Create a context on HIP device `device` (>= 0), or a host-only context
 * (device = -1) that can declare meshes, reorder and build plans but not
 * execute or touch device memory.  A context holds one mesh in the sense of
 * Section 1.1.1 (its sets, maps and dats) and the plans built for its
 * loops.  *out receives the handle.
 * Errors: UM_ERR_ARG (null out, device < -1), UM_ERR_HIP (device unusable). */
um_status um_create(int32_t device, um_ctx *out);

/* Destroy a context and every plan built from it (device memory released
 * after a device synchronisation).  NULL is accepted. */
um_status um_destroy(um_ctx ctx);

/* ------------------------------------------------------------ declaration */

/* Declare a set of `size` elements (size >= 0), a set of Section 1.1.1
 * (cells, edges, nodes, ...).  `name` (may be NULL) is copied.  *set_id
 * receives the id (0, 1, ... in declaration order). */
um_status um_decl_set(um_ctx ctx, int64_t size, const char *name, int32_t *set_id);

/* Declare a map from every element of `from_set` to `arity` elements of
 * `to_set` (Section 1.1.1, fixed arity).  host_table is int32
 * [size(from_set)][arity], row-major, in the sets' current numbering; it is
 * copied and validated.  Errors: UM_ERR_RANGE if an entry is outside
 * 0..size(to_set)-1, UM_ERR_ARG for a bad set id or arity outside 1..16. */
um_status um_decl_map(um_ctx ctx, int32_t from_set, int32_t to_set, int32_t arity,
                      const int32_t *host_table, int32_t *map_id);

/* Declare a dat of `dim` (1..16) values of type `dtype` per element of
 * `set` (a dat of Section 1.1.1), stored at device address `device_ptr` with
 * `layout`, in the sets' current numbering.  The memory stays owned by the
 * caller and must outlive all work that uses it.  device_ptr may be NULL on
 * a host-only context.  The kernels use vector accesses, so device_ptr must
 * be aligned: AoS records of a multiple of 16 bytes to 16, of 8 bytes to 8,
 * otherwise (and SoA) to the value size.  A dat a loop increments must not
 * share memory with a dat the same loop reads (checked when a plan is built
 * and at every execution).  Errors: UM_ERR_ARG (bad set, dim, dtype, layout,
 * null dat_id, misaligned pointer). */
um_status um_decl_dat(um_ctx ctx, int32_t set, int32_t dim, int32_t dtype, int32_t layout,
                      void *device_ptr, int32_t *dat_id);

/* Point an existing dat at another device buffer of the same shape
 * (size(set) * dim values of the dat's dtype in its layout: the caller's
 * guarantee, not checked).  Plans built earlier use the new buffer from
 * their next execution on.  Errors: UM_ERR_ARG for a bad dat id or a
 * misaligned pointer (as um_decl_dat). */
um_status um_set_dat_ptr(um_ctx ctx, int32_t dat, void *device_ptr);

/* ------------------------------------------------------------- reordering */

/* Renumber the mesh (Section 2.3).  Must be called before any dat or plan
 * exists (UM_ERR_STATE otherwise); may be called repeatedly, the
 * renumberings compose.
 *   RCM / GPS: the to-set of driving_map is renumbered by a Cuthill-McKee
 *     traversal of the graph in which the points of each element form a
 *     clique, from a pseudo-peripheral start (RCM reverses the sequence);
 *     the from-set is sorted lexicographically by its elements' sorted new
 *     point ids; every other to-set of a map from that from-set takes
 *     first-touch order over the sorted elements.
 *   PARTITION: the from-set of driving_map is split into contiguous blocks
 *     of at most block_size elements that share as little data as possible
 *     (recursive bisection along the longest extent of element coordinates,
 *     extents within 5 % of each other counting as equal with the lowest
 *     axis first: the mean of the element's points' `coords` through
 *     coord_map, or, if no coordinates are given, graph-distance
 *     coordinates from BFS landmarks on the driving map's point graph);
 *     each connected component of the elements with at least block_size
 *     elements is bisected on its own into ceil(size / block_size) blocks,
 *     smaller ones are packed whole into shared blocks; every split keeps
 *     each side at most (its share of blocks) * block_size elements, so all
 *     blocks end up at most block_size.  Elements are renumbered block by
 *     block, keeping their previous relative order inside a block.  With
 *     point_reorder, every to-set of a map from the from-set is renumbered
 *     by (number of accessing blocks, list of accessing blocks), with
 *     point_reorder = 2 by (smallest accessing block, number, list), or with
 *     point_reorder = 3 by the accessing blocks from the largest down, ties
 *     keeping the previous order.  The blocks are remembered
 *     and used by HIER plans with the same block_size, or with a multiple
 *     k * block_size (k consecutive blocks form one plan block).
 *   USER_BLOCKS: as PARTITION, but the blocks are the caller's: elements
 *     are renumbered by ascending block_of (stable), empty block ids are
 *     dropped, and every block must hold at most block_size elements
 *     (else UM_ERR_ARG); then the same point reordering and the same use
 *     by HIER plans.
 *   LEXICOGRAPHIC: only the from-set of driving_map is renumbered, by the
 *     lexicographic order of each element's sorted point ids (ties keep the
 *     previous order), e.g. boundary edges after their cells were
 *     renumbered by another loop's reordering.
 * Every map is rewritten into the new numbering. */
um_status um_reorder_mesh(um_ctx ctx, const um_reorder_opts *opts);

/* Copy the cumulative renumbering of `set` into host int32[size]:
 * host_new2old[k] = the original (declaration-time) id of current id k. */
um_status um_get_perm(um_ctx ctx, int32_t set, int32_t *host_new2old);

/* Copy the current table of `map` into host int32[from_size][arity]. */
um_status um_get_map(um_ctx ctx, int32_t map, int32_t *host_out);

/* Block partition of `set` from the last PARTITION reorder: *n_blocks
 * receives the count; if host_off is not NULL it receives int32
 * [n_blocks+1] offsets (capacity in elements).  *block_size receives the
 * size it was built for (0 if the set has no partition). */
um_status um_get_blocks(um_ctx ctx, int32_t set, int32_t *block_size, int32_t *n_blocks,
                        int32_t *host_off, int64_t capacity);

/* Device gather/scatter of a dat between the original numbering and the
 * current one (the renumbering of Section 2.3 applied to the data).  direction 0: dst[k] = src[new2old[k]] (original -> current);
 * direction 1: dst[new2old[k]] = src[k] (current -> original).  src and dst
 * are distinct device buffers of size(set)*dim values with the given dtype
 * and layout.  Asynchronous on `stream` (a hipStream_t; NULL = default). */
um_status um_permute_dat(um_ctx ctx, int32_t set, int32_t direction, const void *src, void *dst,
                         int32_t dim, int32_t dtype, int32_t layout, void *stream);

/* ----------------------------------------------------------------- plans */

/* Build an execution plan for `kernel` over `iter_set` with `args` (see
 * um_kernel for the pattern each kernel requires).  Host work (colourings,
 * blocks, staged lists, local index maps) plus one upload, after which the
 * call synchronises on its own upload.  The plan owns its device memory.
 * Errors: UM_ERR_ARITY (argument pattern), UM_ERR_ARG (bad options),
 * UM_ERR_COLOURS (HIER: block colours > max_block_colours; the paper's
 * library could not run such meshes either, Section 3.1.5), UM_ERR_LDS (HIER:
 * a block's staging exceeds lds_limit_bytes and no fallback is allowed). */
um_status um_plan_build(um_ctx ctx, int32_t kernel, const um_arg *args, int32_t nargs,
                        int32_t iter_set, const um_plan_opts *opts, um_plan *out);

/* Copy the plan's statistics (um_plan_stats, fields listed there) to *out.
 * Errors: UM_ERR_ARG for a null out. */
um_status um_plan_stats_get(um_plan plan, um_plan_stats *out);

/* Copy plan contents to host memory for verification.  *n_out receives the
 * number of int32 values of the field; if host_out is not NULL and capacity
 * suffices they are copied, otherwise UM_ERR_ARG after setting *n_out. */
um_status um_plan_export(um_plan plan, int32_t field, int32_t *host_out, int64_t capacity,
                         int64_t *n_out);

/* Release the plan and its device memory after a device synchronisation
 * (so work already enqueued with it completes first).  NULL is accepted. */
um_status um_plan_destroy(um_plan plan);

/* Execute the loop once on `stream` (hipStream_t, NULL = default stream),
 * incrementing the INC dats (they are not cleared): the loop of Section
 * 1.1.1 over every element of the iteration set, executed by the plan's
 * strategy (Section 2.1; HIER: Algorithm 1 of Section 2.2 per block, block
 * colours ordered by kernel launches or by the DATAFLOW schedule).  Asynchronous; the
 * dats bound to the plan's args must stay valid until the work completes.
 * params: kernel constants (listed with each um_kernel).  Errors: UM_ERR_STATE on a
 * host-only context or a dat without device memory, UM_ERR_HIP on launch
 * failure. */
um_status um_loop_exec(um_plan plan, const double *params, int32_t nparams, void *stream);

/* um_loop_exec for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * executes the plan once like um_loop_exec, but the kernels' scratch memory
 * (the DATAFLOW completion flags and control words; the UPDATE loops'
 * per-workgroup partial sums) is a static device array of 256 KiB that the
 * library holds on each GPU it runs on, instead of the plan's own buffers.
 * The call allocates nothing.  Before a DATAFLOW launch the flags and control
 * words are cleared by a kernel (so every such call is execution 1 of its
 * own), and a give-up count of the call is added to the plan's count
 * (um_plan_errors).  Limits: DATAFLOW plans of at most 65,471 blocks, UPDATE
 * plans of at most 32,768 workgroups; larger plans give UM_ERR_ARG.  All
 * calls on one GPU share the array: calls that overlap in time on one GPU
 * (different streams, or several host threads) race and give wrong results.
 * Other plans use no scratch and run exactly as with um_loop_exec.  Errors
 * as um_loop_exec, and UM_ERR_ARG over the limits. */
um_status um_loop_exec_static(um_plan plan, const double *params, int32_t nparams, void *stream);

/* Autotuning: build a plan for each of the n_candidates option sets, run
 * each once untimed and then `reps` times between two HIP events on
 * `stream`, keep the fastest plan in *out and destroy the others.  The
 * loop's written dats (INC, WRITE, RW) are modified by the trial runs: the
 * caller re-initialises them afterwards.  A candidate whose build fails
 * with UM_ERR_LDS, UM_ERR_COLOURS, UM_ERR_UNSUPPORTED or UM_ERR_ARG, or
 * whose DATAFLOW waits time out, is skipped (its time is -1).
 * *best_index receives the chosen candidate; ms_out, if not NULL, receives
 * n_candidates mean times per execution in ms.  Synchronises the device.
 * Errors: UM_ERR_UNSUPPORTED when no candidate could be built, others as
 * um_plan_build and um_loop_exec. */
um_status um_plan_autotune(um_ctx ctx, int32_t kernel, const um_arg *args, int32_t nargs,
                           int32_t iter_set, const um_plan_opts *candidates,
                           int32_t n_candidates, const double *params, int32_t nparams,
                           void *stream, int32_t reps, int32_t *best_index, double *ms_out,
                           um_plan *out);

/* Timing of the plan's launches: when enabled, um_loop_exec records a HIP
 * event pair around every kernel launch; um_plan_timing waits for them and
 * returns the summed kernel time in ms and the number of launches timed
 * since the last reset, then resets. */
um_status um_plan_set_timing(um_plan plan, int32_t enable);

/* Synchronise the device and return in *n_errors the number of block
 * waits of a DATAFLOW plan that gave up on a neighbour since the plan was
 * built or um_plan_reset_errors was last called; 0 for other plans.  An
 * execution in which a wait gave up has read and written its increment
 * targets without ordering, so its results (and every result accumulated
 * on them afterwards) are invalid; the waits of later executions are not
 * affected (each execution has its own epoch).  Errors: UM_ERR_ARG for a
 * null output, UM_ERR_HIP. */
um_status um_plan_errors(um_plan plan, int32_t *n_errors);

/* Synchronise the device and set the plan's count of given-up waits back
 * to zero.  No-op for plans other than DATAFLOW. */
um_status um_plan_reset_errors(um_plan plan);

/* Longest time a DATAFLOW block waits for one neighbour before it gives up
 * and counts an error, in ticks of the GPU's 100 MHz real-time counter;
 * 0 restores the default (20,000,000 = 0.2 s).  A limit far below a
 * block's run time makes waits give up on purpose (a test of the error
 * path; the kernels always exit).  Errors: UM_ERR_ARG for ticks < 0. */
um_status um_plan_set_wait_limit(um_plan plan, int64_t ticks);
/* See um_plan_set_timing: waits for the recorded event pairs, returns their
 * summed time and count, and resets.  Errors: UM_ERR_ARG for null outputs. */
um_status um_plan_timing(um_plan plan, double *ms_total, int64_t *n_launches);

/* Verification entry point: evaluate the elemental flux of every element of
 * the iteration set (current numbering) with floating-point contraction
 * disabled, writing f[n_elements][4] (UM_F64, element-major) to the device
 * buffer f_out.  Used to compare per-edge values bit for bit with a
 * sequential evaluation of the same formula.  Asynchronous on `stream`. */
um_status um_debug_fluxes(um_plan plan, const double *params, int32_t nparams, void *f_out,
                          void *stream);

/* ------------------------------------------------------------ HIP graphs */

/* Capture of the library's launches into a HIP graph, so that a time step of
 * several loops (the batched and time-step loops of Section 3.1.1's solver
 * structure) is replayed with one graph launch.  Between um_graph_begin and
 * um_graph_end on a capturing `stream` (a hipStream_t other than the NULL
 * stream), um_loop_exec on that stream records its kernels instead of
 * running them; nothing else may be enqueued on the stream meanwhile, and a
 * DATAFLOW plan's epochs advance once per replay as with eager executions.
 * Plan timing (um_plan_set_timing) must be off while capturing.  The graph
 * refers to the plans and dats by address: they must outlive it.
 * Errors: UM_ERR_ARG (NULL stream, null output), UM_ERR_HIP. */
um_status um_graph_begin(void *stream);
/* End the capture on `stream` and instantiate it; *out receives the graph. */
um_status um_graph_end(void *stream, um_graph *out);
/* Enqueue one replay of `graph` on `stream` (NULL = default stream). */
um_status um_graph_launch(um_graph graph, void *stream);
/* Release the graph (NULL accepted); replays already enqueued complete. */
um_status um_graph_destroy(um_graph graph);

#ifdef __cplusplus
}
#endif

#endif /* UMESH_H */
