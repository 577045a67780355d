/*
 * dsg.h - C ABI of libdsg.so: Bahmani's (2+2eps)-approximate densest
 * subgraph peeling on one AMD Instinct MI355X (gfx950).
 *
 * Method (Section 3.1 of De Zoysa et al., "Parallel Algorithms for Densest
 * Subgraph Discovery Using Shared Memory Model", Algorithm 1 "P-Bahmani";
 * the approximation algorithm of Bahmani, Kumar and Vassilvitskii it
 * parallelises): the current graph starts as G.  Each pass removes, all at
 * once, every vertex whose degree inside the current graph is at most
 * 2(1+eps) times the current edge density rho = |E| / |V| (Definition 1),
 * decrements the degrees of their surviving neighbours, and keeps the
 * densest intermediate graph seen so far.  Passes repeat until no vertex is
 * left.  The kept graph S~ satisfies rho(S~) >= rho*(G) / (2 + 2 eps)
 * (Definition 3) and O(log_{1+eps} n) passes suffice.
 *
 * Exactness: eps = eps_num / eps_den is a rational and every test is done in
 * integers.  A vertex of degree d fails a pass that starts with |V| vertices
 * and |E| edges when d * |V| * eps_den <= 2 (eps_num + eps_den) |E|.  An edge
 * whose two ends fail in the same pass is removed once.  The whole graph is
 * the pass-0 candidate; a later graph replaces the best only when its density
 * is strictly larger.  "passes" counts every pass, including the one that
 * empties the graph.  Results are fully deterministic (no floating point, no
 * order dependence).
 *
 * Input graph: vertices 0..n-1, undirected, simple, stored as a symmetric
 * int32 CSR (both directions of every edge) with ascending neighbours in
 * every row and no self loops.  row_ptr has n+1 entries with row_ptr[0] = 0
 * and row_ptr[n] = 2m.  Isolated vertices count in n.
 *
 * Memory: pointers documented as "device" must point to device memory of the
 * current HIP device; "host" pointers to host memory.  The library never
 * frees or keeps caller memory.  Calls with distinct workspaces may run
 * concurrently on different streams.
 *
 * Errors: every entry point returns DSG_OK (0) or a negative dsg_status.
 * Argument checks run before any HIP call.  No C++ exception crosses this
 * boundary.
 */
#ifndef DSG_H
#define DSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DSG_OK = 0,
    DSG_EINVAL = -1,      /* bad argument, too small workspace, or an input
                             that violates the CSR contract when detected */
    DSG_EOVERFLOW = -2,   /* sizes or eps outside the exact int64 range */
    DSG_ENOMEM = -3,      /* device allocation failed */
    DSG_EDEVICE = -4,     /* a HIP runtime call failed */
    DSG_EINTERNAL = -5    /* pass watchdog or invariant check tripped */
} dsg_status;

/* Graph in device memory, borrowed read-only for the duration of a call. */
typedef struct {
    const int32_t* row_ptr; /* device, n+1 entries */
    const int32_t* col_idx; /* device, 2m entries */
} dsg_csr;

/* Result of one peel (host struct). */
typedef struct {
    int64_t dens_num;  /* |E(S~)|, unreduced numerator of rho(S~)        */
    int64_t dens_den;  /* |S~|, unreduced denominator (0 only when n = 0) */
    int32_t passes;    /* passes until the graph was empty (0 when n = 0) */
    int32_t best_pass; /* S~ is the graph left after this pass (0 = G)    */
    int64_t best_size; /* |S~| = number of result ids at the front of best_ids */
} dsg_result;

/* One pass, as recorded when a trace is requested (host struct). */
typedef struct {
    int64_t s_in;    /* |V| at the start of the pass */
    int64_t e_in;    /* |E| at the start of the pass */
    int64_t thresh;  /* floor(2(num+den)|E| / (|V| den)), capped at INT32_MAX */
    int64_t removed; /* vertices that failed */
    int64_t cross;   /* adjacency entries from failed vertices to survivors */
    int64_t intra;   /* adjacency entries between failed vertices (even)   */
    int64_t walked;  /* adjacency entries the GPU walked in this pass      */
    int64_t s_out;   /* |V| after the pass */
    int64_t e_out;   /* |E| after the pass */
} dsg_pass_trace;

/* Launch shape overrides; 0 selects the library default.  Results never
 * depend on these. */
typedef struct {
    int32_t mark_grid;  /* workgroups of the mark / extract kernels */
    int32_t walk_grid;  /* workgroups of the neighbour-walk kernels (at most 4096 are used) */
    int32_t pass_batch; /* 0: a peel runs one pass ahead of the device (each
                         * pass's tile scan posts to a pinned host word whether
                         * the pass leaves survivors, and the host then
                         * enqueues the next pass); > 0: passes are enqueued in
                         * batches of this many (doubling up to 64) with a host
                         * check after each.  CBDS-P always uses batches. */
    int32_t flags;      /* DSG_LAUNCH_* bits */
} dsg_launch;

/* Keep degree-update records in per-bin regions (one device atomic per
 * record) instead of per-tile regions.  The library does this by itself when
 * a pass leaves more than 1024 * 32768 survivors (and does not key the
 * records by neighbour id); the flag forces it and turns the id keying off. */
#define DSG_LAUNCH_BIN_REGIONS 1

/* The tile scan posts no progress, so a peel running one pass ahead of the
 * device waits for a post that does not come: after 20 ms with the stream
 * idle it finishes with batches of passes.  For testing that path. */
#define DSG_LAUNCH_NO_PROGRESS 2

/* Degree-update records keyed by neighbour id.  In a pass that leaves more
 * than 65536 survivors and walks at least 2^25 adjacency entries (graphs of
 * at most 2^25 vertices, not CBDS-P), the walk writes every walked entry as
 * its neighbour's position in a bucket of 32768 consecutive ids, and the
 * degree update finds the survivors among them, instead of the walk looking
 * up each neighbour's survivor rank.  DSG_LAUNCH_ID_BUCKETS uses this in
 * every peel pass that leaves a survivor, whatever the survivor count and
 * walk length; DSG_LAUNCH_NO_ID_BUCKETS never uses it. */
#define DSG_LAUNCH_ID_BUCKETS 4
#define DSG_LAUNCH_NO_ID_BUCKETS 8

/* Optional per-kernel timing, measured with HIP events on the call's stream
 * around every launch of the call (host struct, filled on return).  Launches
 * enqueued after the last pass return at once and are counted too. */
typedef struct {
    double ms_init;     /* init kernels */
    double ms_mark;     /* mark-count + tile-scan + mark-scatter kernels */
    double ms_walk;     /* neighbour-walk kernel */
    double ms_apply;    /* pass completion and degree-update kernels (sum of the walk's
                           partial counts, per-bin LDS counts, degree reduction) */
    double ms_extract;  /* extract kernels */
    double ms_total;    /* first launch to last kernel end */
    int32_t launches_walk;
    int32_t launches_mark;
    int32_t launches_apply;
    int32_t reserved;
    int64_t walked;       /* adjacency entries walked over all passes */
    int64_t cross;        /* degree decrements over all passes */
    int64_t live_scanned; /* live-list entries tested over all passes */
    int64_t walk_list;    /* failed vertices whose rows were walked, all passes */
} dsg_profile;

/* Library ABI version (increments on any incompatible change). */
int32_t dsg_version(void);

/* Human-readable text of a dsg_status; never NULL. */
const char* dsg_strerror(int32_t status);

/* Bytes of device workspace dsg_peel needs for a graph with n vertices and
 * m undirected edges; 0 for invalid sizes.  About 28 n + 4 m bytes, plus
 * 2 * (ceil(2m / 2048) + 1) * (min(ceil(n / 32768) + 1, 1024) + 1) bytes of
 * per-tile bin offsets, min(n, 32768) * 4 bytes per degree-update work item
 * (at most n / 32768 + 514 items) and about 40 KB of fixed tables. */
size_t dsg_workspace_bytes(int64_t n, int64_t m);

/*
 * Peel g with eps = eps_num / eps_den (eps_num >= 0, eps_den >= 1) and
 * return S~ and its density.
 *
 *   g           CSR as above (device pointers).
 *   n, m        vertices and undirected edges; the kernels check
 *               row_ptr[0] = 0 and row_ptr[n] = 2m (DSG_EINVAL otherwise).
 *   best_ids    device, room for n int32; receives S~ in ascending order
 *               (out->best_size entries; the entries after them are
 *               overwritten with earlier candidates and hold no result).
 *               May be NULL to skip extraction.
 *   out         host; filled on DSG_OK.
 *   workspace   device, at least dsg_workspace_bytes(n, m) bytes, 256-byte
 *               aligned; NULL makes the library allocate and free it.
 *   stream      a hipStream_t (NULL = the null stream).  All device work is
 *               ordered on it; the call returns after *out is valid.
 *
 * Errors: DSG_EINVAL for NULL pointers where data is needed, n < 0, m < 0,
 * eps_den < 1, eps_num < 0 or a short workspace; DSG_EOVERFLOW when
 * n > INT32_MAX - 1, 2m > INT32_MAX, 2(eps_num + eps_den) m >= 2^63 or
 * n eps_den >= 2^63; DSG_EDEVICE / DSG_ENOMEM for HIP failures;
 * DSG_EINTERNAL when the pass watchdog (more passes than the
 * O(log_{1+eps} n) bound of Section 3.1 allows) or an edge-count invariant
 * trips, which only an input violating the CSR contract can cause.
 */
int32_t dsg_peel(const dsg_csr* g, int64_t n, int64_t m, int64_t eps_num, int64_t eps_den,
                 int32_t* best_ids, dsg_result* out, void* workspace, size_t ws_bytes,
                 void* stream);

/*
 * dsg_peel with optional extras (each may be NULL / 0):
 *   removed_at  device, n int32: the pass in which each vertex failed
 *               (S~ = { v : removed_at[v] > best_pass }).
 *   trace       host, trace_cap records: one dsg_pass_trace per pass, for
 *               the first min(passes, trace_cap, 4096) passes.
 *   launch      host: launch shape overrides.
 *   prof        host: per-kernel timing (adds HIP events between launches).
 */
int32_t dsg_peel_ex(const dsg_csr* g, int64_t n, int64_t m, int64_t eps_num, int64_t eps_den,
                    int32_t* best_ids, int32_t* removed_at, dsg_result* out,
                    dsg_pass_trace* trace, int32_t trace_cap, const dsg_launch* launch,
                    dsg_profile* prof, void* workspace, size_t ws_bytes, void* stream);

/*
 * Check on the device that g satisfies the input contract above (O(m log d)
 * work; for debugging and loaders).  Returns DSG_OK, DSG_EINVAL with
 * *detail set to the first violated rule (1 row_ptr[0] != 0, 2 row_ptr not
 * monotone, 3 row_ptr[n] != 2m, 4 neighbour id out of range, 5 self loop,
 * 6 row not strictly ascending, 7 missing reverse edge), or a HIP error.
 * `detail` (host) may be NULL.  Allocates a few bytes of device memory.
 */
int32_t dsg_validate_csr(const dsg_csr* g, int64_t n, int64_t m, int32_t* detail, void* stream);

/* ------------------------------------------------------------------------
 * CBDS-P (Section 3.2, Algorithm 2): the densest k-core, extended by the
 * outside vertices that raise its density.
 *
 * Phase 1 peels k-core levels: for k = 0, 1, ... every vertex of degree <= k
 * is removed, repeatedly, until none is left (the PKC level loop); the
 * remaining graph is then the (k+1)-core, and the next level is the least
 * degree left.  A vertex removed at level k has core number k.  The densest
 * core C_K is the non-empty core of greatest density |E|/|V|, the smallest
 * order K among equal densities (the whole graph, K = 0, included).
 *
 * Phase 2: with rho = |E(C_K)| / |C_K|, an outside vertex v is eligible when
 * its core number exceeds rho, and legitimate when it has more than rho
 * neighbours in C_K.  All legitimate vertices L join at once: the result is
 * S = C_K u L, with |E(S)| = |E(C_K)| + (edges from L into C_K) + |E(L)|.
 * Every comparison is exact (int64 cross-multiplication).
 * ------------------------------------------------------------------------ */

/* Result of dsg_cbds (host struct). */
typedef struct {
    int64_t dens_num;   /* |E(S)| of the result S = C_K u L */
    int64_t dens_den;   /* |S| */
    int64_t core_num;   /* |E(C_K)| */
    int64_t core_den;   /* |C_K| */
    int32_t core_k;     /* K, the order of the densest core */
    int32_t kmax;       /* the largest core number */
    int32_t passes;     /* phase-1 passes (removal rounds and level ends) */
    int32_t reserved;
    int64_t n_eligible; /* outside vertices with core number > rho */
    int64_t n_legit;    /* |L| */
    int64_t best_size;  /* ids written to best_ids (|S|, or 0 without best_ids) */
} dsg_cbds_result;

/*
 * Run CBDS-P on g (CSR as for dsg_peel).
 *
 *   best_ids   device, room for n int32, or NULL: S in ascending order.
 *   core       device, n int32, or NULL: the core number of every vertex.
 *   out        host; filled on DSG_OK.
 *   trace      host, trace_cap records, or NULL: one dsg_pass_trace per
 *              phase-1 pass (thresh is the level k).
 *   workspace  device, >= dsg_workspace_bytes(n, m) bytes, 256-byte
 *              aligned; NULL makes the library allocate and free it.
 *
 * Errors as for dsg_peel (eps does not apply); the pass watchdog is 2n + 2
 * phase-1 passes.
 */
int32_t dsg_cbds(const dsg_csr* g, int64_t n, int64_t m, int32_t* best_ids, int32_t* core,
                 dsg_cbds_result* out, dsg_pass_trace* trace, int32_t trace_cap,
                 void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched peeling: many independent graphs in one persistent launch.
 *
 * Every graph of a batch is peeled exactly as dsg_peel peels it (same
 * passes, same S~, same density); the batch only changes how the work is
 * scheduled.  Graphs are stored back to back in three caller arrays:
 *
 *   row_ptr  device int32: graph g's n+1 row offsets start at
 *            graphs[g].row_ptr_off and are local to the graph (its first
 *            entry is 0, its last 2m).
 *   col_idx  device int32: its 2m neighbour ids (local, 0..n-1) start at
 *            graphs[g].col_idx_off.
 *   best_ids / removed_at
 *            device int32: graph g owns n slots from graphs[g].out_off; the
 *            slot ranges of different graphs must not overlap.
 *
 * A persistent workgroup takes the next graph from a device queue ordered
 * by decreasing size and runs all of that graph's passes: the mark, the
 * neighbour walk and the degree update of Algorithm 1 (Section 3.1) with
 * workgroup barriers in place of the paper's global barrier, and the degree
 * and presence state of the graph's vertices held in LDS.
 * ------------------------------------------------------------------------ */

/* One graph of a batch (host struct). */
typedef struct {
    int64_t row_ptr_off; /* first of the graph's n+1 entries in row_ptr    */
    int64_t col_idx_off; /* first of its 2m entries in col_idx              */
    int64_t out_off;     /* first of its n slots in best_ids / removed_at   */
    int64_t n;           /* vertices */
    int64_t m;           /* undirected edges */
    int64_t eps_num;     /* eps = eps_num / eps_den, per graph              */
    int64_t eps_den;
    int64_t reserved;    /* must be 0 */
} dsg_batch_graph;

/* Result of one graph of a batch (device struct, written by the kernel). */
typedef struct {
    int64_t dens_num;  /* |E(S~)| */
    int64_t dens_den;  /* |S~| */
    int32_t passes;
    int32_t best_pass;
    int64_t best_size; /* ids written to the graph's best_ids slots */
    int32_t status;    /* DSG_OK; DSG_EINVAL when the device found the graph's
                          row_ptr or col_idx outside the CSR contract;
                          DSG_EINTERNAL when the pass watchdog or an
                          edge-count invariant tripped */
    int32_t reserved;
} dsg_batch_result;

/* Launch shape of the persistent kernel; 0 selects the library default
 * (512 threads, one workgroup per CU, 8 entries per lane).  Results never
 * depend on these. */
typedef struct {
    int32_t block;         /* threads per workgroup: 256, 512 or 1024        */
    int32_t blocks_per_cu; /* workgroups resident per CU (LDS is split): 1..8 */
    int32_t grid;          /* persistent workgroups (default CUs x blocks_per_cu) */
    int32_t walk_items;    /* adjacency entries per lane per walk tile: 4, 8 or 16
                              (16 only with 256 or 512 threads) */
} dsg_batch_launch;

/* A prepared batch (host struct, filled by dsg_batch_prepare and only read
 * afterwards).  It refers to the workspace, which must stay allocated and
 * unmodified while the plan is used. */
typedef struct {
    int32_t count;        /* graphs */
    int32_t block;        /* chosen launch shape */
    int32_t blocks_per_cu;
    int32_t grid;
    int32_t walk_items;
    int32_t lds_bytes;    /* dynamic LDS per workgroup (vertex states) */
    int32_t lds_vertices; /* vertices per graph whose state lives in LDS */
    int32_t state_bits;   /* 16, or 8 when the batch's largest graph has more
                             vertices than 16-bit states fit in the LDS
                             (degrees of 240 and more then sit in an LDS
                             hash table) */
    int64_t out_len;      /* slots of best_ids / removed_at */
    void* workspace;
    uint64_t ws_bytes;
    int64_t reserved[4];
} dsg_batch_plan;

/* Device workspace bytes for a batch of `count` graphs with `entries`
 * adjacency entries in total (the sum of 2m over the batch) whose output
 * slots span out_len entries: 24 bytes per slot, 64 bytes per graph and
 * 4 bytes per 256 adjacency entries (plus 8 per graph); 0 for invalid
 * sizes. */
size_t dsg_batch_workspace_bytes(int32_t count, int64_t entries, int64_t out_len);

/*
 * Check a batch on the host, order it for the device queue and upload its
 * table into the workspace.  Synchronises `stream` once (the upload), makes
 * no allocation, and fills *plan.
 *
 *   graphs       host, count entries (count >= 0).
 *   row_ptr_len, col_idx_len, out_len
 *                entries of the caller's row_ptr, col_idx and best_ids /
 *                removed_at arrays; every graph's ranges must lie inside.
 *   launch       host or NULL.
 *   workspace    device, >= dsg_batch_workspace_bytes(count, sum of 2m,
 *                out_len) bytes, 256-byte aligned.
 *
 * Errors: DSG_EINVAL for NULL pointers, count < 0, a short or misaligned
 * workspace, a range outside its array, overlapping output ranges, a
 * nonzero reserved field or an unsupported launch shape; DSG_EOVERFLOW
 * when a graph fails the size limits of dsg_peel; DSG_EDEVICE for HIP
 * failures.
 */
int32_t dsg_batch_prepare(const dsg_batch_graph* graphs, int32_t count, int64_t row_ptr_len,
                          int64_t col_idx_len, int64_t out_len, const dsg_batch_launch* launch,
                          void* workspace, size_t ws_bytes, void* stream, dsg_batch_plan* plan);

/*
 * Peel every graph of a prepared batch: two kernel launches on `stream`,
 * no host synchronisation and no allocation, so the call can be captured
 * into a HIP graph and replayed.  On completion results[i] (device, count
 * entries, indexed like the caller's table) holds graph i's result and its
 * best_ids slots hold S~ in ascending local ids.
 *
 *   row_ptr, col_idx  device batch arrays described to dsg_batch_prepare.
 *   best_ids          device, out_len entries, or NULL to skip extraction.
 *   removed_at        device, out_len entries, or NULL; receives the pass in
 *                     which every vertex failed.
 *
 * Errors: DSG_EINVAL for a NULL plan or results or a plan that was not
 * filled by dsg_batch_prepare; DSG_EDEVICE when a launch fails.  Per-graph
 * problems are reported in results[i].status.  Calls sharing a workspace
 * must be ordered (same stream).
 */
int32_t dsg_batch_run(const dsg_batch_plan* plan, const int32_t* row_ptr, const int32_t* col_idx,
                      int32_t* best_ids, int32_t* removed_at, dsg_batch_result* results,
                      void* stream);

/* ------------------------------------------------------------------------
 * The exact densest subgraph (Section 2: Goldberg's max-flow construction,
 * the exact method the (2 + 2 eps) guarantee is measured against).
 *
 * For a guess rho = p/q, Goldberg's network has a source, a sink and the
 * graph's vertices; a minimum cut's source side S maximises
 * q |E(S)| - p |S|.  Dinkelbach's iteration starts from the density of G
 * and moves to the density of the cut side while that is strictly larger;
 * at the optimum the largest minimum-cut source side is the largest
 * densest subgraph S* (the union of every subset of greatest density).
 * Each maximum flow is a push-relabel preflow on the device.
 * ------------------------------------------------------------------------ */

/* Result of dsg_exact_density (host struct). */
typedef struct {
    int64_t dens_num;  /* |E(S*)| */
    int64_t dens_den;  /* |S*| (n when the graph has no edge; 0 when n = 0) */
    int64_t set_size;  /* ids written to set_ids (|S*|, or 0 without set_ids) */
    int32_t flows;     /* maximum flows solved (Dinkelbach steps) */
    int32_t relabels;  /* global relabels over all flows */
} dsg_exact_result;

/* Device workspace bytes of dsg_exact_density for n vertices and m edges:
 * 12 per adjacency entry (2m of them), 20 per vertex and small tables; 0
 * for invalid sizes. */
size_t dsg_exact_workspace_bytes(int64_t n, int64_t m);

/*
 * The exact maximum density rho* = |E(S*)| / |S*| of g and the largest
 * densest subgraph S*.
 *
 *   g, n, m     CSR as for dsg_peel (device pointers).
 *   set_ids     device, room for n int32, or NULL: S* in ascending order.
 *   out         host; filled on DSG_OK.
 *   workspace   device, >= dsg_exact_workspace_bytes(n, m) bytes, 256-byte
 *               aligned; NULL makes the library allocate and free it.
 *   stream      a hipStream_t; the call returns when the result is final
 *               (it synchronises the stream between the steps of a flow).
 *
 * Errors: DSG_EINVAL / DSG_EOVERFLOW for the argument errors of dsg_peel;
 * DSG_ENOMEM / DSG_EDEVICE for HIP failures; DSG_EINTERNAL if a flow or the
 * iteration exceeds its step bound or the optimum's cut side is not of the
 * optimum density (only a CSR outside the contract can cause that).
 */
int32_t dsg_exact_density(const dsg_csr* g, int64_t n, int64_t m, int32_t* set_ids,
                          dsg_exact_result* out, void* workspace, size_t ws_bytes,
                          void* stream);

/* ------------------------------------------------------------------------
 * Peeling without the host.
 * ------------------------------------------------------------------------ */

/*
 * dsg_peel without the host: every pass of Algorithm 1 (Section 3.1) runs
 * in device work enqueued on `stream` up front, and the call returns once
 * it is enqueued.  No host synchronisation, no allocation and no host
 * memory: the call can be captured into a HIP graph and replayed.
 *
 * The loop "while |V| > 0" runs on the device: the first passes are the
 * seven kernels of dsg_peel, each becoming a no-op once the graph is empty
 * (16 of them, or launch->pass_batch when set, at most the pass bound);
 * if the pass bound allows more, one workgroup then runs every remaining
 * pass in a device loop until the graph is empty (or the watchdog or an
 * invariant stops it).  Results equal dsg_peel's.
 *
 *   g, n, m, eps_num, eps_den, best_ids, removed_at
 *               as for dsg_peel_ex (best_ids and removed_at may be NULL).
 *   result      device, one dsg_batch_result (the struct of a batch's
 *               per-graph result): written by the last kernel of the call
 *               with status DSG_OK, DSG_EINVAL (row_ptr outside the CSR
 *               contract) or DSG_EINTERNAL (watchdog or invariant), the
 *               density (|E(S~)|, |S~|; 0 unless DSG_OK), passes, best pass
 *               and the number of ids in best_ids.
 *   launch      host or NULL: grid overrides as for dsg_peel_ex;
 *               pass_batch is the number of passes enqueued as kernels
 *               (>= 1); flags as for dsg_peel_ex except that no progress is
 *               ever posted.
 *   workspace   device, at least dsg_workspace_bytes(n, m) bytes, 256-byte
 *               aligned (required: the call allocates nothing).  It must
 *               not be used by other work until the enqueued work is done.
 *
 * Returns DSG_OK once enqueued; DSG_EINVAL / DSG_EOVERFLOW for the argument
 * errors of dsg_peel plus a NULL result or workspace; DSG_EDEVICE if a
 * launch fails.  Problems the device finds are reported in *result.
 */
int32_t dsg_peel_async(const dsg_csr* g, int64_t n, int64_t m, int64_t eps_num,
                       int64_t eps_den, int32_t* best_ids, int32_t* removed_at,
                       dsg_batch_result* result, const dsg_launch* launch,
                       void* workspace, size_t ws_bytes, void* stream);

/*
 * dsg_peel_async for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same work and results as dsg_peel_async, with the workspace taken
 * from a static device array of 256 MiB that the library holds on every
 * GPU it runs on until the process ends.  The caller still passes the graph,
 * best_ids, removed_at and the device result as for dsg_peel_async.
 *
 * The graph must fit the array: dsg_workspace_bytes(n, m) <= 256 MiB
 * (about n = 2^20 vertices with m = 16 M edges); larger graphs return
 * DSG_EINVAL.  Every call on one GPU uses that GPU's array, and the array
 * keeps what the last call left (the peel initialises what it reads), so
 * calls that overlap on one GPU (other streams, other threads) race: order
 * them.  Allocates nothing; the first call on a device looks up the
 * array's device address.  Errors as for dsg_peel_async.
 */
int32_t dsg_peel_async_noalloc(const dsg_csr* g, int64_t n, int64_t m, int64_t eps_num,
                               int64_t eps_den, int32_t* best_ids, int32_t* removed_at,
                               dsg_batch_result* result, const dsg_launch* launch,
                               void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DSG_H */
