/*
 * sphview.h -- C-ABI of libsphview.so: temporary, local AoS-to-SoA views around
 * SPH particle-interaction kernels, on AMD Instinct MI355X (gfx950).
 *
 * The problem statement follows the paper's formalism (Sec. 4, eq. "view"):
 * a user array D of N structs (records of a fixed byte stride) and a loop body f
 * over it are evaluated as
 *
 *     f(D) = (W_out o C^T o f_hat o C o N_{in u out}) (D)
 *
 * where N narrows each record to the members the loop reads (A_in) or writes
 * (A_out), C converts AoS to SoA (into explicit storage, Sec. 4.2), f_hat is the
 * loop over the converted data, C^T converts back and W_out widens only the
 * written members into the records.  Here:
 *
 *   sphv_view_create   plans the explicit storage of one view   (Sec. 3.1)
 *   sphv_aos_to_soa    N then C: gather of A_in                 (Sec. 3.1 prologue)
 *   sphv_sph_density   f_hat for the density loop               (Sec. 2.1 step 1)
 *   sphv_sph_force     f_hat for the force loop                 (Sec. 2.1 step 2)
 *   sphv_step_reduce   CFL time step and conservation sums      (Sec. 2.1, leapfrog)
 *   sphv_soa_to_aos   C^T then W: scatter of A_out only        (Sec. 3.1 epilogue)
 *   sphv_kick_drift    the linear kick / drift / kick updates   (Sec. 2.1 steps 3-5)
 *
 * and sphv_cells_build sorts particles into cells (Sec. 2.1, the mesh helper) so
 * that a local cell's active set is its neighbour cells (Sec. 2.3).
 *
 * Conventions for every entry point:
 *  - Return value: SPHV_OK (0) or a negative SPHV_E_* code; no C++ exception
 *    crosses this boundary.  sphv_status_string() names a code.
 *  - "device" pointers are HIP device memory of the current device; the caller
 *    owns them (AoS, workspaces, state block) and keeps them alive while any
 *    handle or queued work uses them.  The library never allocates or frees
 *    device memory; it allocates only small host handles freed by *_destroy.
 *  - The records (aos_dev) may also be managed memory or pinned host memory
 *    that the device maps at the same address (hipHostMalloc): every record
 *    access then crosses the host link, which the views limit to one per
 *    member per loop (Sec. 7.5 compares such placements).  A call that is
 *    about to enqueue work on records checks their first and last bytes with
 *    hipPointerGetAttributes and fails with SPHV_E_INVALID_ARG, before
 *    enqueuing anything, on memory the device cannot address (pageable
 *    host memory, another device's memory); a view is checked at its first
 *    gather or loop call.
 *  - "stream" is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is enqueued asynchronously on it; only sphv_read_state and
 *    sphv_write_state synchronise with the host.
 *  - Asynchronous conditions (non-finite input, h iteration not converged, ...)
 *    set SPHV_F_* bits in the device state block instead of returning errors.
 */
#ifndef SPHVIEW_H
#define SPHVIEW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */

enum {
    SPHV_OK = 0,
    SPHV_E_INVALID_ARG = -1,   /* NULL pointer, negative size, bad enum value        */
    SPHV_E_DESCRIPTOR = -2,    /* field outside the record, overlap, misaligned,     */
                               /* unsupported dtype, missing role the loop needs     */
    SPHV_E_WORKSPACE = -3,     /* workspace too small or misaligned (256 B)          */
    SPHV_E_ALIAS = -4,         /* another open view on the same records writes what  */
                               /* this one reads or writes, or vice versa (Sec. 3.3) */
    SPHV_E_STATE = -5,         /* call out of order (e.g. density before gather)     */
    SPHV_E_HIP = -6,           /* a HIP runtime call or kernel launch failed         */
    SPHV_E_UNSUPPORTED = -7    /* valid request this build does not implement       */
};

/* bits of sphv_state.flags (sticky until sphv_state_init) */
enum {
    SPHV_F_NONFINITE_INPUT = 1u << 0,  /* NaN/inf position or h seen by cells_build     */
    SPHV_F_H_NOT_CONVERGED = 1u << 1,  /* some particle used all max_iter density passes */
    SPHV_F_H_CAP_HIT = 1u << 2,        /* h wanted to exceed its cell reach: use a     */
                                       /* coarser grid or a larger headroom            */
    SPHV_F_QUEUE_OVERFLOW = 1u << 3,   /* work items exceeded the planned capacity      */
    SPHV_F_NONFINITE_OUTPUT = 1u << 4, /* NaN/inf density or force result               */
    SPHV_F_GRID_TOO_SMALL = 1u << 5,   /* a reach window wraps onto itself (periodic)   */
    SPHV_F_LIST_MISMATCH = 1u << 7,    /* symmetric force: a pair in one particle's list */
                                       /* but not its partner's (never expected)        */
    SPHV_F_OUT_OF_BOX = 1u << 6        /* a particle lies outside an open box, or       */
                                       /* outside [lo, lo+len) on a periodic axis: the  */
                                       /* records must hold wrapped coordinates (such a */
                                       /* particle is binned into an edge cell, and     */
                                       /* pairs across that face may be missed)         */
};

const char* sphv_status_string(int32_t status);
int32_t sphv_version(void);   /* 100 * major + minor */

/* ------------------------------------------------------------ descriptor */

enum { SPHV_F64 = 1, SPHV_F32 = 2, SPHV_I64 = 3, SPHV_I32 = 4 };
/* A_in only, A_out only, A_in and A_out (one instance in the view, Sec. 3.3) */
enum { SPHV_IN = 1, SPHV_OUT = 2, SPHV_INOUT = 3 };

/* Role of a member in the SPH loops; SPHV_ROLE_USER for any other member. */
enum {
    SPHV_ROLE_USER = 0,
    SPHV_X, SPHV_Y, SPHV_Z, SPHV_VX, SPHV_VY, SPHV_VZ, SPHV_VHX, SPHV_VHY, SPHV_VHZ,
    SPHV_AX, SPHV_AY, SPHV_AZ, SPHV_M, SPHV_H, SPHV_RHO, SPHV_OMEGA, SPHV_U, SPHV_UH,
    SPHV_UDT, SPHV_ALPHA, SPHV_VSIG, SPHV_WCOUNT,
    SPHV_NROLES
};

/* One struct member: byte offset inside a record, its dtype, whether the loop
 * reads and/or writes it, and its SPH role. */
typedef struct {
    uint64_t offset;
    uint32_t role;
    uint16_t dtype;
    uint16_t access;
} sphv_field;

/* The records and the members a loop touches.  Record i's member f lives at
 * base + i*stride + fields[f].offset.  Two storage shapes are accepted:
 *  - array of structs: every member lies inside the stride (offset+size <= stride);
 *  - struct of arrays: stride equals the member size and members are whole
 *    arrays of n elements that do not overlap (offset >= previous + n*size).
 * Members must be naturally aligned and must not overlap; a role may appear
 * at most once.
 *
 * flags = SPHV_DESC_RECORD_POINTERS: the records are scattered, reached through
 * a list of their addresses (paper Sec. 5.1: the particles of a cell held as a
 * list of pointers, and generic kernels over such lists).  The aos_dev of every
 * call taking this descriptor is then the device address of an array of n
 * uint64_t record addresses, record i's member f living at ptrs[i] +
 * fields[f].offset (array-of-structs shape, stride the record size, each
 * record aligned to 8 bytes).  cells_build, views of kind SOA, AOSOA and DIRECT
 * (gather, loops, step reduction, scatter) and kick_drift accept it; views of
 * kind SORTED, sphv_autotune and sphv_autotune_grid fail with
 * SPHV_E_UNSUPPORTED (to move such records into cell order, permute the
 * address list instead; sphv_records_sort moves contiguous records only).
 * The address list itself is checked like records (device-addressable); the
 * records it names are the caller's: each must be device-addressable and they
 * must not overlap.  The alias rule of open views compares address lists:
 * views through different lists are taken to name different records. */
enum { SPHV_DESC_RECORD_POINTERS = 1u };
typedef struct {
    uint64_t stride;
    uint32_t n_fields;
    uint32_t flags;     /* 0, or SPHV_DESC_RECORD_POINTERS */
    const sphv_field* fields;
} sphv_descriptor;

/* ---------------------------------------------------------------- params */

/* Box, grid and physics constants.  cell[d] = len[d]/grid[d] and
 * inv_cell[d] = grid[d]/len[d] are filled by sphv_params_init and used as given
 * (the binning formula below depends on their exact values). */
typedef struct {
    double lo[3];
    double len[3];
    double cell[3];
    double inv_cell[3];
    int32_t grid[3];
    int32_t periodic[3];
    double gamma;      /* adiabatic index (5/3)                                  */
    double eta;        /* density target rho h^3 = m eta^3                        */
    double cfl;        /* Courant factor of dt = cfl min h / v_sig                */
    double h_tol;      /* Newton stop |h+ - h| <= h_tol h                         */
    double headroom;   /* cell reach: R = ceil(2 h headroom / min cell), >= 1     */
    int32_t max_iter;  /* density passes, 1..64                                   */
    int32_t kernel;    /* smoothing kernel, SPHV_KERNEL_CUBIC or SPHV_KERNEL_QUARTIC */
    int32_t list_cap;  /* 0: the pair loops walk cell windows per work item; 1..4096: */
                       /* they walk per-particle neighbour lists of at most list_cap */
                       /* entries (the cells workspace holds them; see below)       */
    int32_t symmetric; /* 1 (with list_cap > 0, FP64): the force loop evaluates each */
                       /* pair once (Newton's third law), see below; 0: twice        */
} sphv_params;

/* Smoothing kernels W(r, h) = w(q) / (pi h^3), q = r/h, both with support
 * r < 2h, so cells, reach and the pair predicate do not depend on the choice:
 *  - SPHV_KERNEL_CUBIC: the cubic M4 spline (Monaghan & Lattanzio),
 *    w = (2-q)_+^3 / 4 - (1-q)_+^3;
 *  - SPHV_KERNEL_QUARTIC: the quartic M5 spline the paper employs (Sec. 2.1,
 *    after Monaghan 1985), its knots 0.5, 1.5, 2.5 of s = 1.25 q placed at
 *    q = 0.4, 1.2, 2: w = (15625/65536) ((2-q)_+^4 - 5 (1.2-q)_+^4 + 10 (0.4-q)_+^4).
 * Any other value is rejected with SPHV_E_INVALID_ARG by every call that
 * takes parameters. */
enum { SPHV_KERNEL_CUBIC = 0, SPHV_KERNEL_QUARTIC = 1 };

/* Neighbour lists (list_cap > 0; the active set of each particle made explicit,
 * paper Sec. 2.3).  One lane per particle.  The density loop first lists, in
 * its window's order, every candidate within 2 h_l, h_l = min(h_cap,
 * (1 + 1/16) h) at the h it starts from, then runs every Newton pass over
 * that list; a particle whose h leaves h_l, or whose list would exceed
 * list_cap, runs its remaining passes over the whole window instead (same
 * candidates, same order).  The force loop lists exactly its pairs
 * (r < 2 max(h_i, h_j) at the converged h) and evaluates them; a particle
 * with more than list_cap pairs evaluates them from the window.  The layout's
 * tpi and masked do not apply to list walks (every list entry is evaluated,
 * out-of-range density entries as the neutral element).  The lists need
 * list_cap * n * 4 bytes of the cells workspace.
 * Symmetric pairs (symmetric = 1; paper Sec. 5.3, F(p1, p2) = -F(p2, p1)): the
 * force lists hold each particle's pairs in ascending sorted position; a first
 * pass evaluates each pair (i, j), i < j, once, adds i's side to i and stores
 * j's side (its acceleration and du/dt terms and the pair's v_sig) in j's slot
 * for i, found by bisection in j's list; a second pass adds, per particle, the
 * stored sides of its partners below it in list order, after the sum over
 * those above it.  Every sum has a fixed order, so results are deterministic;
 * they differ from the twice-evaluated form in rounding only.  The slots take
 * 40 * list_cap * n bytes of the cells workspace.  Should any list overflow,
 * the second pass evaluates every particle's pairs twice from its window.
 * FP32 views fail with SPHV_E_UNSUPPORTED.
 * Defaults: gamma 5/3, eta 1.2, cfl 0.3, h_tol 1e-13, headroom 1.1, max_iter 16,
 * kernel SPHV_KERNEL_CUBIC, list_cap 0, symmetric 0. */
int32_t sphv_params_init(sphv_params* p, const double lo[3], const double len[3],
                         const int32_t grid[3], const int32_t periodic[3]);

/* ----------------------------------------------------------- state block */

/* Host mirror of the device state block (sphv_state_bytes() bytes, caller-owned
 * device memory): what a step of the time-stepping scheme of paper Sec. 2.1
 * carries from one step to the next (the time step size, the step count) and
 * what it reports (error flags, conservation sums, pair counts; the paper
 * states no error model, and reporting errors asynchronously in this block is
 * this library's choice).  dt is written by sphv_step_reduce (dt_prev keeps the one
 * before, nstep counts its calls); sums are fixed-order FP64 totals over particles:
 *   [0..2] sum m v, [3] sum m (|v|^2/2 + u), [4..6] sum m a, [7] sum m (v.a + du/dt)
 * pairs_* count ordered pairs (i, j != i) inside the support at the accepted h
 * (density: r < 2 h_i; force: r < 2 max(h_i, h_j)); pair_evals_density counts
 * such pairs over every density pass that was executed; pairs_total keeps
 * adding pairs_density and pairs_force over all steps (not reset per step). */
typedef struct {
    uint32_t flags;
    int32_t max_iters;
    int64_t nstep;
    double dt;
    double dt_prev;
    double t;
    double sums[8];
    int64_t pairs_density;
    int64_t pairs_force;
    int64_t pair_evals_density;
    int64_t pairs_total;     /* density + force pairs since sphv_state_init */
    int64_t reserved[3];
} sphv_state;

size_t sphv_state_bytes(void);
/* Zero the whole block (flags, dt history, counters) with a fill kernel. */
int32_t sphv_state_init(void* state_dev, void* stream);
/* Zero the per-step pair counters only (a fill kernel; graph-capturable). */
int32_t sphv_begin_step(void* state_dev, void* stream);
/* Copy the block to the host; synchronises the stream. */
int32_t sphv_read_state(const void* state_dev, sphv_state* out, void* stream);
/* Copy a host block to the device; synchronises the stream. */
int32_t sphv_write_state(void* state_dev, const sphv_state* in, void* stream);

/* ----------------------------------------------------------------- cells */

/* Uniform linked-cell grid (paper Sec. 2.1: particles sorted into cells so that
 * only neighbouring cells interact; Sec. 5.2: particles of a cell as one chunk
 * with CSR-like chunk offsets).
 *   key_i = (kz ny + ky) nx + kx,  k_d = clamp(floor((x_d - lo_d) * inv_cell_d), 0, n_d - 1)
 *   perm  = stable sort of i by key (ties keep index order): sorted position -> record
 *   cell_start[c] .. cell_start[c+1] = the sorted positions of cell c.
 * A cell's reach R (cells per axis) covers 2 h headroom of its largest h; the
 * density loop of a particle in cell c visits the (2R+1)^3 cells around c and
 * its h is capped at R * min(cell) / 2.  The force loop (sphv_sph_force) sets
 * its own window from the converged h: R_f(c) is the largest of ceil(2 h_max(c)
 * / min cell) and the Chebyshev distance of every cell whose own such reach
 * covers c, h_max(c) being the largest h of c seen by the force calls since
 * the last sphv_cells_build (so repeated force calls never narrow a window).
 * That exact window is computed when every own reach is at most 4; otherwise
 * the window is the cover G(c), the largest own reach among the cells whose
 * own reach covers c (at least the exact window, and G(c) min cell bounds 2h
 * of every force partner of c's particles).
 * Work items are (cell, first sorted position, count<=64). */
typedef struct sphv_cells sphv_cells;

typedef struct {
    const int32_t* perm;        /* [n]          sorted position -> record index   */
    const int32_t* cell_start;  /* [n_cells+1]                                     */
    const int32_t* key;         /* [n]          key of record i (unsorted order)   */
    const int32_t* reach;       /* [3*n_cells]  density reach, then the force window and the cover G
                                   (both set by sph_force) */
    int64_t n;
    int64_t n_cells;
    int64_t max_items;
} sphv_cells_info;

/* The cells workspace also holds the force loops' per-particle constants
 * (A = P/(Omega rho^2), c, 1/h, 1/(pi h^4), (2h)^2; 40 bytes per particle),
 * which sphv_sph_force computes once per particle before its pairs, and with
 * list_cap > 0 the neighbour lists. */
size_t sphv_cells_workspace_bytes(int64_t n, const sphv_params* p);
int32_t sphv_cells_create(sphv_cells** out, int64_t n, const sphv_params* p,
                          void* ws_dev, size_t ws_bytes);
/* Bin, sort, offsets, per-cell reach and work items from the records' x, y, z, h
 * (roles SPHV_X, SPHV_Y, SPHV_Z, SPHV_H of d; any access).  state_dev gets flags. */
int32_t sphv_cells_build(sphv_cells* c, const void* aos_dev, const sphv_descriptor* d,
                         void* state_dev, void* stream);
int32_t sphv_cells_get_info(const sphv_cells* c, sphv_cells_info* out);
void sphv_cells_destroy(sphv_cells* c);

/* Records stored cell by cell (paper Sec. 2.2 and Sec. 5.2: the particle sort
 * may move the records after each drift so that the particles of one cell form
 * one contiguous chunk of memory).  After sphv_cells_build on c, moves the
 * whole records (stride bytes each, every member, cold ones included) so that
 * record p becomes the record that was at perm[p]; then c's perm is the
 * identity and its key follows the records, so c stays valid for those
 * records until the next sphv_cells_build.  Stable: particles of one cell keep
 * their order, so a following cells_build gives the same cells and loops sum
 * in the same order.  Only views of kind SPHV_LAYOUT_SORTED require it.
 *   aos_dev  the n records c was built from; base aligned to 4 bytes.
 *   stride   record bytes, a multiple of 4.
 *   ws_dev   device scratch of sphv_records_sort_workspace_bytes(stride, n)
 *            bytes, 256-B aligned; its contents are not kept.
 * Two kernels on stream (graph-capturable).  Errors: SPHV_E_INVALID_ARG (NULL
 * handle, stride or alignment), SPHV_E_WORKSPACE, SPHV_E_STATE (c not built). */
size_t sphv_records_sort_workspace_bytes(uint32_t stride, int64_t n);
int32_t sphv_records_sort(sphv_cells* c, void* aos_dev, uint32_t stride, void* ws_dev, size_t ws_bytes,
                          void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation as sphv_records_sort, with the same kernels and results, but the
 * sorted copy goes to a fixed device array of SPHV_RECORDS_SORT_STATIC_MAX_BYTES
 * bytes that the library holds on each GPU it runs on until the process ends,
 * instead of a caller workspace.  The call allocates nothing.
 *   stride * n (n = the records c was built for) must not exceed the maximum,
 *   else SPHV_E_WORKSPACE before anything is enqueued.
 * Every call on one GPU shares that GPU's array, and the array keeps the last
 * call's contents (every byte a call reads it wrote first): calls that overlap
 * on one GPU (two streams, or two host threads) race and corrupt each other's
 * records; order them on one stream.  The array's device address is looked up
 * on the first call on each device (SPHV_E_HIP if that fails).  Other errors
 * as sphv_records_sort. */
#define SPHV_RECORDS_SORT_STATIC_MAX_BYTES (96ull << 20)
int32_t sphv_records_sort_static(sphv_cells* c, void* aos_dev, uint32_t stride, void* stream);

/* ----------------------------------------------------------------- views */

enum {
    SPHV_LAYOUT_SOA = 0,     /* one array per member (Sec. 2.4, Listing 2)           */
    SPHV_LAYOUT_AOSOA = 1,   /* blocks of aosoa_width particles, SoA inside a block  */
    SPHV_LAYOUT_DIRECT = 2,  /* no conversion: loops read and write the records      */
                             /* through the index (the paper's unconverted kernels)  */
    SPHV_LAYOUT_SORTED = 3   /* no conversion, records stored cell by cell          */
                             /* (sphv_records_sort): element p is record p          */
};
enum { SPHV_PREC_FP64 = 0, SPHV_PREC_FP32 = 1 };

/* Layout and tile shape of one view and of the pair loops run over it.
 * tpi: lanes that share one local particle (1..64, 0 = automatic: 64 / count
 * of the work item).  masked: 1 evaluates every candidate pair and multiplies
 * out-of-range terms by zero (Sec. 5.6, neutral elements), 0 branches.  Both
 * give bit-identical results; tpi changes the summation order.  Either form of
 * the density loop caches, per work item, which candidates lie within twice
 * its cell cap; a branching force loop with the same tpi and precision reuses
 * them instead of testing every candidate again. */
typedef struct {
    uint32_t kind;
    uint32_t aosoa_width;   /* power of two, 1..1024, for SPHV_LAYOUT_AOSOA (1: each */
                            /* particle's view members packed together)          */
    uint32_t tpi;
    uint32_t masked;
} sphv_layout;

/* Precision of the view (SPHV_PREC_*):
 *  FP64: every member is a bit copy of the record's member.
 *  FP32: members read only (A_in \ A_out) of dtype f64 are stored as float:
 *        positions relative to the lower corner of their cell,
 *        float(x - (lo + k * cell)), other members float(v), both rounded to
 *        nearest even; members written (A_out) stay f64.  The pair loops then
 *        run in FP32 with compensated FP32 sums; the h iteration's Newton step
 *        and convergence test stay FP64. */
typedef struct sphv_view sphv_view;

size_t sphv_view_workspace_bytes(const sphv_descriptor* d, int64_t n, const sphv_layout* l,
                                 int32_t precision);
/* Plan a view of n records of aos_dev described by d.  index_dev (device int32[n],
 * or NULL for 0..n-1) is the loop's container: view element p is record
 * index_dev[p] (paper Sec. 2.3, the local/active particle lists).  The SPH loops
 * need the view indexed by the cells' perm.  Host-only: validates and plans the
 * workspace; enqueues nothing. */
int32_t sphv_view_create(sphv_view** out, const sphv_descriptor* d, int64_t n,
                         const sphv_layout* l, int32_t precision, void* aos_dev,
                         const int32_t* index_dev, void* ws_dev, size_t ws_bytes);
/* Gather A_in (the prologue).  Opens the view: until sphv_soa_to_aos the
 * records' members in A_in u A_out are temporarily invalid (Sec. 3.2); other
 * members stay valid and are never touched.  A_out \ A_in is not initialised
 * (Sec. 3.1).  cells is required for FP32 views (cell of each element) and may
 * be NULL otherwise.  Fails with SPHV_E_ALIAS if another open view on
 * overlapping records writes a member this one touches, or touches a member
 * this one writes; views of kind SPHV_LAYOUT_DIRECT and SPHV_LAYOUT_SORTED
 * (which copy nothing but write the records' members in place) open and
 * take part in this rule like the others. */
int32_t sphv_aos_to_soa(sphv_view* v, const sphv_cells* cells, void* stream);
/* Prefetch: gathers ahead the members of A_in that the view only reads and
 * that no open (or prefetched) view on the same records writes, so that the
 * copy can overlap other work, e.g. the force view's positions, velocities,
 * masses, u and alpha on a second stream while the density loop runs (the
 * paper's Sec. 7.5 on overlapping transfers with kernels; with records in
 * pinned host memory this hides their transfer).  The view is then registered
 * as a reader of those members: a view that writes one of them fails to open
 * with SPHV_E_ALIAS, and the caller must not change them in the records before
 * the view closes.  sphv_aos_to_soa later gathers the remaining members and
 * opens the view; only the prefetched members' bits are taken at prefetch
 * time.  A view on the records themselves copies nothing (SPHV_OK, no
 * effect); so does a view none of whose members qualify.  SPHV_E_STATE if the
 * view is open or prefetched already, or cells are missing for an FP32 view.
 * Ordering between the two streams is the caller's: the prefetch must follow
 * cells_build (the view's index), and the loop must follow the prefetch. */
int32_t sphv_aos_to_soa_prefetch(sphv_view* v, const sphv_cells* cells, void* stream);
/* Scatter A_out only (the epilogue) and close the view. */
int32_t sphv_soa_to_aos(sphv_view* v, void* stream);
/* Device address, dtype and element stride (bytes between consecutive elements
 * inside one block; blocks are block_bytes apart, block_len elements each) of
 * field k of an SoA/AoSoA view, for inspection. */
int32_t sphv_view_field(const sphv_view* v, uint32_t k, void** dev_ptr, int32_t* dtype,
                        uint64_t* block_len, uint64_t* block_bytes);
void sphv_view_destroy(sphv_view* v);

/* Density loop (paper Sec. 2.1 step 1) over an open view indexed by the cells'
 * perm.  View members: IN x, y, z, m; INOUT h; OUT rho, omega, wcount.
 * For each particle i, at its current h, over j in its cells' window:
 *   rho_i = sum_j m_j W(r_ij, h), drho_i/dh = sum_j m_j dW/dh, n_i = sum_j W
 * (j = i included), W the kernel p->kernel selects (support 2h); then a Newton step
 * on rho_i(h) h^3 = m_i eta^3, h+ = h - f/f', f' = drho/dh + 3 m eta^3/h^4,
 * clamped to [h/2, 2h] and to the cell cap (fixed point eta (m/rho)^(1/3) if
 * f' <= 0).  The current h is accepted when |h+ - h| <= h_tol h, else h = h+
 * and the sums are redone, at most max_iter times.  Outputs at the accepted h:
 * rho, omega = 1 + h/(3 rho) drho/dh, wcount = (4 pi/3)(2h)^3 n. */
int32_t sphv_sph_density(sphv_view* v, const sphv_cells* c, const sphv_params* p,
                         void* state_dev, void* stream);
/* Force loop (paper Sec. 2.1 step 2) over an open view indexed by the cells'
 * perm.  View members: IN x, y, z, vx, vy, vz, m, h, rho, omega, u, alpha;
 * OUT ax, ay, az, u_dt, v_sig.  Pairs j != i with r < 2 max(h_i, h_j):
 *   P = (gamma-1) rho u, c = sqrt(gamma (gamma-1) u), A = P/(omega rho^2),
 *   g = dW/dr(r, h) per side, gbar = (g_i + g_j)/2, w = v_ij . r_hat,
 *   mu = min(w, 0), v_sig,ij = c_i + c_j - 3 mu,
 *   Pi = -(alpha_i + alpha_j)/4 v_sig,ij mu / ((rho_i + rho_j)/2),
 *   a_i  -= m_j (A_i g_i + A_j g_j + Pi gbar) r_hat
 *   u_dt += m_j (A_i g_i + Pi gbar / 2) w,   v_sig,i = max(2 c_i, max_j v_sig,ij).
 * One view may serve both loops (the union of their members, h, rho and omega
 * INOUT): the force loop then reads the density's results inside the view,
 * and its windows take h from the view.  FP32 views must hold the twelve IN
 * members as members the view only reads (stored as floats); a view that
 * also writes one of them fails with SPHV_E_DESCRIPTOR (likewise x, y, z, m
 * for the density loop). */
int32_t sphv_sph_force(sphv_view* v, const sphv_cells* c, const sphv_params* p,
                       void* state_dev, void* stream);
/* Time-step reduction over an open force view after sphv_sph_force: in one
 * fixed-order FP64 tree (deterministic), dt = cfl min_i h_i / v_sig,i (the
 * division rounded per particle) and the conservation sums of sphv_state.
 * Updates the state block: t += old dt, dt_prev = old dt, dt = new dt,
 * nstep += 1.  Outputs are read from where the loop wrote them.  Inputs m,
 * v, u, h are read from an FP64 view, which holds them as exact copies (or
 * holds the density's h, in one view over both loops).  Otherwise they come
 * from the records: members a view only reads are never modified while it
 * is open, and an FP32 view holds them as floats.  The sums do not depend on
 * the source.  The force loop's windows take h from the same place. */
int32_t sphv_step_reduce(sphv_view* v, const sphv_params* p, void* state_dev, void* stream);

/* Kick / drift / kick with prediction (paper Sec. 2.1 steps 3-5) on the records
 * directly (linear loop, no view), every product and sum rounded on its own:
 *   if nstep > 1: v = vh + a (dt_prev/2), u = uh + u_dt (dt_prev/2)   (close step)
 *   vh = v + a (dt/2), uh = u + u_dt (dt/2)                           (open step)
 *   x = x + vh dt, wrapped once into [lo, lo+len) on periodic axes     (drift;
 *       a drift over more than one box length stays outside and the next
 *       sphv_cells_build sets SPHV_F_OUT_OF_BOX)
 *   v = vh + a (dt/2), u = uh + u_dt (dt/2)                           (predict)
 * dt, dt_prev and nstep are read from the device state block.  Members: x, y, z,
 * vx, vy, vz, vhx, vhy, vhz, ax, ay, az, u, uh, u_dt. */
int32_t sphv_kick_drift(void* aos_dev, const sphv_descriptor* d, int64_t n,
                        const sphv_params* p, const void* state_dev, void* stream);

/* ------------------------------------------------------------- autotuner */

/* Per-loop choice of layout and tile shape (the batching layer's tuner: which
 * layout pays differs per kernel in the paper's measurements, Sec. 7, Table 2
 * and Sec. 7.5).
 * A candidate is an sphv_layout; one trial times, with HIP events on stream,
 * the gather of A_in, the loop and the scatter of A_out of a view with that
 * layout, over the records aos_dev (described by d, indexed by the cells'
 * perm), starting from the records as they are.  Each candidate runs reps
 * trials, in reps rounds over all candidates; its figure is their median.  Medians within 1.5 % of the smallest
 * count as equal (timing noise): *best is the first such candidate in the
 * given order, so repeated tuning settles on one choice.  The medians, in
 * candidate order, go to ms (NULL: not reported).
 *
 * candidates: NULL for the built-in set (sphv_autotune_candidates), else an
 *   array of n_candidates (1..128) layouts.
 * Records: every member d names is copied out bit for bit before the first
 *   trial and copied back after each trial and at the end, so the records
 *   leave the call as they came in.  Run it on records that hold a valid
 *   state for the loop (for the force loop: after a density scatter).
 * Coupling: the force loop reuses the candidate masks the density loop cached
 *   in the cells when both ran unmasked with the same tpi.  Force trials read
 *   the cache as the caller's last density call left it (density trials
 *   overwrite it with their last unmasked candidate's), so tune the density
 *   loop first, run it once with the chosen layout, then tune the force loop.
 * SPHV_LAYOUT_SORTED candidates: the trial starts with sphv_records_sort (its
 *   time counts, as the layout needs it) and afterwards moves the records,
 *   the cells' perm and key back to where they were, so cells (const for the
 *   caller) is modified during the call and restored before it returns.
 * ws_dev: device workspace of sphv_autotune_workspace_bytes(...) bytes, 256-B
 *   aligned (state block, bit copy of the members, the largest candidate view,
 *   and with sorted candidates a copy of the records and of perm and key).
 * The call synchronises stream (it times on the host) and fails with
 * SPHV_E_STATE while stream is being captured into a graph, SPHV_E_ALIAS if an
 * open view on the same records conflicts with a trial view, SPHV_E_WORKSPACE
 * for a small or misaligned workspace.  Every kernel exits normally on every
 * candidate; flags of the trials go to the private state block, not the
 * caller's.  Cells are left built; the density mask cache keeps the last
 * trial's contents, which the next density call rewrites. */
enum { SPHV_LOOP_DENSITY = 0, SPHV_LOOP_FORCE = 1 };

/* Writes up to cap built-in candidates to out (NULL: none), returns their count. */
int32_t sphv_autotune_candidates(sphv_layout* out, int32_t cap);
/* 0 on invalid arguments. */
size_t sphv_autotune_workspace_bytes(const sphv_descriptor* d, int64_t n, int32_t precision,
                                     const sphv_layout* candidates, int32_t n_candidates);
int32_t sphv_autotune(int32_t loop, void* aos_dev, const sphv_descriptor* d, const sphv_cells* cells,
                      const sphv_params* p, int32_t precision, const sphv_layout* candidates,
                      int32_t n_candidates, int32_t reps, void* ws_dev, size_t ws_bytes,
                      sphv_layout* best, float* ms, void* stream);

/* Cells per support length, the tuner's grid axis (the mesh of Sec. 2.1 sized
 * for the largest smoothing length h_ref): along each axis
 *   grid[a] = max(floor(len[a] k / (2 h_ref 1.1)), 3 if periodic else 1),
 * i.e. k cells of edge >= 2 h_ref 1.1 / k span one support.  k = 1 gives the
 * plain 27-cell stencil for particles with h <= h_ref; larger k give smaller
 * cells and wider (per-cell) windows.  k in 1..4; SPHV_E_UNSUPPORTED beyond
 * 4096 cells on an axis. */
int32_t sphv_grid_for(const sphv_params* p, double h_ref, int32_t cells_per_support, int32_t* grid);

/* Picks the grid for the density + force pair.  For each candidate grid
 * (grids[3g..3g+2], n_grids in 1..16) it times, on stream with HIP events,
 * reps trials of: cells_build on that grid, then the density view (gather,
 * loop, scatter) and the force view (gather, loop, scatter) with layouts
 * l_density and l_force (not SPHV_LAYOUT_SORTED: SPHV_E_UNSUPPORTED).  The
 * members of d_density and d_force are restored bit for bit after each trial,
 * as in sphv_autotune; cells_build takes x, y, z, h from d_density.  *best is
 * the index of the first grid whose median is within 1.5 % of the smallest,
 * ms the medians (NULL: not reported).  The caller then builds its own cells with that grid.  Host
 * timing: synchronises stream, SPHV_E_STATE under graph capture. */
size_t sphv_autotune_grid_workspace_bytes(const sphv_descriptor* d_density, const sphv_descriptor* d_force,
                                          int64_t n, const sphv_params* p, int32_t precision,
                                          const sphv_layout* l_density, const sphv_layout* l_force,
                                          const int32_t* grids, int32_t n_grids);
int32_t sphv_autotune_grid(void* aos_dev, const sphv_descriptor* d_density, const sphv_descriptor* d_force,
                           int64_t n, const sphv_params* p, int32_t precision, const sphv_layout* l_density,
                           const sphv_layout* l_force, const int32_t* grids, int32_t n_grids, int32_t reps,
                           void* ws_dev, size_t ws_bytes, int32_t* best, float* ms, void* stream);

/* ---------------------------------------------------------------- graphs */

/* Capture everything enqueued on stream between begin and end into a HIP graph
 * (thread-local capture mode); launch replays it on any stream.  A whole step
 * becomes one launch: the answer here to the many small kernels whose launch
 * overhead the paper's GPU measurements single out (Sec. 7.5).  Arguments: the
 * stream (a hipStream_t, null for the default stream); out receives a handle the
 * caller releases with sphv_graph_destroy.  Errors: SPHV_E_HIP when capture or
 * instantiation fails, SPHV_E_INVALID_ARG for a null handle. */
typedef struct sphv_graph sphv_graph;
int32_t sphv_graph_begin(void* stream);
int32_t sphv_graph_end(void* stream, sphv_graph** out);
int32_t sphv_graph_launch(sphv_graph* g, void* stream);
void sphv_graph_destroy(sphv_graph* g);

#ifdef __cplusplus
}
#endif
#endif /* SPHVIEW_H */
