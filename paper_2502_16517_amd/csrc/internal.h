// Internal declarations shared by the host ABI layer and the HIP kernels of
// libsphview.so.  Not installed; the public contract is include/sphview.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sphview.h"

namespace sphv {

constexpr int kMaxFields = 32;
constexpr int kWave = 64;
constexpr int kNumXcd = 8;       // MI355X: 8 accelerator complex dies, one L2 each
constexpr int kRedBlock = 256;   // particles per block of the fixed-order reductions
constexpr int kMaskChunks = 12;  // candidate chunks per work item whose hit masks are cached
constexpr int kQStride = 1024;   // ints between two queue heads: one 4 KiB page each, so that their
                                 // atomics do not queue up at one memory channel
constexpr int kMaxPairBlocks = 256 * 20;   // largest grid of a pair loop
constexpr int kPartSlots = 4;    // per-wave counters a pair loop leaves for its fold
constexpr int kDense = 64;       // cells of more particles are ordered by sub-cell inside
constexpr int kSubBits = 4;      // sub-cells per cell edge: 2^kSubBits
constexpr int kBlock = 16;       // sorted positions per bounding block of the list walks (divides 64)
constexpr int kBlockWords = 8;   // per block: lo x y z, hi x y z, largest 2h, spare

// Device state block (mirrors sphv_state field for field).
struct DevState {
    uint32_t flags;
    int32_t max_iters;
    int64_t nstep;
    double dt;
    double dt_prev;
    double t;
    double sums[8];
    unsigned long long pairs_density;
    unsigned long long pairs_force;
    unsigned long long pair_evals_density;
    unsigned long long pairs_total;
    int64_t reserved[3];
};
static_assert(sizeof(DevState) == sizeof(sphv_state), "state mirror");

// Where element p of one field lives.
//  view (SoA / AoSoA): base + off + (p >> lw) * block_bytes + (p & mask) * size
//  direct (records):   base + off + index[p] * stride
struct FieldRef {
    char* base;
    uint64_t off;
    uint32_t size;     // bytes of one element
    uint32_t dtype;    // storage dtype (SPHV_F64 / F32 / I64 / I32)
    int32_t rel_axis;  // >= 0: FP32 cell-relative coordinate along this axis
    int32_t pad;
};

struct Access {
    uint32_t lw;          // log2 block length (view); 63 for plain SoA
    uint32_t pad;
    uint64_t mask;        // block length - 1 (view); all ones for plain SoA
    uint64_t block_bytes; // view
    const int32_t* index; // direct
    uint64_t stride;      // direct
    const uint64_t* ptrs; // direct, records by address: record r at ptrs[r] (the members' base is null)
};

// Grid geometry passed to kernels.
struct Geom {
    double lo[3], len[3], cell[3], inv_cell[3];
    int32_t n[3], periodic[3];
    double cmin;      // min cell edge
    double headroom;
};

struct CellsDev {
    int32_t* key;          // [n] key of record i
    int32_t* sub;          // [n] sub-cell code of record i (Morton index of its 16^3 sub-cell)
    int32_t* perm;         // [n]
    int32_t* perm_tmp;     // [n] cell-grouped, not yet ordered within a cell
    int32_t* key_sorted;   // [n] cell of sorted position p
    int32_t* cell_start;   // [nc + 1]
    int32_t* counts;       // [nc]
    int32_t* cursor;       // [nc]
    uint32_t* hmax_bits;   // [nc] float bits of the largest 2 h (times the headroom for the density reach)
    uint32_t* hmax_f;      // [nc] float bits of the largest 2 h the force loops saw since cells_build
                           // (directly after hmax_bits: one clear covers both)
    int32_t* reach_d;      // [nc] density reach (cells_build, from h before the density loop)
    int32_t* reach_f;      // [nc] force window radius (sph_force, from the converged h)
    int32_t* reach_s;      // [nc] cover of the own force reach: the largest own reach among the cells
                           // whose reach covers this one (bounds 2h / cmin of every force partner)
    uint64_t* cover;       // [2][nc] masks of the cover's axis passes
    int32_t* tmp_a;        // [nc] scratch for the reach filter / item counts
    int32_t* tmp_b;        // [nc]
    int32_t* item_start;   // [nc + 1]
    int4* items;           // [max_items]  (cell, first sorted pos, count, 0)
    uint64_t* item_masks;  // [max_items][kMaskChunks][64] candidate hit masks of the density loop
    int64_t* pair_part;    // [kMaxPairBlocks][kPartSlots] per-wave counters of the last pair loop
    int32_t* scan_part;    // [scan blocks + 1]
    int32_t* meta;         // [META_SIZE]: item count, mask tag, force R_global, queue heads
    int32_t* list;         // [list_cap][n] neighbour lists (list walks only, else null)
    double* fconst;        // [5][n] per-particle force constants (of the pair precision)
    double* blocks;        // [n / 64 + 1][kBlockWords] bounds of each run of 64 sorted positions (list walks)
    int32_t* list_len;     // [n] entries of each particle's list (list walks)
    double* slots;         // [5][list_cap][n] symmetric force: the stored j sides (else null)
    int32_t list_cap;
    int32_t pad_l;
    int64_t n;
    int64_t nc;
    int64_t max_items;
};

// meta[] slots
enum {
    META_NITEMS = 0,
    META_MASKS = 2,                          // 0: no cached masks; else 1 + lanes-per-particle setting (+128 for FP32)
    META_RGLOBAL_F = 3,                      // largest own force reach
    META_SCAN = 4,                           // block tickets of the scans of cells_build (two slots)
    META_LIST_OVF = 6,                       // list walks: some particle left its list (see k_list.hip)
    META_QHEAD_D = kQStride,                       // 8 per-XCD heads of the density queue, kQStride apart
    META_QHEAD_F = kQStride + kNumXcd * kQStride,  // the same for the force queue
    META_SIZE = kQStride + 2 * kNumXcd * kQStride
};

// Arguments of the pair kernels.
struct PairArgs {
    FieldRef f[SPHV_NROLES];   // by role (only the loop's roles are filled)
    Access acc;
    Geom g;
    const int4* items;
    const int32_t* cell_start;
    const int32_t* reach;      // density or force reach
    const int32_t* key_sorted; // cell of sorted position p
    const int32_t* reach_d;    // density reach (the force loop compares it with its own)
    const int32_t* reach_s;    // force: cover of the own force reach (largest own reach covering the cell)
    uint64_t* item_masks;      // cached candidate masks (see CellsDev)
    int32_t* meta;             // queue counters
    int64_t* part;             // per-wave counters, folded by the launch that follows
    int32_t qhead, pad2;       // meta slot of this kernel's first queue head
    DevState* state;
    double eta, tol, gamma;
    int32_t max_iter;
    int32_t tpi;               // 0 = automatic
    int32_t nblocks;           // grid size (<= kMaxPairBlocks: one counter slot per wave)
    int32_t pad;
    double* red_part;          // force: per reduction block partials
    int64_t n;
    double cfl;
    int32_t* list;             // list walks: entry k of sorted position p at list[k n + p]
    void* fconst;              // force: per-particle constants (R[5][n], R the pair precision)
    const double* blocks;      // list walks: bounds of each run of kBlock sorted positions, or null
    const uint32_t* cell_h;    // force list walk: float bits of each cell's largest 2h (rounded up)
    int32_t* list_len;         // list walks: entries of each list
    double* slots;             // symmetric force: stored j sides, slot (k, e, j) at k cap n + e n + j
    int32_t list_cap;
    int32_t pad3;
};

}  // namespace sphv

// launchers (defined in the .hip files), return hipError_t
namespace sphv {
hipError_t launch_fill_u32(void* p, uint32_t v, int64_t count, hipStream_t s);
hipError_t launch_state_init(DevState* st, int full, hipStream_t s);
hipError_t launch_cells_build(const CellsDev& c, const FieldRef* xyzh, const Access& rec,
                              const Geom& g, DevState* st, hipStream_t s);
// h from the records (through perm, stride bytes apart), or from a view (view_acc
// not null: element p of the view is sorted position p)
hipError_t launch_force_reach(const CellsDev& c, const FieldRef& h, uint64_t stride, const Access* view_acc,
                              const Geom& g, DevState* st, hipStream_t s, const uint64_t* rec_ptrs = nullptr);
hipError_t launch_gather(const FieldRef* src, const FieldRef* dst, int nf, const Access& src_acc,
                         const Access& dst_acc, const int32_t* cell_key, const Geom& g, int64_t n,
                         hipStream_t s);
hipError_t launch_scatter(const FieldRef* src, const FieldRef* dst, int nf, const Access& src_acc,
                          const Access& dst_acc, int64_t n, hipStream_t s);
hipError_t launch_density(const PairArgs& a, int direct, int fp32, int masked, int kernel, hipStream_t s);
hipError_t launch_force(const PairArgs& a, int direct, int fp32, int masked, int kernel, hipStream_t s);
// the list walks (k_list.hip); each ends with the fold of its counters
hipError_t launch_density_list(const PairArgs& a, int direct, int fp32, int kernel, hipStream_t s);
hipError_t launch_force_list(const PairArgs& a, int direct, int fp32, int kernel, hipStream_t s);
// the symmetric force (FP64 list walks): lists, one evaluation per pair, the stored sides
hipError_t launch_force_sym(const PairArgs& a, int direct, int kernel, hipStream_t s);
// per-particle constants of both force loops (k_list.hip), into a.fconst
hipError_t launch_force_prep(const PairArgs& a, int direct, int fp32, hipStream_t s);
// bounds of each run of kBlock sorted positions into blocks (k_list.hip)
hipError_t launch_block_bounds(const PairArgs& a, double* blocks, int direct, int fp32, hipStream_t s);
hipError_t launch_pair_fold(const PairArgs& a, int nblocks, int density, hipStream_t s);
// in_view: in6 are members of the view (read with outacc) instead of the records
hipError_t launch_force_reduce(const FieldRef* in6, const Access& rec, const FieldRef* out5,
                               const Access& outacc, int out_direct, int in_view, DevState* st,
                               double cfl, int64_t n, double* partials, hipStream_t s);
// whole records: dst[didx ? didx[p] : p] = src[sidx ? sidx[p] : p], stride bytes
// each (stride and both bases multiples of 4 bytes)
hipError_t launch_rec_move(const void* src, void* dst, const int32_t* sidx, const int32_t* didx,
                           uint32_t stride, int64_t n, hipStream_t s);
// perm[p] = p, key[p] = key_sorted[p]
hipError_t launch_sorted_index(int32_t* perm, int32_t* key, const int32_t* key_sorted, int64_t n,
                               hipStream_t s);
hipError_t launch_kick_drift(const FieldRef* f, const Access& rec, const Geom& g,
                             const DevState* st, int64_t n, hipStream_t s);
int pair_grid_blocks(int64_t max_items);
// the parts of a cells handle that the tuner saves and puts back around its
// trials on records stored cell by cell (abi.cpp)
// SPHV_OK when the device may address every member of records 0..n-1 of aos
// (device, managed, or pinned host memory mapped at the same address), else
// SPHV_E_INVALID_ARG; checked on the host before anything is enqueued
int32_t check_records(const void* aos, const sphv_descriptor* d, int64_t n);
CellsDev* cells_dev(sphv_cells* c);
bool cells_sorted(const sphv_cells* c);
void cells_set_sorted(sphv_cells* c, bool sorted);
}  // namespace sphv
