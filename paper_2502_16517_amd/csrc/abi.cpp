// Host side of libsphview.so: argument validation, view planning, the alias
// registry for open views, workspace carving and kernel launch set-up.
// Every exported function is extern "C" and returns an sphv status code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"

using namespace sphv;

namespace {

constexpr uint64_t kAlign = 256;
constexpr int32_t kMaxListCap = 4096;

uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

uint32_t dtype_size(uint32_t dt)
{
    switch (dt) {
    case SPHV_F64: case SPHV_I64: return 8;
    case SPHV_F32: case SPHV_I32: return 4;
    default: return 0;
    }
}

bool is_pow2(uint64_t v) { return v && !(v & (v - 1)); }

// Validate a descriptor for n records; on success fill a role -> field table.
int32_t check_descriptor(const sphv_descriptor* d, int64_t n, int role_field[SPHV_NROLES])
{
    if (!d || n < 0) return SPHV_E_INVALID_ARG;
    if (d->n_fields > (uint32_t)kMaxFields) return SPHV_E_DESCRIPTOR;
    if (d->n_fields && !d->fields) return SPHV_E_INVALID_ARG;
    if (d->stride == 0) return SPHV_E_DESCRIPTOR;
    if (d->flags & ~(uint32_t)SPHV_DESC_RECORD_POINTERS) return SPHV_E_DESCRIPTOR;
    // records reached by address: array-of-structs shape, 8-byte aligned records
    if ((d->flags & SPHV_DESC_RECORD_POINTERS) && d->stride % 8) return SPHV_E_DESCRIPTOR;
    for (int r = 0; r < SPHV_NROLES; ++r) role_field[r] = -1;
    bool aos = true;
    for (uint32_t k = 0; k < d->n_fields; ++k) {
        const sphv_field& f = d->fields[k];
        uint32_t sz = dtype_size(f.dtype);
        if (!sz) return SPHV_E_DESCRIPTOR;
        if (f.access < SPHV_IN || f.access > SPHV_INOUT) return SPHV_E_DESCRIPTOR;
        if (f.role >= SPHV_NROLES) return SPHV_E_DESCRIPTOR;
        if (f.offset % sz) return SPHV_E_DESCRIPTOR;
        if (f.role != SPHV_ROLE_USER) {
            if (role_field[f.role] >= 0) return SPHV_E_DESCRIPTOR;
            role_field[f.role] = (int)k;
        }
        if (f.offset + sz > d->stride) aos = false;
    }
    if (!aos && (d->flags & SPHV_DESC_RECORD_POINTERS)) return SPHV_E_DESCRIPTOR;
    if (aos) {
        for (uint32_t k = 0; k < d->n_fields; ++k) {
            uint32_t sz = dtype_size(d->fields[k].dtype);
            if (d->stride % sz) return SPHV_E_DESCRIPTOR;
            for (uint32_t l = k + 1; l < d->n_fields; ++l) {
                uint64_t a0 = d->fields[k].offset, a1 = a0 + sz;
                uint64_t b0 = d->fields[l].offset, b1 = b0 + dtype_size(d->fields[l].dtype);
                if (a0 < b1 && b0 < a1) return SPHV_E_DESCRIPTOR;
            }
        }
        return SPHV_OK;
    }
    // struct of arrays: stride == element size, whole arrays disjoint
    for (uint32_t k = 0; k < d->n_fields; ++k) {
        uint64_t sz = dtype_size(d->fields[k].dtype);
        if (sz != d->stride) return SPHV_E_DESCRIPTOR;
        for (uint32_t l = k + 1; l < d->n_fields; ++l) {
            uint64_t a0 = d->fields[k].offset, a1 = a0 + sz * (uint64_t)n;
            uint64_t b0 = d->fields[l].offset, b1 = b0 + sz * (uint64_t)n;
            if (n > 0 && a0 < b1 && b0 < a1) return SPHV_E_DESCRIPTOR;
        }
    }
    return SPHV_OK;
}

uint64_t record_span(const sphv_descriptor* d, int64_t n)
{
    // records reached by address: the span of the address list
    if (d->flags & SPHV_DESC_RECORD_POINTERS) return 8 * (uint64_t)std::max<int64_t>(n, 0);
    uint64_t hi = 0;
    for (uint32_t k = 0; k < d->n_fields; ++k) {
        uint64_t sz = dtype_size(d->fields[k].dtype);
        uint64_t e = d->fields[k].offset + sz + (n > 0 ? (uint64_t)(n - 1) * d->stride : 0);
        hi = std::max(hi, e);
    }
    return hi;
}

bool finite_params(const sphv_params* p)
{
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(p->lo[d]) || !(p->len[d] > 0.0) || p->grid[d] < 1 ||
            !(p->cell[d] > 0.0) || !(p->inv_cell[d] > 0.0))
            return false;
    return std::isfinite(p->gamma) && p->gamma > 1.0 && p->eta > 0.0 && p->cfl > 0.0 &&
           p->h_tol >= 0.0 && p->headroom >= 1.0 && p->max_iter >= 1 && p->max_iter <= 64 &&
           (p->kernel == SPHV_KERNEL_CUBIC || p->kernel == SPHV_KERNEL_QUARTIC) && p->list_cap >= 0 &&
           p->list_cap <= kMaxListCap && (p->symmetric == 0 || (p->symmetric == 1 && p->list_cap > 0));
}

Geom geom_of(const sphv_params* p)
{
    Geom g;
    for (int d = 0; d < 3; ++d) {
        g.lo[d] = p->lo[d];
        g.len[d] = p->len[d];
        g.cell[d] = p->cell[d];
        g.inv_cell[d] = p->inv_cell[d];
        g.n[d] = p->grid[d];
        g.periodic[d] = p->periodic[d] ? 1 : 0;
    }
    g.cmin = std::min(p->cell[0], std::min(p->cell[1], p->cell[2]));
    g.headroom = p->headroom;
    return g;
}

int32_t hip_status(hipError_t e) { return e == hipSuccess ? SPHV_OK : SPHV_E_HIP; }

}  // namespace

// ------------------------------------------------------------------ handles

struct sphv_cells {
    CellsDev dev;
    sphv_params params;
    bool built = false;
    bool sorted = false;   // records moved into cell order since the last build
};

struct FieldPlan {
    sphv_field f;          // as described by the caller
    uint32_t view_dtype;
    uint32_t view_size;
    int32_t rel_axis;
    uint64_t view_off;     // byte offset of the field (SoA: array start; AoSoA: inside a block)
};

struct sphv_view {
    bool records_ok = false;          // the records' addresses passed check_records
    std::vector<sphv_field> fields;   // own copy of the caller's descriptor fields
    std::vector<FieldPlan> plan;
    int role_field[SPHV_NROLES];
    sphv_descriptor desc;
    int64_t n = 0;
    sphv_layout layout{};
    int32_t precision = 0;
    char* aos = nullptr;
    const int32_t* index = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    uint64_t fields_bytes = 0;
    uint64_t block_len = 0;     // elements per block (SoA: n rounded)
    uint64_t block_bytes = 0;
    uint32_t lw = 63;
    double* red_part = nullptr; // reduction partials
    int open = 0;               // 1 between aos_to_soa and soa_to_aos; 2 after a prefetch
    int gathered = 0;
    uint64_t prefetched = 0;    // bit k: member k of the plan was gathered by a prefetch
};

struct sphv_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

std::mutex g_open_mutex;
std::vector<sphv_view*> g_open;

// How view v uses member k while registered: as described when open, read
// only and only the prefetched members after a prefetch.
uint16_t member_use(const sphv_view* v, size_t k)
{
    if (v->open == 2) return ((v->prefetched >> k) & 1u) ? (uint16_t)SPHV_IN : (uint16_t)0;
    return v->plan[k].f.access;
}

bool members_meet(const sphv_view* a, uint16_t amask, const sphv_view* b, uint16_t bmask)
{
    for (size_t i = 0; i < a->plan.size(); ++i) {
        const FieldPlan& x = a->plan[i];
        if (!(member_use(a, i) & amask)) continue;
        uint64_t x0 = x.f.offset, x1 = x0 + dtype_size(x.f.dtype);
        for (size_t k = 0; k < b->plan.size(); ++k) {
            const FieldPlan& y = b->plan[k];
            if (!(member_use(b, k) & bmask)) continue;
            uint64_t y0 = y.f.offset, y1 = y0 + dtype_size(y.f.dtype);
            if (x0 < y1 && y0 < x1) return true;
        }
    }
    return false;
}

bool views_conflict(const sphv_view* a, const sphv_view* b)
{
    uint64_t a0 = (uint64_t)a->aos, a1 = a0 + record_span(&a->desc, a->n);
    uint64_t b0 = (uint64_t)b->aos, b1 = b0 + record_span(&b->desc, b->n);
    if (!(a0 < b1 && b0 < a1)) return false;
    if (a->desc.stride != b->desc.stride) return true;   // different shapes: be strict
    // A_out of one meets A_in u A_out of the other (paper Sec. 3.3)
    return members_meet(a, SPHV_OUT, b, SPHV_INOUT) || members_meet(b, SPHV_OUT, a, SPHV_INOUT);
}

FieldRef ref_view(const sphv_view* v, const FieldPlan& p)
{
    FieldRef r;
    r.base = v->ws;
    r.off = p.view_off;
    r.size = p.view_size;
    r.dtype = p.view_dtype;
    r.rel_axis = p.rel_axis;
    r.pad = 0;
    return r;
}

bool by_pointer(const sphv_descriptor& d) { return (d.flags & SPHV_DESC_RECORD_POINTERS) != 0; }

// A member of the records: base + offset of record 0, or (records reached by
// address) a null base to which each record's address is added.
FieldRef ref_rec(char* aos, const sphv_field& f, const sphv_descriptor& d)
{
    FieldRef r;
    r.base = by_pointer(d) ? nullptr : aos;
    r.off = f.offset;
    r.size = dtype_size(f.dtype);
    r.dtype = f.dtype;
    r.rel_axis = -1;
    r.pad = 0;
    return r;
}

Access acc_view(const sphv_view* v)
{
    Access a{};
    a.lw = v->lw;
    a.mask = v->lw >= 63 ? ~0ull : (v->block_len - 1);
    a.block_bytes = v->lw >= 63 ? 0 : v->block_bytes;
    a.index = nullptr;
    a.stride = 0;
    return a;
}

Access acc_rec(const int32_t* index, const sphv_descriptor& d, const void* aos)
{
    Access a{};
    a.lw = 0;
    a.mask = 0;
    a.block_bytes = 0;
    a.index = index;
    a.stride = d.stride;
    a.ptrs = by_pointer(d) ? (const uint64_t*)aos : nullptr;
    return a;
}

// Cells workspace carving (all arrays 256-B aligned).
uint64_t carve_cells(CellsDev* c, char* base, int64_t n, int64_t nc, int32_t list_cap, int32_t symmetric)
{
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) { char* p = base ? base + off : nullptr; off = align_up(off + bytes, kAlign); return p; };
    // a non-empty cell of c particles gives ceil(c / 64) <= 1 + c / 64 items and a
    // run of sparse cells one item, so items <= min(cells, particles) + n / 64
    int64_t max_items = std::min<int64_t>(nc, n) + (n + kWave - 1) / kWave + 1;
    int64_t scan_blocks = (std::max(nc, max_items) + 1023) / 1024 + 1;
    c->key = (int32_t*)take(4 * (uint64_t)std::max<int64_t>(n, 1));
    c->sub = (int32_t*)take(4 * (uint64_t)std::max<int64_t>(n, 1));
    c->perm = (int32_t*)take(4 * (uint64_t)std::max<int64_t>(n, 1));
    c->perm_tmp = (int32_t*)take(4 * (uint64_t)std::max<int64_t>(n, 1));
    c->key_sorted = (int32_t*)take(4 * (uint64_t)std::max<int64_t>(n, 1));
    c->cell_start = (int32_t*)take(4 * (uint64_t)(nc + 1));
    c->counts = (int32_t*)take(4 * (uint64_t)nc);
    c->cursor = (int32_t*)take(4 * (uint64_t)nc);
    c->hmax_bits = (uint32_t*)take(4 * (uint64_t)nc * 2);
    c->hmax_f = c->hmax_bits ? c->hmax_bits + nc : nullptr;
    c->reach_d = (int32_t*)take(4 * (uint64_t)nc * 3);
    c->reach_f = c->reach_d ? c->reach_d + nc : nullptr;
    c->reach_s = c->reach_d ? c->reach_d + 2 * nc : nullptr;
    c->tmp_a = (int32_t*)take(4 * (uint64_t)nc);
    c->tmp_b = (int32_t*)take(4 * (uint64_t)nc);
    c->cover = (uint64_t*)take(8 * 2 * (uint64_t)nc);
    c->item_start = (int32_t*)take(4 * (uint64_t)(nc + 1));
    c->items = (int4*)take(16 * (uint64_t)max_items);
    c->item_masks = (uint64_t*)take(8ull * kMaskChunks * kWave * (uint64_t)max_items);
    c->pair_part = (int64_t*)take(8ull * kPartSlots * kMaxPairBlocks);
    c->scan_part = (int32_t*)take(4 * (uint64_t)scan_blocks);
    c->meta = (int32_t*)take(4 * META_SIZE);
    c->list_cap = list_cap;
    c->list = list_cap > 0 ? (int32_t*)take(4 * (uint64_t)list_cap * (uint64_t)std::max<int64_t>(n, 1)) : nullptr;
    c->fconst = (double*)take(5 * 8 * (uint64_t)std::max<int64_t>(n, 1));
    c->blocks = list_cap > 0 ? (double*)take(8ull * kBlockWords * (uint64_t)(n / kBlock + 1)) : nullptr;
    c->list_len = list_cap > 0 ? (int32_t*)take(4 * (uint64_t)std::max<int64_t>(n, 1)) : nullptr;
    c->slots = list_cap > 0 && symmetric
                   ? (double*)take(5 * 8 * (uint64_t)list_cap * (uint64_t)std::max<int64_t>(n, 1)) : nullptr;
    c->n = n;
    c->nc = nc;
    c->max_items = max_items;
    return off;
}

// View planning: field storage in the workspace, then the reduction partials.
void plan_view(sphv_view* v)
{
    const sphv_layout& l = v->layout;
    int64_t n = v->n;
    v->plan.clear();
    for (uint32_t k = 0; k < v->desc.n_fields; ++k) {
        FieldPlan p;
        p.f = v->desc.fields[k];
        p.view_dtype = p.f.dtype;
        p.rel_axis = -1;
        if (v->precision == SPHV_PREC_FP32 && p.f.access == SPHV_IN && p.f.dtype == SPHV_F64) {
            p.view_dtype = SPHV_F32;
            if (p.f.role == SPHV_X) p.rel_axis = 0;
            if (p.f.role == SPHV_Y) p.rel_axis = 1;
            if (p.f.role == SPHV_Z) p.rel_axis = 2;
        }
        p.view_size = dtype_size(p.view_dtype);
        p.view_off = 0;
        v->plan.push_back(p);
    }
    uint64_t off = 0;
    if (l.kind == SPHV_LAYOUT_SOA) {
        v->lw = 63;
        v->block_len = (uint64_t)std::max<int64_t>(n, 1);
        for (FieldPlan& p : v->plan) {
            p.view_off = off;
            off = align_up(off + (uint64_t)std::max<int64_t>(n, 1) * p.view_size, kAlign);
        }
        v->block_bytes = off;
    } else if (l.kind == SPHV_LAYOUT_AOSOA) {
        uint64_t w = l.aosoa_width;
        uint32_t lw = 0;
        while ((1ull << lw) < w) ++lw;
        v->lw = lw;
        v->block_len = w;
        uint64_t bo = 0;
        for (FieldPlan& p : v->plan) {
            p.view_off = bo;
            bo += w * p.view_size;
        }
        v->block_bytes = align_up(bo, 64);
        off = align_up(v->block_bytes * (((uint64_t)n + w - 1) / w), kAlign);
    } else {
        v->lw = 0;
        v->block_len = 0;
        v->block_bytes = 0;
    }
    v->fields_bytes = off;
}

uint64_t view_bytes_of(const sphv_view* v)
{
    uint64_t nred = ((uint64_t)v->n + kRedBlock - 1) / kRedBlock + 1;
    return v->fields_bytes + align_up(nred * 16 * sizeof(double), kAlign);
}

// layouts whose loops run on the records themselves (no explicit storage)
bool is_direct(uint32_t kind) { return kind == SPHV_LAYOUT_DIRECT || kind == SPHV_LAYOUT_SORTED; }

int32_t check_layout(const sphv_layout* l, int32_t precision)
{
    if (!l) return SPHV_E_INVALID_ARG;
    if (l->kind > SPHV_LAYOUT_SORTED) return SPHV_E_INVALID_ARG;
    if (l->kind == SPHV_LAYOUT_AOSOA && (!is_pow2(l->aosoa_width) || l->aosoa_width < 1 || l->aosoa_width > 1024))
        return SPHV_E_INVALID_ARG;
    if (l->tpi > 64) return SPHV_E_INVALID_ARG;
    if (l->masked > 1) return SPHV_E_INVALID_ARG;
    if (precision != SPHV_PREC_FP64 && precision != SPHV_PREC_FP32) return SPHV_E_INVALID_ARG;
    return SPHV_OK;
}

// role requirements: readable (IN bit) or writable (OUT bit), f64 in the records
// The view's records are addressable by the device (checked once per view).
int32_t records_ok(sphv_view* v)
{
    if (v->records_ok) return SPHV_OK;
    if (int32_t r = check_records(v->aos, &v->desc, v->n)) return r;
    v->records_ok = true;
    return SPHV_OK;
}

int32_t need(const sphv_view* v, int role, uint16_t bits)
{
    int k = v->role_field[role];
    if (k < 0) return SPHV_E_DESCRIPTOR;
    const sphv_field& f = v->plan[k].f;
    if ((f.access & bits) != bits) return SPHV_E_DESCRIPTOR;
    if (f.dtype != SPHV_F64) return SPHV_E_DESCRIPTOR;
    return SPHV_OK;
}

}  // namespace

// ================================================================= exports

extern "C" {

const char* sphv_status_string(int32_t s)
{
    switch (s) {
    case SPHV_OK: return "ok";
    case SPHV_E_INVALID_ARG: return "invalid argument";
    case SPHV_E_DESCRIPTOR: return "invalid or insufficient descriptor";
    case SPHV_E_WORKSPACE: return "workspace too small or misaligned";
    case SPHV_E_ALIAS: return "conflicting open view on the same records";
    case SPHV_E_STATE: return "call out of order";
    case SPHV_E_HIP: return "HIP runtime error";
    case SPHV_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

int32_t sphv_version(void) { return 100; }

int32_t sphv_params_init(sphv_params* p, const double lo[3], const double len[3],
                         const int32_t grid[3], const int32_t periodic[3])
{
    if (!p || !lo || !len || !grid || !periodic) return SPHV_E_INVALID_ARG;
    std::memset(p, 0, sizeof(*p));
    for (int d = 0; d < 3; ++d) {
        if (!(len[d] > 0.0) || grid[d] < 1) return SPHV_E_INVALID_ARG;
        p->lo[d] = lo[d];
        p->len[d] = len[d];
        p->grid[d] = grid[d];
        p->periodic[d] = periodic[d] ? 1 : 0;
        p->cell[d] = len[d] / (double)grid[d];
        p->inv_cell[d] = (double)grid[d] / len[d];
    }
    p->gamma = 5.0 / 3.0;
    p->eta = 1.2;
    p->cfl = 0.3;
    p->h_tol = 1e-13;
    p->headroom = 1.1;
    p->max_iter = 16;
    return SPHV_OK;
}

size_t sphv_state_bytes(void) { return sizeof(DevState); }

int32_t sphv_state_init(void* st, void* stream)
{
    if (!st) return SPHV_E_INVALID_ARG;
    return hip_status(launch_state_init((DevState*)st, 1, (hipStream_t)stream));
}

int32_t sphv_begin_step(void* st, void* stream)
{
    if (!st) return SPHV_E_INVALID_ARG;
    return hip_status(launch_state_init((DevState*)st, 0, (hipStream_t)stream));
}

int32_t sphv_read_state(const void* st, sphv_state* out, void* stream)
{
    if (!st || !out) return SPHV_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(out, st, sizeof(sphv_state), hipMemcpyDeviceToHost, s) != hipSuccess)
        return SPHV_E_HIP;
    return hip_status(hipStreamSynchronize(s));
}

int32_t sphv_write_state(void* st, const sphv_state* in, void* stream)
{
    if (!st || !in) return SPHV_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(st, in, sizeof(sphv_state), hipMemcpyHostToDevice, s) != hipSuccess)
        return SPHV_E_HIP;
    return hip_status(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------- cells

size_t sphv_cells_workspace_bytes(int64_t n, const sphv_params* p)
{
    if (!p || n < 0 || !finite_params(p)) return 0;
    int64_t nc = (int64_t)p->grid[0] * p->grid[1] * p->grid[2];
    CellsDev c{};
    return (size_t)carve_cells(&c, nullptr, n, nc, p->list_cap, p->symmetric);
}

int32_t sphv_cells_create(sphv_cells** out, int64_t n, const sphv_params* p, void* ws, size_t ws_bytes)
{
    if (!out || !p || n < 0 || (n > 0 && !ws)) return SPHV_E_INVALID_ARG;
    *out = nullptr;
    if (!finite_params(p)) return SPHV_E_INVALID_ARG;
    if (n > INT32_MAX - 1) return SPHV_E_UNSUPPORTED;
    int64_t nc = (int64_t)p->grid[0] * p->grid[1] * p->grid[2];
    if (nc > INT32_MAX / 2) return SPHV_E_UNSUPPORTED;
    if ((uintptr_t)ws % kAlign) return SPHV_E_WORKSPACE;
    CellsDev c{};
    uint64_t need_b = carve_cells(&c, nullptr, n, nc, p->list_cap, p->symmetric);
    if (ws_bytes < need_b) return SPHV_E_WORKSPACE;
    sphv_cells* h = new (std::nothrow) sphv_cells;
    if (!h) return SPHV_E_INVALID_ARG;
    carve_cells(&h->dev, (char*)ws, n, nc, p->list_cap, p->symmetric);
    h->params = *p;
    *out = h;
    return SPHV_OK;
}

int32_t sphv_cells_build(sphv_cells* c, const void* aos, const sphv_descriptor* d, void* state, void* stream)
{
    if (!c || !d || !state || (c->dev.n > 0 && !aos)) return SPHV_E_INVALID_ARG;
    int rf[SPHV_NROLES];
    int32_t st = check_descriptor(d, c->dev.n, rf);
    if (st) return st;
    if ((st = check_records(aos, d, c->dev.n))) return st;
    const int roles[4] = {SPHV_X, SPHV_Y, SPHV_Z, SPHV_H};
    FieldRef f[4];
    for (int k = 0; k < 4; ++k) {
        if (rf[roles[k]] < 0 || d->fields[rf[roles[k]]].dtype != SPHV_F64) return SPHV_E_DESCRIPTOR;
        f[k] = ref_rec((char*)aos, d->fields[rf[roles[k]]], *d);
    }
    Access rec = acc_rec(nullptr, *d, aos);
    Geom g = geom_of(&c->params);
    c->sorted = false;
    hipError_t e = launch_cells_build(c->dev, f, rec, g, (DevState*)state, (hipStream_t)stream);
    if (e != hipSuccess) return SPHV_E_HIP;
    c->built = true;
    return SPHV_OK;
}

size_t sphv_records_sort_workspace_bytes(uint32_t stride, int64_t n)
{
    if (stride == 0 || stride % 4 || n < 0) return 0;
    return (size_t)align_up((uint64_t)stride * (uint64_t)std::max<int64_t>(n, 1), kAlign);
}

int32_t sphv_records_sort(sphv_cells* c, void* aos, uint32_t stride, void* ws, size_t ws_bytes, void* stream)
{
    if (!c || stride == 0 || stride % 4 || (uintptr_t)aos % 4) return SPHV_E_INVALID_ARG;
    const int64_t n = c->dev.n;
    if (n > 0 && !aos) return SPHV_E_INVALID_ARG;
    if (!ws || (uintptr_t)ws % kAlign || ws_bytes < sphv_records_sort_workspace_bytes(stride, n))
        return SPHV_E_WORKSPACE;

    if (!c->built) return SPHV_E_STATE;
    {
        // whole records: from aos to the last byte of record n-1
        const sphv_field last{stride - 4u, SPHV_ROLE_USER, SPHV_I32, SPHV_INOUT};
        const sphv_descriptor dl{stride, 1, 0, &last};
        if (int32_t r = check_records(aos, &dl, n)) return r;
    }
    hipStream_t s = (hipStream_t)stream;
    // sorted copy in the workspace, then back over the records in storage order
    if (launch_rec_move(aos, ws, c->dev.perm, nullptr, stride, n, s) != hipSuccess) return SPHV_E_HIP;
    if (launch_rec_move(ws, aos, nullptr, nullptr, stride, n, s) != hipSuccess) return SPHV_E_HIP;
    if (launch_sorted_index(c->dev.perm, c->dev.key, c->dev.key_sorted, n, s) != hipSuccess) return SPHV_E_HIP;
    c->sorted = true;
    return SPHV_OK;
}

// ------------------------------------------- records sort without allocation
//
// The sorted copy of sphv_records_sort_static lives in one file-scope device
// array per GPU.  In host code the array's name is only a stand-in for the
// symbol: its device address is looked up once per device (with that device
// current) and only that address is ever handed to kernels.

static __device__ __align__(256) unsigned char scratch[SPHV_RECORDS_SORT_STATIC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Device address of this device's scratch array, or nullptr on a HIP error.
void* scratch_of_current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

int32_t sphv_records_sort_static(sphv_cells* c, void* aos, uint32_t stride, void* stream)
{
    if (!c || stride == 0 || stride % 4 || (uintptr_t)aos % 4) return SPHV_E_INVALID_ARG;
    const int64_t n = c->dev.n;
    if (n > 0 && !aos) return SPHV_E_INVALID_ARG;
    if ((uint64_t)stride * (uint64_t)n > (uint64_t)SPHV_RECORDS_SORT_STATIC_MAX_BYTES) return SPHV_E_WORKSPACE;
    if (!c->built) return SPHV_E_STATE;
    {
        const sphv_field last{stride - 4u, SPHV_ROLE_USER, SPHV_I32, SPHV_INOUT};
        const sphv_descriptor dl{stride, 1, 0, &last};
        if (int32_t r = check_records(aos, &dl, n)) return r;
    }
    void* ws = scratch_of_current_device();
    if (!ws) return SPHV_E_HIP;
    hipStream_t s = (hipStream_t)stream;
    // the same three kernels as sphv_records_sort, the copy in this device's array
    if (launch_rec_move(aos, ws, c->dev.perm, nullptr, stride, n, s) != hipSuccess) return SPHV_E_HIP;
    if (launch_rec_move(ws, aos, nullptr, nullptr, stride, n, s) != hipSuccess) return SPHV_E_HIP;
    if (launch_sorted_index(c->dev.perm, c->dev.key, c->dev.key_sorted, n, s) != hipSuccess) return SPHV_E_HIP;
    c->sorted = true;
    return SPHV_OK;
}

int32_t sphv_cells_get_info(const sphv_cells* c, sphv_cells_info* out)
{
    if (!c || !out) return SPHV_E_INVALID_ARG;
    out->perm = c->dev.perm;
    out->cell_start = c->dev.cell_start;
    out->key = c->dev.key;
    out->reach = c->dev.reach_d;
    out->n = c->dev.n;
    out->n_cells = c->dev.nc;
    out->max_items = c->dev.max_items;
    return SPHV_OK;
}

void sphv_cells_destroy(sphv_cells* c) { delete c; }

// ------------------------------------------------------------------- views

size_t sphv_view_workspace_bytes(const sphv_descriptor* d, int64_t n, const sphv_layout* l, int32_t precision)
{
    int rf[SPHV_NROLES];
    if (check_descriptor(d, n, rf) || check_layout(l, precision)) return 0;
    sphv_view v;
    v.desc = *d;
    v.n = n;
    v.layout = *l;
    v.precision = precision;
    plan_view(&v);
    return (size_t)view_bytes_of(&v);
}

int32_t sphv_view_create(sphv_view** out, const sphv_descriptor* d, int64_t n, const sphv_layout* l,
                         int32_t precision, void* aos, const int32_t* index, void* ws, size_t ws_bytes)
{
    if (!out) return SPHV_E_INVALID_ARG;
    *out = nullptr;
    if (n > INT32_MAX - 1) return SPHV_E_UNSUPPORTED;
    if (!aos && n > 0) return SPHV_E_INVALID_ARG;
    int32_t st = check_layout(l, precision);
    if (st) return st;
    sphv_view* v = new (std::nothrow) sphv_view;
    if (!v) return SPHV_E_INVALID_ARG;
    st = check_descriptor(d, n, v->role_field);
    if (st) { delete v; return st; }
    // the sorted layout needs records moved into cell order: contiguous ones only
    if ((d->flags & SPHV_DESC_RECORD_POINTERS) && l->kind == SPHV_LAYOUT_SORTED) { delete v; return SPHV_E_UNSUPPORTED; }
    v->fields.assign(d->fields, d->fields + d->n_fields);
    v->desc = *d;
    v->desc.fields = v->fields.data();
    v->n = n;
    v->layout = *l;
    v->precision = precision;
    v->aos = (char*)aos;
    v->index = index;
    plan_view(v);
    uint64_t need_b = view_bytes_of(v);
    if (!ws || (uintptr_t)ws % kAlign) { delete v; return SPHV_E_WORKSPACE; }
    if (ws_bytes < need_b) { delete v; return SPHV_E_WORKSPACE; }
    v->ws = (char*)ws;
    v->ws_bytes = ws_bytes;
    v->red_part = (double*)(v->ws + v->fields_bytes);
    *out = v;
    return SPHV_OK;
}

int32_t sphv_view_field(const sphv_view* v, uint32_t k, void** ptr, int32_t* dtype, uint64_t* block_len,
                        uint64_t* block_bytes)
{
    if (!v || !ptr || !dtype || !block_len || !block_bytes) return SPHV_E_INVALID_ARG;
    if (k >= v->plan.size()) return SPHV_E_INVALID_ARG;
    if (is_direct(v->layout.kind)) return SPHV_E_UNSUPPORTED;
    *ptr = v->ws + v->plan[k].view_off;
    *dtype = (int32_t)v->plan[k].view_dtype;
    *block_len = v->layout.kind == SPHV_LAYOUT_SOA ? (uint64_t)v->n : v->block_len;
    *block_bytes = v->layout.kind == SPHV_LAYOUT_SOA ? v->block_bytes : v->block_bytes;
    return SPHV_OK;
}

namespace {

// Gathers the plan members of v selected by mask (records -> view storage).
int32_t gather_members(sphv_view* v, const sphv_cells* cells, bool needs_cells, uint64_t mask, void* stream)
{
    FieldRef src[kMaxFields], dst[kMaxFields];
    int nf = 0;
    for (size_t k = 0; k < v->plan.size(); ++k) {
        if (!((mask >> k) & 1u)) continue;
        src[nf] = ref_rec(v->aos, v->plan[k].f, v->desc);
        dst[nf] = ref_view(v, v->plan[k]);
        ++nf;
    }
    if (!nf) return SPHV_OK;
    Access sa = acc_rec(v->index, v->desc, v->aos);
    Access da = acc_view(v);
    Geom g{};
    const int32_t* key = nullptr;
    if (needs_cells) {
        g = geom_of(&cells->params);
        key = cells->dev.key;
    }
    return hip_status(launch_gather(src, dst, nf, sa, da, key, g, v->n, (hipStream_t)stream));
}

bool cells_fit(const sphv_view* v, const sphv_cells* cells, bool& needs_cells)
{
    needs_cells = false;
    for (const FieldPlan& p : v->plan) needs_cells |= p.rel_axis >= 0;
    return !(needs_cells && (!cells || !cells->built || cells->dev.n != v->n || v->index != cells->dev.perm));
}

}  // namespace

int32_t sphv_aos_to_soa_prefetch(sphv_view* v, const sphv_cells* cells, void* stream)
{
    if (!v) return SPHV_E_INVALID_ARG;
    if (v->open) return SPHV_E_STATE;
    bool needs_cells = false;
    if (!cells_fit(v, cells, needs_cells)) return SPHV_E_STATE;
    if (is_direct(v->layout.kind) || v->n == 0) return SPHV_OK;     // nothing is copied
    if (int32_t r = records_ok(v)) return r;
    uint64_t mask = 0;
    {
        std::lock_guard<std::mutex> lk(g_open_mutex);
        // the members v only reads and that no registered view writes
        for (size_t k = 0; k < v->plan.size(); ++k) {
            if (v->plan[k].f.access != SPHV_IN) continue;
            v->prefetched = 1ull << k;
            v->open = 2;
            bool free = true;
            for (sphv_view* o : g_open) free = free && !views_conflict(v, o);
            if (free) mask |= 1ull << k;
        }
        v->prefetched = mask;
        v->open = mask ? 2 : 0;
        if (mask) g_open.push_back(v);
    }
    return gather_members(v, cells, needs_cells, mask, stream);
}

int32_t sphv_aos_to_soa(sphv_view* v, const sphv_cells* cells, void* stream)
{
    if (!v) return SPHV_E_INVALID_ARG;
    if (v->open == 1) return SPHV_E_STATE;
    bool needs_cells = false;
    if (!cells_fit(v, cells, needs_cells)) return SPHV_E_STATE;
    // the gather reads the records: checked once per view, before its first
    // gather (a view on the records is checked by the first loop call instead)
    if (!is_direct(v->layout.kind))
        if (int32_t r = records_ok(v)) return r;
    {
        // views on the records themselves (direct, sorted) write the records'
        // members in place, so they take part in the rule like any other view;
        // after a prefetch the view is registered already, as a reader of the
        // members it prefetched, and now takes all of its members
        std::lock_guard<std::mutex> lk(g_open_mutex);
        const int was = v->open;
        v->open = 1;
        for (sphv_view* o : g_open)
            if (o != v && views_conflict(v, o)) {
                v->open = was;
                return SPHV_E_ALIAS;
            }
        if (!was) g_open.push_back(v);
    }
    v->gathered = 1;
    if (is_direct(v->layout.kind) || v->n == 0) return SPHV_OK;
    uint64_t mask = 0;
    for (size_t k = 0; k < v->plan.size(); ++k)
        if ((v->plan[k].f.access & SPHV_IN) && !((v->prefetched >> k) & 1u)) mask |= 1ull << k;  // A_out \ A_in: none
    return gather_members(v, cells, needs_cells, mask, stream);
}

int32_t sphv_soa_to_aos(sphv_view* v, void* stream)
{
    if (!v) return SPHV_E_INVALID_ARG;
    if (v->open != 1) return SPHV_E_STATE;
    {
        std::lock_guard<std::mutex> lk(g_open_mutex);
        g_open.erase(std::remove(g_open.begin(), g_open.end(), v), g_open.end());
    }
    v->open = 0;
    v->prefetched = 0;
    if (is_direct(v->layout.kind) || v->n == 0) return SPHV_OK;
    FieldRef src[kMaxFields], dst[kMaxFields];
    int nf = 0;
    for (const FieldPlan& p : v->plan) {
        if (!(p.f.access & SPHV_OUT)) continue;    // only A_out goes back
        src[nf] = ref_view(v, p);
        dst[nf] = ref_rec(v->aos, p.f, v->desc);
        ++nf;
    }
    if (!nf) return SPHV_OK;
    Access sa = acc_view(v);
    Access da = acc_rec(v->index, v->desc, v->aos);
    return hip_status(launch_scatter(src, dst, nf, sa, da, v->n, (hipStream_t)stream));
}

void sphv_view_destroy(sphv_view* v)
{
    if (!v) return;
    {
        std::lock_guard<std::mutex> lk(g_open_mutex);
        g_open.erase(std::remove(g_open.begin(), g_open.end(), v), g_open.end());
    }
    delete v;
}

// -------------------------------------------------------------- pair loops

namespace {

// nstaged: the first roles_in that the loop stages for its neighbours; an FP32
// loop reads those from a view as stored floats
int32_t pair_setup(sphv_view* v, const sphv_cells* c, const sphv_params* p, void* state,
                   const int* roles_in, int nin, int nstaged, const int* roles_out, int nout, PairArgs* a)
{
    if (!v || !c || !p || !state) return SPHV_E_INVALID_ARG;
    if (!finite_params(p)) return SPHV_E_INVALID_ARG;
    if (v->open != 1) return SPHV_E_STATE;
    if (!c->built || c->dev.n != v->n || v->index != c->dev.perm) return SPHV_E_STATE;
    for (int k = 0; k < nin; ++k) if (int32_t s = need(v, roles_in[k], SPHV_IN)) return s;
    for (int k = 0; k < nout; ++k) if (int32_t s = need(v, roles_out[k], SPHV_OUT)) return s;
    bool direct = is_direct(v->layout.kind);
    // an FP32 view stores a member as a float only when the loop only reads it
    // (the gather's rounding); a member it also writes stays a double, which
    // the FP32 loops cannot stage
    if (v->precision == SPHV_PREC_FP32 && !direct)
        for (int k = 0; k < nstaged; ++k)
            if (v->plan[v->role_field[roles_in[k]]].view_dtype != SPHV_F32) return SPHV_E_DESCRIPTOR;
    if (int32_t r = records_ok(v)) return r;
    std::memset(a, 0, sizeof(*a));
    // a view over records stored cell by cell indexes them in storage order
    const bool sorted = v->layout.kind == SPHV_LAYOUT_SORTED;
    if (sorted && !c->sorted) return SPHV_E_STATE;
    for (int r = 1; r < SPHV_NROLES; ++r) {
        int k = v->role_field[r];
        if (k < 0) continue;
        a->f[r] = direct ? ref_rec(v->aos, v->plan[k].f, v->desc) : ref_view(v, v->plan[k]);
    }
    if (direct && v->precision == SPHV_PREC_FP32) {
        // FP32 loops over the records convert positions on the fly, exactly as
        // an FP32 view stores them: relative to the corner of their cell
        a->f[SPHV_X].rel_axis = 0;
        a->f[SPHV_Y].rel_axis = 1;
        a->f[SPHV_Z].rel_axis = 2;
    }
    a->acc = direct ? acc_rec(sorted ? nullptr : v->index, v->desc, v->aos) : acc_view(v);
    a->g = geom_of(p);
    a->items = c->dev.items;
    a->cell_start = c->dev.cell_start;
    a->key_sorted = c->dev.key_sorted;
    a->reach_d = c->dev.reach_d;
    a->item_masks = c->dev.item_masks;
    a->meta = c->dev.meta;
    a->part = c->dev.pair_part;
    a->state = (DevState*)state;
    a->eta = p->eta;
    a->tol = p->h_tol;
    a->gamma = p->gamma;
    a->cfl = p->cfl;
    a->max_iter = p->max_iter;
    a->tpi = (int32_t)v->layout.tpi;
    a->nblocks = pair_grid_blocks(c->dev.max_items);
    a->n = v->n;
    a->red_part = v->red_part;
    return SPHV_OK;
}

}  // namespace

int32_t sphv_sph_density(sphv_view* v, const sphv_cells* c, const sphv_params* p, void* state, void* stream)
{
    const int in[] = {SPHV_X, SPHV_Y, SPHV_Z, SPHV_M, SPHV_H};
    const int out[] = {SPHV_H, SPHV_RHO, SPHV_OMEGA, SPHV_WCOUNT};
    PairArgs a;
    int32_t s = pair_setup(v, c, p, state, in, 5, 4, out, 4, &a);
    if (s) return s;
    if (c->params.grid[0] != p->grid[0] || c->params.grid[1] != p->grid[1] || c->params.grid[2] != p->grid[2])
        return SPHV_E_INVALID_ARG;
    if (v->n == 0) return SPHV_OK;
    a.reach = c->dev.reach_d;
    a.qhead = META_QHEAD_D;
    if (c->dev.list_cap > 0) {
        a.list = c->dev.list;
        a.list_cap = c->dev.list_cap;
        a.list_len = c->dev.list_len;
        // the force constants' storage holds the hand-over of particles that leave
        // their list (the force loop fills it with its constants only later)
        a.fconst = c->dev.fconst;
        const int direct = is_direct(v->layout.kind), fp32 = v->precision == SPHV_PREC_FP32;
        if (launch_block_bounds(a, c->dev.blocks, direct, fp32, (hipStream_t)stream) != hipSuccess)
            return SPHV_E_HIP;
        a.blocks = c->dev.blocks;
        return hip_status(launch_density_list(a, direct, fp32, p->kernel, (hipStream_t)stream));
    }
    return hip_status(launch_density(a, is_direct(v->layout.kind), v->precision == SPHV_PREC_FP32,
                                     (int)v->layout.masked, p->kernel, (hipStream_t)stream));
}

int32_t sphv_sph_force(sphv_view* v, const sphv_cells* c, const sphv_params* p, void* state, void* stream)
{
    const int in[] = {SPHV_X, SPHV_Y, SPHV_Z, SPHV_VX, SPHV_VY, SPHV_VZ, SPHV_M, SPHV_H,
                      SPHV_RHO, SPHV_OMEGA, SPHV_U, SPHV_ALPHA};
    const int out[] = {SPHV_AX, SPHV_AY, SPHV_AZ, SPHV_UDT, SPHV_VSIG};
    PairArgs a;
    int32_t s = pair_setup(v, c, p, state, in, 12, 12, out, 5, &a);
    if (s) return s;
    // each pair once: the FP64 list walks only
    if (c->dev.slots && v->precision == SPHV_PREC_FP32) return SPHV_E_UNSUPPORTED;
    if (c->params.grid[0] != p->grid[0] || c->params.grid[1] != p->grid[1] || c->params.grid[2] != p->grid[2])
        return SPHV_E_INVALID_ARG;
    if (v->n == 0) return SPHV_OK;
    a.reach = c->dev.reach_f;
    a.reach_s = c->dev.reach_s;
    a.qhead = META_QHEAD_F;
    hipStream_t st = (hipStream_t)stream;
    bool direct = is_direct(v->layout.kind);
    // windows from the converged h: from the view when it holds h as a double
    // (an exact copy, or the density's h in a view over both loops), else from
    // the records (a member the view only reads is never modified while it is
    // open; an FP32 view holds it rounded to float)
    const FieldPlan& hp = v->plan[v->role_field[SPHV_H]];
    hipError_t e;
    if (!direct && hp.view_dtype == SPHV_F64) {
        const Access va = acc_view(v);
        e = launch_force_reach(c->dev, ref_view(v, hp), 0, &va, a.g, (DevState*)state, st);
    } else {
        e = launch_force_reach(c->dev, ref_rec(v->aos, hp.f, v->desc), v->desc.stride, nullptr, a.g, (DevState*)state, st,
                               by_pointer(v->desc) ? (const uint64_t*)v->aos : nullptr);
    }
    if (e != hipSuccess) return SPHV_E_HIP;
    a.fconst = c->dev.fconst;
    if (launch_force_prep(a, direct, v->precision == SPHV_PREC_FP32, st) != hipSuccess) return SPHV_E_HIP;
    if (c->dev.list_cap > 0) {
        a.list = c->dev.list;
        a.list_cap = c->dev.list_cap;
        if (launch_block_bounds(a, c->dev.blocks, direct, v->precision == SPHV_PREC_FP32, st) != hipSuccess)
            return SPHV_E_HIP;
        a.blocks = c->dev.blocks;
        a.cell_h = c->dev.hmax_f;
        a.list_len = c->dev.list_len;
        if (c->dev.slots) {
            a.slots = c->dev.slots;
            return hip_status(launch_force_sym(a, direct, p->kernel, st));
        }
        return hip_status(launch_force_list(a, direct, v->precision == SPHV_PREC_FP32, p->kernel, st));
    }
    return hip_status(launch_force(a, direct, v->precision == SPHV_PREC_FP32, (int)v->layout.masked, p->kernel, st));
}

int32_t sphv_step_reduce(sphv_view* v, const sphv_params* p, void* state, void* stream)
{
    if (!v || !p || !state) return SPHV_E_INVALID_ARG;
    if (!finite_params(p)) return SPHV_E_INVALID_ARG;
    if (v->open != 1) return SPHV_E_STATE;
    const int rin[6] = {SPHV_M, SPHV_VX, SPHV_VY, SPHV_VZ, SPHV_U, SPHV_H};
    const int rout[5] = {SPHV_AX, SPHV_AY, SPHV_AZ, SPHV_UDT, SPHV_VSIG};
    for (int k = 0; k < 6; ++k) if (int32_t s = need(v, rin[k], SPHV_IN)) return s;
    for (int k = 0; k < 5; ++k) if (int32_t s = need(v, rout[k], SPHV_OUT)) return s;
    if (int32_t s = records_ok(v)) return s;
    if (v->n == 0) return SPHV_OK;
    // outputs from where the loop wrote them; inputs from the view when it
    // holds them as doubles (an FP64 view: exact copies, or the density's h
    // in a view over both loops), else from the records (members a view only
    // reads are never modified while it is open)
    const bool direct = is_direct(v->layout.kind);
    bool in_view = !direct;
    for (int k = 0; k < 6; ++k) in_view = in_view && v->plan[v->role_field[rin[k]]].view_dtype == SPHV_F64;
    if (!direct && !in_view && (v->plan[v->role_field[SPHV_H]].f.access & SPHV_OUT))
        return SPHV_E_DESCRIPTOR;    // h written in the view but the other inputs stored as floats
    FieldRef in6[6], out5[5];
    for (int k = 0; k < 6; ++k) {
        const FieldPlan& fp = v->plan[v->role_field[rin[k]]];
        in6[k] = in_view ? ref_view(v, fp) : ref_rec(v->aos, fp.f, v->desc);
    }
    for (int k = 0; k < 5; ++k) {
        const FieldPlan& fp = v->plan[v->role_field[rout[k]]];
        out5[k] = direct ? ref_rec(v->aos, fp.f, v->desc) : ref_view(v, fp);
    }
    Access ra = acc_rec(v->index, v->desc, v->aos);
    Access oa = direct ? ra : acc_view(v);
    return hip_status(launch_force_reduce(in6, ra, out5, oa, direct, in_view, (DevState*)state, p->cfl, v->n,
                                          v->red_part, (hipStream_t)stream));
}

// -------------------------------------------------------------- kick/drift

int32_t sphv_kick_drift(void* aos, const sphv_descriptor* d, int64_t n, const sphv_params* p,
                        const void* state, void* stream)
{
    if (!d || !p || !state || (n > 0 && !aos)) return SPHV_E_INVALID_ARG;
    if (!finite_params(p)) return SPHV_E_INVALID_ARG;
    int rf[SPHV_NROLES];
    int32_t s = check_descriptor(d, n, rf);
    if (s) return s;
    if ((s = check_records(aos, d, n))) return s;
    const int roles[15] = {SPHV_X, SPHV_Y, SPHV_Z, SPHV_VX, SPHV_VY, SPHV_VZ, SPHV_VHX, SPHV_VHY, SPHV_VHZ,
                           SPHV_AX, SPHV_AY, SPHV_AZ, SPHV_U, SPHV_UH, SPHV_UDT};
    FieldRef f[15];
    for (int k = 0; k < 15; ++k) {
        int i = rf[roles[k]];
        if (i < 0 || d->fields[i].dtype != SPHV_F64) return SPHV_E_DESCRIPTOR;
        f[k] = ref_rec((char*)aos, d->fields[i], *d);
    }
    if (n == 0) return SPHV_OK;
    return hip_status(launch_kick_drift(f, acc_rec(nullptr, *d, aos), geom_of(p), (const DevState*)state, n,
                                        (hipStream_t)stream));
}

// ------------------------------------------------------------------ graphs

int32_t sphv_graph_begin(void* stream)
{
    return hip_status(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
}

int32_t sphv_graph_end(void* stream, sphv_graph** out)
{
    if (!out) return SPHV_E_INVALID_ARG;
    *out = nullptr;
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture((hipStream_t)stream, &g) != hipSuccess || !g) return SPHV_E_HIP;
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return SPHV_E_HIP;
    }
    sphv_graph* h = new (std::nothrow) sphv_graph;
    if (!h) {
        (void)hipGraphExecDestroy(ex);
        (void)hipGraphDestroy(g);
        return SPHV_E_INVALID_ARG;
    }
    h->graph = g;
    h->exec = ex;
    *out = h;
    return SPHV_OK;
}

int32_t sphv_graph_launch(sphv_graph* g, void* stream)
{
    if (!g) return SPHV_E_INVALID_ARG;
    return hip_status(hipGraphLaunch(g->exec, (hipStream_t)stream));
}

void sphv_graph_destroy(sphv_graph* g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"

namespace sphv {
namespace {
// An address the kernels may dereference: memory of the current device,
// managed memory, or pinned host memory that the device maps at the same
// address (hipHostMalloc).  Pageable host memory is not mapped, and another
// device's memory needs peer access: a kernel reading either could fault.
bool device_addressable(const void* p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (a.type == hipMemoryTypeManaged) return true;
    if (a.type == hipMemoryTypeDevice) {
        int dev = -1;
        return hipGetDevice(&dev) == hipSuccess && a.device == dev;
    }
    return a.type == hipMemoryTypeHost && a.devicePointer == p;
}
}  // namespace

int32_t check_records(const void* aos, const sphv_descriptor* d, int64_t n)
{
    if (n <= 0 || !d || !aos) return SPHV_OK;
    if (d->flags & SPHV_DESC_RECORD_POINTERS) {
        // the address list (the records it names are the caller's)
        const char* b = (const char*)aos;
        return device_addressable(b) && device_addressable(b + 8 * (uint64_t)n - 1) ? SPHV_OK : SPHV_E_INVALID_ARG;
    }
    uint64_t end = 0;
    for (uint32_t k = 0; k < d->n_fields; ++k) {
        const uint64_t e = d->fields[k].offset + (uint64_t)(n - 1) * d->stride + dtype_size(d->fields[k].dtype);
        end = e > end ? e : end;
    }
    const char* b = (const char*)aos;
    return device_addressable(b) && (end == 0 || device_addressable(b + end - 1)) ? SPHV_OK : SPHV_E_INVALID_ARG;
}

CellsDev* cells_dev(sphv_cells* c) { return &c->dev; }
bool cells_sorted(const sphv_cells* c) { return c->sorted; }
void cells_set_sorted(sphv_cells* c, bool sorted) { c->sorted = sorted; }
}  // namespace sphv
