// Autotuner of the batching layer: picks, per pair loop, the view layout
// (records directly, records stored cell by cell, SoA, AoSoA of width 8..64)
// and the tile shape (lanes per local particle, masked or branching predicate)
// by timing each candidate on the caller's own records and cells; and, for the
// whole density + force pair, the grid (cells per support length).
//
// One trial is the span the view method adds up to for that loop: gather of
// A_in, the loop, scatter of A_out (the paper's prologue, converted loop and
// epilogue, Sec. 3.1), timed with HIP events on the caller's stream.  Trials
// must not change the data the next trial starts from, so every member the
// descriptor names is copied out of the records once, bit for bit, before the
// first trial and copied back after each one; the records leave the call as
// they came in.  A trial on records stored cell by cell includes the move into
// that order (the price of the layout); afterwards the records, the cells' perm
// and key are moved back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using namespace sphv;

namespace {

constexpr uint64_t kAlignT = 256;
constexpr int kMaxCand = 128;
constexpr int kMaxGrids = 16;
constexpr double kGridHeadroom = 1.1;   // cell edge over the support it is sized for
// Candidates whose medians lie within this fraction of the fastest are taken
// as equal (run-to-run timing noise); the first of them in the caller's order
// is chosen, so repeated tuning returns the same choice.
constexpr float kTieMul = 1.015f;

int pick(const std::vector<float>& med)
{
    float lo = med[0];
    for (float m : med) lo = std::min(lo, m);
    for (size_t k = 0; k < med.size(); ++k)
        if (med[k] <= lo * kTieMul) return (int)k;
    return 0;
}

uint64_t up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

uint32_t size_of(uint32_t dt) { return (dt == SPHV_F64 || dt == SPHV_I64) ? 8u : 4u; }

// Default candidates: every layout kind x lanes per particle {auto, 1, 2, 4, 8}
// x {branching, masked}.
int default_candidates(sphv_layout* out, int cap)
{
    const uint32_t kinds[7][2] = {{SPHV_LAYOUT_SOA, 0},      {SPHV_LAYOUT_AOSOA, 8},  {SPHV_LAYOUT_AOSOA, 16},
                                  {SPHV_LAYOUT_AOSOA, 32},   {SPHV_LAYOUT_AOSOA, 64}, {SPHV_LAYOUT_DIRECT, 0},
                                  {SPHV_LAYOUT_SORTED, 0}};
    const uint32_t tpis[5] = {0, 1, 2, 4, 8};
    int k = 0;
    for (const auto& kd : kinds)
        for (uint32_t t : tpis)
            for (uint32_t m = 0; m < 2; ++m) {
                if (k < cap && out) out[k] = sphv_layout{kd[0], kd[1], t, m};
                ++k;
            }
    return k;
}

// Bytes of the bit copy of every member the descriptor names (SoA, one array
// per member).
uint64_t backup_bytes(const sphv_descriptor* d, int64_t n)
{
    uint64_t b = 0;
    for (uint32_t k = 0; k < d->n_fields; ++k) b = up(b + (uint64_t)std::max<int64_t>(n, 1) * size_of(d->fields[k].dtype), kAlignT);
    return b;
}

struct Backup {
    FieldRef rec[kMaxFields], copy[kMaxFields];
    Access ra{}, ca{};
    int nf = 0;
    int64_t n = 0;
};

void plan_backup(Backup* b, char* aos, const sphv_descriptor* d, int64_t n, char* ws)
{
    uint64_t off = 0;
    b->nf = (int)d->n_fields;
    b->n = n;
    for (uint32_t k = 0; k < d->n_fields; ++k) {
        const sphv_field& f = d->fields[k];
        b->rec[k] = FieldRef{aos, f.offset, size_of(f.dtype), f.dtype, -1, 0};
        b->copy[k] = FieldRef{ws, off, size_of(f.dtype), f.dtype, -1, 0};
        off = up(off + (uint64_t)std::max<int64_t>(n, 1) * size_of(f.dtype), kAlignT);
    }
    // records in index order 0..n-1; the copy is plain SoA
    b->ra.lw = 0;
    b->ra.index = nullptr;
    b->ra.stride = d->stride;
    b->ca.lw = 63;
    b->ca.mask = ~0ull;
}

hipError_t save(const Backup& b, hipStream_t s)
{
    Geom g{};
    return launch_gather(b.rec, b.copy, b.nf, b.ra, b.ca, nullptr, g, b.n, s);
}

hipError_t restore(const Backup& b, hipStream_t s)
{
    return launch_scatter(b.copy, b.rec, b.nf, b.ca, b.ra, b.n, s);
}

bool any_sorted(const sphv_layout* cand, int n_cand)
{
    for (int k = 0; k < n_cand; ++k)
        if (cand[k].kind == SPHV_LAYOUT_SORTED) return true;
    return false;
}

// Scratch of the trials on records stored cell by cell: the sorted copy of the
// records, and the cells' perm and key as they were.
uint64_t sort_bytes(uint32_t stride, int64_t n)
{
    return up(sphv_records_sort_workspace_bytes(stride, n), kAlignT) + 2 * up(4 * (uint64_t)std::max<int64_t>(n, 1), kAlignT);
}

struct SortSave {
    char* recs = nullptr;     // sphv_records_sort scratch, then the unsort staging
    size_t rec_bytes = 0;
    int32_t* perm = nullptr;  // the cells' perm and key before the first trial
    int32_t* key = nullptr;
};

SortSave plan_sort(char* ws, uint32_t stride, int64_t n)
{
    SortSave ss;
    ss.recs = ws;
    ss.rec_bytes = up(sphv_records_sort_workspace_bytes(stride, n), kAlignT);
    ss.perm = (int32_t*)(ws + ss.rec_bytes);
    ss.key = (int32_t*)(ws + ss.rec_bytes + up(4 * (uint64_t)std::max<int64_t>(n, 1), kAlignT));
    return ss;
}

hipError_t save_index(const SortSave& ss, const CellsDev& c, hipStream_t s)
{
    hipError_t e = launch_rec_move(c.perm, ss.perm, nullptr, nullptr, 4, c.n, s);
    if (e == hipSuccess) e = launch_rec_move(c.key, ss.key, nullptr, nullptr, 4, c.n, s);
    return e;
}

// Undo sphv_records_sort: record perm[p] (the saved perm) gets back the record
// now at p; then the saved perm and key.
hipError_t unsort(const SortSave& ss, const CellsDev& c, void* aos, uint32_t stride, hipStream_t s)
{
    hipError_t e = launch_rec_move(aos, ss.recs, nullptr, nullptr, stride, c.n, s);
    if (e == hipSuccess) e = launch_rec_move(ss.recs, aos, nullptr, ss.perm, stride, c.n, s);
    if (e == hipSuccess) e = launch_rec_move(ss.perm, c.perm, nullptr, nullptr, 4, c.n, s);
    if (e == hipSuccess) e = launch_rec_move(ss.key, c.key, nullptr, nullptr, 4, c.n, s);
    return e;
}

// p with another grid: cell edges and their inverses as sphv_params_init sets them
sphv_params with_grid(const sphv_params* p, const int32_t* grid)
{
    sphv_params q = *p;
    for (int a = 0; a < 3; ++a) {
        q.grid[a] = grid[a];
        q.cell[a] = q.len[a] / (double)grid[a];
        q.inv_cell[a] = (double)grid[a] / q.len[a];
    }
    return q;
}

float median(std::vector<float>& t)
{
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

struct Events {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = false;
    Events()
    {
        ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    }
    ~Events()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

int32_t refuse_capture(hipStream_t s)
{
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) return SPHV_E_HIP;
    return cap != hipStreamCaptureStatusNone ? SPHV_E_STATE : SPHV_OK;   // it times on the host
}

}  // namespace

extern "C" {

int32_t sphv_autotune_candidates(sphv_layout* out, int32_t cap)
{
    return default_candidates(out, out ? cap : 0);
}

size_t sphv_autotune_workspace_bytes(const sphv_descriptor* d, int64_t n, int32_t precision,
                                     const sphv_layout* cand, int32_t n_cand)
{
    if (!d || n < 0 || !d->fields || d->n_fields == 0 || d->n_fields > (uint32_t)kMaxFields) return 0;
    sphv_layout def[kMaxCand];
    if (!cand) {
        n_cand = default_candidates(def, kMaxCand);
        cand = def;
    }
    if (n_cand <= 0 || n_cand > kMaxCand) return 0;
    uint64_t view = 0;
    for (int k = 0; k < n_cand; ++k) {
        size_t b = sphv_view_workspace_bytes(d, n, &cand[k], precision);
        if (!b) return 0;
        view = std::max<uint64_t>(view, b);
    }
    uint64_t total = up(sizeof(sphv_state), kAlignT) + backup_bytes(d, n) + up(view, kAlignT);
    if (any_sorted(cand, n_cand)) {
        if (!sphv_records_sort_workspace_bytes(d->stride, n)) return 0;
        total += sort_bytes(d->stride, n);
    }
    return (size_t)total;
}

int32_t sphv_autotune(int32_t loop, void* aos, const sphv_descriptor* d, const sphv_cells* cells,
                      const sphv_params* p, int32_t precision, const sphv_layout* cand, int32_t n_cand,
                      int32_t reps, void* ws, size_t ws_bytes, sphv_layout* best, float* ms_out, void* stream)
{
    if (loop != SPHV_LOOP_DENSITY && loop != SPHV_LOOP_FORCE) return SPHV_E_INVALID_ARG;
    if (!d || !cells || !p || !best || reps < 1 || reps > 100) return SPHV_E_INVALID_ARG;
    if (d->flags & SPHV_DESC_RECORD_POINTERS) return SPHV_E_UNSUPPORTED;
    sphv_cells_info info;
    int32_t st = sphv_cells_get_info(cells, &info);
    if (st) return st;
    const int64_t n = info.n;
    if (n > 0 && !aos) return SPHV_E_INVALID_ARG;
    sphv_layout def[kMaxCand];
    if (!cand) {
        n_cand = default_candidates(def, kMaxCand);
        cand = def;
    }
    if (n_cand <= 0 || n_cand > kMaxCand) return SPHV_E_INVALID_ARG;
    const size_t need_b = sphv_autotune_workspace_bytes(d, n, precision, cand, n_cand);
    if (!need_b) return SPHV_E_INVALID_ARG;
    if (!ws || (uintptr_t)ws % kAlignT || ws_bytes < need_b) return SPHV_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (int32_t c = refuse_capture(s)) return c;
    if ((st = check_records(aos, d, n))) return st;

    // trials on sorted records move them, and the cells' perm and key, and put
    // all of it back before the next trial
    sphv_cells* mc = const_cast<sphv_cells*>(cells);
    const bool sorted_in = cells_sorted(cells);
    const bool with_sort = any_sorted(cand, n_cand);

    char* base = (char*)ws;
    void* state = base;
    char* bk = base + up(sizeof(sphv_state), kAlignT);
    char* sws = bk + backup_bytes(d, n);
    const SortSave ss = plan_sort(sws, d->stride, n);
    char* vws = sws + (with_sort ? sort_bytes(d->stride, n) : 0);
    const size_t vbytes = ws_bytes - (size_t)(vws - base);

    Backup b;
    plan_backup(&b, (char*)aos, d, n, bk);
    if (n > 0 && save(b, s) != hipSuccess) return SPHV_E_HIP;
    if (with_sort && n > 0 && save_index(ss, *cells_dev(mc), s) != hipSuccess) return SPHV_E_HIP;

    Events ev;
    if (!ev.ok) return SPHV_E_HIP;
    int32_t status = SPHV_OK;
    // rounds over all candidates, reps times, so that a slow drift of the
    // clocks during the call touches every candidate alike
    std::vector<float> times((size_t)n_cand * (size_t)reps);
    for (int r = 0; r < reps && status == SPHV_OK; ++r) {
        for (int k = 0; k < n_cand && status == SPHV_OK; ++k) {
            const bool srt = cand[k].kind == SPHV_LAYOUT_SORTED;
            sphv_view* v = nullptr;
            status = sphv_view_create(&v, d, n, &cand[k], precision, aos, (const int32_t*)info.perm, vws, vbytes);
            if (status) break;
            bool moved = false;   // the records were moved into cell order by this trial
            status = sphv_state_init(state, stream);
            if (!status && hipEventRecord(ev.e0, s) != hipSuccess) status = SPHV_E_HIP;
            if (!status && srt) {
                status = sphv_records_sort(mc, aos, d->stride, ss.recs, ss.rec_bytes, stream);
                moved = status == SPHV_OK;
            }
            if (!status) status = sphv_aos_to_soa(v, cells, stream);
            if (!status) status = loop == SPHV_LOOP_DENSITY ? sphv_sph_density(v, cells, p, state, stream)
                                                            : sphv_sph_force(v, cells, p, state, stream);
            if (!status) status = sphv_soa_to_aos(v, stream);
            if (!status && hipEventRecord(ev.e1, s) != hipSuccess) status = SPHV_E_HIP;
            if (moved && n > 0 && unsort(ss, *cells_dev(mc), aos, d->stride, s) != hipSuccess && !status)
                status = SPHV_E_HIP;
            cells_set_sorted(mc, sorted_in);
            if (!status && n > 0 && restore(b, s) != hipSuccess) status = SPHV_E_HIP;
            if (!status && hipEventSynchronize(ev.e1) != hipSuccess) status = SPHV_E_HIP;
            float ms = 0.f;
            if (!status && hipEventElapsedTime(&ms, ev.e0, ev.e1) != hipSuccess) status = SPHV_E_HIP;
            times[(size_t)k * reps + r] = ms;
            sphv_view_destroy(v);   // also closes it when a call failed half way
        }
    }
    std::vector<float> meds;
    if (status == SPHV_OK) {
        std::vector<float> trial((size_t)reps);
        for (int k = 0; k < n_cand; ++k) {
            for (int r = 0; r < reps; ++r) trial[(size_t)r] = times[(size_t)k * reps + r];
            const float med = median(trial);
            if (ms_out) ms_out[k] = med;
            meds.push_back(med);
        }
    }
    // the records as they came in, whatever happened above
    if (n > 0 && restore(b, s) != hipSuccess && status == SPHV_OK) status = SPHV_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess && status == SPHV_OK) status = SPHV_E_HIP;
    if (status == SPHV_OK) *best = cand[pick(meds)];
    return status;
}

int32_t sphv_grid_for(const sphv_params* p, double h_ref, int32_t cells_per_support, int32_t* grid)
{
    if (!p || !grid || !(h_ref > 0.0) || !std::isfinite(h_ref) || cells_per_support < 1 || cells_per_support > 4)
        return SPHV_E_INVALID_ARG;
    for (int a = 0; a < 3; ++a) {
        if (!(p->len[a] > 0.0) || !std::isfinite(p->len[a])) return SPHV_E_INVALID_ARG;
        // one cell spans 2 h_ref / cells_per_support, times a 10 % headroom
        const double cells = std::floor(p->len[a] * cells_per_support / (2.0 * h_ref * kGridHeadroom));
        const double lo = p->periodic[a] ? 3.0 : 1.0;
        const double g = std::max(cells, lo);
        if (g > 4096.0) return SPHV_E_UNSUPPORTED;
        grid[a] = (int32_t)g;
    }
    return SPHV_OK;
}

size_t sphv_autotune_grid_workspace_bytes(const sphv_descriptor* d_density, const sphv_descriptor* d_force,
                                          int64_t n, const sphv_params* p, int32_t precision,
                                          const sphv_layout* l_density, const sphv_layout* l_force,
                                          const int32_t* grids, int32_t n_grids)
{
    if (!d_density || !d_force || !p || !l_density || !l_force || !grids || n < 0) return 0;
    if (n_grids < 1 || n_grids > kMaxGrids) return 0;
    if (!d_density->fields || !d_force->fields || d_density->n_fields == 0 || d_force->n_fields == 0 ||
        d_density->n_fields > (uint32_t)kMaxFields || d_force->n_fields > (uint32_t)kMaxFields)
        return 0;
    uint64_t cells = 0;
    for (int g = 0; g < n_grids; ++g) {
        for (int a = 0; a < 3; ++a)
            if (grids[3 * g + a] < 1) return 0;
        const sphv_params pg = with_grid(p, grids + 3 * g);
        const size_t b = sphv_cells_workspace_bytes(n, &pg);
        if (!b) return 0;
        cells = std::max<uint64_t>(cells, b);
    }
    const size_t vd = sphv_view_workspace_bytes(d_density, n, l_density, precision);
    const size_t vf = sphv_view_workspace_bytes(d_force, n, l_force, precision);
    if (!vd || !vf) return 0;
    return (size_t)(up(sizeof(sphv_state), kAlignT) + backup_bytes(d_density, n) + backup_bytes(d_force, n) +
                    up(cells, kAlignT) + up(vd, kAlignT) + up(vf, kAlignT));
}

int32_t sphv_autotune_grid(void* aos, const sphv_descriptor* d_density, const sphv_descriptor* d_force, int64_t n,
                           const sphv_params* p, int32_t precision, const sphv_layout* l_density,
                           const sphv_layout* l_force, const int32_t* grids, int32_t n_grids, int32_t reps,
                           void* ws, size_t ws_bytes, int32_t* best, float* ms_out, void* stream)
{
    if (!d_density || !d_force || !p || !l_density || !l_force || !grids || !best || n < 0) return SPHV_E_INVALID_ARG;
    if (reps < 1 || reps > 100 || n_grids < 1 || n_grids > kMaxGrids) return SPHV_E_INVALID_ARG;
    if ((d_density->flags | d_force->flags) & SPHV_DESC_RECORD_POINTERS) return SPHV_E_UNSUPPORTED;
    if (n > 0 && !aos) return SPHV_E_INVALID_ARG;
    if (l_density->kind == SPHV_LAYOUT_SORTED || l_force->kind == SPHV_LAYOUT_SORTED) return SPHV_E_UNSUPPORTED;
    const size_t need_b = sphv_autotune_grid_workspace_bytes(d_density, d_force, n, p, precision, l_density,
                                                             l_force, grids, n_grids);
    if (!need_b) return SPHV_E_INVALID_ARG;
    if (!ws || (uintptr_t)ws % kAlignT || ws_bytes < need_b) return SPHV_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (int32_t c = refuse_capture(s)) return c;
    if (int32_t r = check_records(aos, d_density, n)) return r;
    if (int32_t r = check_records(aos, d_force, n)) return r;

    char* base = (char*)ws;
    void* state = base;
    char* bkd = base + up(sizeof(sphv_state), kAlignT);
    char* bkf = bkd + backup_bytes(d_density, n);
    char* cws = bkf + backup_bytes(d_force, n);
    uint64_t cells_b = 0;
    for (int g = 0; g < n_grids; ++g) {
        const sphv_params pg = with_grid(p, grids + 3 * g);
        cells_b = std::max<uint64_t>(cells_b, sphv_cells_workspace_bytes(n, &pg));
    }
    char* vwd = cws + up(cells_b, kAlignT);
    const size_t vd_b = sphv_view_workspace_bytes(d_density, n, l_density, precision);
    char* vwf = vwd + up(vd_b, kAlignT);
    const size_t vf_b = ws_bytes - (size_t)(vwf - base);

    Backup bd, bf;
    plan_backup(&bd, (char*)aos, d_density, n, bkd);
    plan_backup(&bf, (char*)aos, d_force, n, bkf);
    if (n > 0 && (save(bd, s) != hipSuccess || save(bf, s) != hipSuccess)) return SPHV_E_HIP;

    Events ev;
    if (!ev.ok) return SPHV_E_HIP;
    int32_t status = SPHV_OK;
    std::vector<float> meds;
    std::vector<float> trial((size_t)reps);
    for (int g = 0; g < n_grids && status == SPHV_OK; ++g) {
        const sphv_params pg = with_grid(p, grids + 3 * g);
        sphv_cells* c = nullptr;
        sphv_view *vd = nullptr, *vf = nullptr;
        status = sphv_cells_create(&c, n, &pg, cws, (size_t)cells_b);
        sphv_cells_info info{};
        if (!status) status = sphv_cells_get_info(c, &info);
        if (!status) status = sphv_view_create(&vd, d_density, n, l_density, precision, aos, info.perm, vwd, vd_b);
        if (!status) status = sphv_view_create(&vf, d_force, n, l_force, precision, aos, info.perm, vwf, vf_b);
        for (int r = 0; r < reps && status == SPHV_OK; ++r) {
            status = sphv_state_init(state, stream);
            if (!status && hipEventRecord(ev.e0, s) != hipSuccess) status = SPHV_E_HIP;
            if (!status) status = sphv_cells_build(c, aos, d_density, state, stream);
            if (!status) status = sphv_aos_to_soa(vd, c, stream);
            if (!status) status = sphv_sph_density(vd, c, &pg, state, stream);
            if (!status) status = sphv_soa_to_aos(vd, stream);
            if (!status) status = sphv_aos_to_soa(vf, c, stream);
            if (!status) status = sphv_sph_force(vf, c, &pg, state, stream);
            if (!status) status = sphv_soa_to_aos(vf, stream);
            if (!status && hipEventRecord(ev.e1, s) != hipSuccess) status = SPHV_E_HIP;
            if (!status && n > 0 && (restore(bf, s) != hipSuccess || restore(bd, s) != hipSuccess))
                status = SPHV_E_HIP;
            if (!status && hipEventSynchronize(ev.e1) != hipSuccess) status = SPHV_E_HIP;
            if (!status && hipEventElapsedTime(&trial[(size_t)r], ev.e0, ev.e1) != hipSuccess) status = SPHV_E_HIP;
        }
        sphv_view_destroy(vf);
        sphv_view_destroy(vd);
        sphv_cells_destroy(c);
        if (status) break;
        const float med = median(trial);
        if (ms_out) ms_out[g] = med;
        meds.push_back(med);
    }
    if (n > 0 && (restore(bf, s) != hipSuccess || restore(bd, s) != hipSuccess) && status == SPHV_OK)
        status = SPHV_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess && status == SPHV_OK) status = SPHV_E_HIP;
    if (status == SPHV_OK) *best = pick(meds);
    return status;
}

}  // extern "C"
