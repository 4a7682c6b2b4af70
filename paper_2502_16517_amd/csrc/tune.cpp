// Autotuner of the batching layer: picks, per pair loop, the view layout
// (records directly, SoA, AoSoA of width 8..64) and the tile shape (lanes per
// local particle, masked or branching predicate) by timing each candidate on
// the caller's own records and cells.
//
// One trial is the span the view method adds up to for that loop: gather of
// A_in, the loop, scatter of A_out (the paper's prologue, converted loop and
// epilogue, Sec. 3.1), timed with HIP events on the caller's stream.  Trials
// must not change the data the next trial starts from, so every member the
// descriptor names is copied out of the records once, bit for bit, before the
// first trial and copied back after each one; the records leave the call as
// they came in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using namespace sphv;

namespace {

constexpr uint64_t kAlignT = 256;
constexpr int kMaxCand = 64;

uint64_t up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

uint32_t size_of(uint32_t dt) { return (dt == SPHV_F64 || dt == SPHV_I64) ? 8u : 4u; }

// Default candidates: every layout kind x lanes per particle {auto, 1, 2, 4, 8}
// x {branching, masked}.
int default_candidates(sphv_layout* out, int cap)
{
    const uint32_t kinds[6][2] = {{SPHV_LAYOUT_SOA, 0},    {SPHV_LAYOUT_AOSOA, 8},  {SPHV_LAYOUT_AOSOA, 16},
                                  {SPHV_LAYOUT_AOSOA, 32}, {SPHV_LAYOUT_AOSOA, 64}, {SPHV_LAYOUT_DIRECT, 0}};
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
    return (size_t)(up(sizeof(sphv_state), kAlignT) + backup_bytes(d, n) + up(view, kAlignT));
}

int32_t sphv_autotune(int32_t loop, void* aos, const sphv_descriptor* d, const sphv_cells* cells,
                      const sphv_params* p, int32_t precision, const sphv_layout* cand, int32_t n_cand,
                      int32_t reps, void* ws, size_t ws_bytes, sphv_layout* best, float* ms_out, void* stream)
{
    if (loop != SPHV_LOOP_DENSITY && loop != SPHV_LOOP_FORCE) return SPHV_E_INVALID_ARG;
    if (!d || !cells || !p || !best || reps < 1 || reps > 100) return SPHV_E_INVALID_ARG;
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
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) return SPHV_E_HIP;
    if (cap != hipStreamCaptureStatusNone) return SPHV_E_STATE;   // it times on the host

    char* base = (char*)ws;
    void* state = base;
    char* bk = base + up(sizeof(sphv_state), kAlignT);
    char* vws = bk + backup_bytes(d, n);
    const size_t vbytes = ws_bytes - (size_t)(vws - base);

    Backup b;
    plan_backup(&b, (char*)aos, d, n, bk);
    if (n > 0 && save(b, s) != hipSuccess) return SPHV_E_HIP;

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return SPHV_E_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SPHV_E_HIP;
    }
    int32_t status = SPHV_OK;
    float best_ms = 0.f;
    int best_k = -1;
    std::vector<float> trial((size_t)reps);
    for (int k = 0; k < n_cand && status == SPHV_OK; ++k) {
        sphv_view* v = nullptr;
        status = sphv_view_create(&v, d, n, &cand[k], precision, aos, (const int32_t*)info.perm, vws, vbytes);
        if (status) break;
        for (int r = 0; r < reps && status == SPHV_OK; ++r) {
            status = sphv_state_init(state, stream);
            if (!status && hipEventRecord(e0, s) != hipSuccess) status = SPHV_E_HIP;
            if (!status) status = sphv_aos_to_soa(v, cells, stream);
            if (!status) status = loop == SPHV_LOOP_DENSITY ? sphv_sph_density(v, cells, p, state, stream)
                                                            : sphv_sph_force(v, cells, p, state, stream);
            if (!status) status = sphv_soa_to_aos(v, stream);
            if (!status && hipEventRecord(e1, s) != hipSuccess) status = SPHV_E_HIP;
            if (!status && n > 0 && restore(b, s) != hipSuccess) status = SPHV_E_HIP;
            if (!status && hipEventSynchronize(e1) != hipSuccess) status = SPHV_E_HIP;
            if (!status && hipEventElapsedTime(&trial[(size_t)r], e0, e1) != hipSuccess) status = SPHV_E_HIP;
        }
        sphv_view_destroy(v);   // also closes it when a call failed half way
        if (status) break;
        std::sort(trial.begin(), trial.end());
        const float med = trial[(size_t)reps / 2];
        if (ms_out) ms_out[k] = med;
        if (best_k < 0 || med < best_ms) {
            best_ms = med;
            best_k = k;
        }
    }
    // the records as they came in, whatever happened above
    if (n > 0 && restore(b, s) != hipSuccess && status == SPHV_OK) status = SPHV_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess && status == SPHV_OK) status = SPHV_E_HIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status == SPHV_OK) *best = cand[best_k];
    return status;
}

}  // extern "C"
