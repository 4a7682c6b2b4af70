// View conversions and the linear kick/drift loop.
//
// gather  (prologue, N o C of the paper's eq. "view"): view[p].f = record[index[p]].f
//         for every member f in A_in; f64 members are bit copies (NaN payloads
//         kept), or, in an FP32 view, rounded to float (positions relative to
//         the lower corner of their cell).
// scatter (epilogue, C^T o W): record[index[p]].f = view[p].f for f in A_out only.
// kick_drift: per record, every product and sum rounded on its own.
#include <algorithm>

#include "k_common.h"

namespace sphv {

namespace {

struct FieldPack {
    FieldRef src[kMaxFields];
    FieldRef dst[kMaxFields];
};

constexpr int kConvThreads = 256;

// one thread per view element p; the record's members come from one record span
__global__ __launch_bounds__(kConvThreads) void k_gather(FieldPack fp, int nf, Access sa, Access da,
                                                         const int32_t* cell_key, Geom g, int64_t n)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    Loc<true> ls = locate<true>(sa, p);
    Loc<false> ld = locate<false>(da, p);
    int key = cell_key ? cell_key[sa.index ? sa.index[p] : p] : 0;
    for (int k = 0; k < nf; ++k) {
        const FieldRef& s = fp.src[k];
        const FieldRef& d = fp.dst[k];
        if (s.size == 8 && d.size == 8) {
            *(uint64_t*)ld.at(d) = *(const uint64_t*)ls.at(s);
        } else if (s.size == 4 && d.size == 4) {
            *(uint32_t*)ld.at(d) = *(const uint32_t*)ls.at(s);
        } else {
            // f64 member narrowed to float (FP32 view); d carries rel_axis
            FieldRef q = s;
            q.rel_axis = d.rel_axis;
            *(float*)ld.at(d) = ld_as_f32(q, ls, g, key);
        }
    }
}

// Scatter with one lane per (element, member): the lanes of a wave store the
// written members of a few records side by side, so a store instruction
// touches a few cache lines of those records instead of one line per lane.
__global__ __launch_bounds__(kConvThreads) void k_scatter_lanes(FieldPack fp, int nf, Access sa, Access da,
                                                                int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n * nf) return;
    const int64_t p = q / nf;
    const int k = (int)(q - p * nf);
    const Loc<false> ls = locate<false>(sa, p);
    const Loc<true> ld = locate<true>(da, p);
    const FieldRef s = fp.src[k];
    const FieldRef d = fp.dst[k];
    if (d.size == 8) *(uint64_t*)ld.at(d) = *(const uint64_t*)ls.at(s);
    else *(uint32_t*)ld.at(d) = *(const uint32_t*)ls.at(s);
}

// k_gather on records staged through LDS (all source members 8 bytes).
__global__ __launch_bounds__(kStageThreads) void k_gather_staged(FieldPack fp, int nf, StagePlan sp, Access sa,
                                                                 Access da, const int32_t* cell_key, Geom g,
                                                                 int64_t n)
{
    extern __shared__ uint4 tile[];
    const int64_t r0 = (int64_t)blockIdx.x * kStageThreads;
    stage_in(tile, fp.src[0].base, sa.stride, sa.index, r0, n, sp);
    const int64_t p = r0 + threadIdx.x;
    if (p >= n) return;
    const LocTile ls{(char*)&tile[threadIdx.x * sp.nch] - (uint64_t)sp.c0 * 16};
    Loc<false> ld = locate<false>(da, p);
    int key = cell_key ? cell_key[sa.index ? sa.index[p] : p] : 0;
    for (int k = 0; k < nf; ++k) {
        const FieldRef& s = fp.src[k];
        const FieldRef& d = fp.dst[k];
        if (d.size == 8) {
            *(uint64_t*)ld.at(d) = *(const uint64_t*)ls.at(s);
        } else {
            FieldRef q = s;
            q.rel_axis = d.rel_axis;
            *(float*)ld.at(d) = ld_as_f32(q, ls, g, key);
        }
    }
}

__global__ __launch_bounds__(kConvThreads) void k_scatter(FieldPack fp, int nf, Access sa, Access da, int64_t n)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    Loc<false> ls = locate<false>(sa, p);
    Loc<true> ld = locate<true>(da, p);
    for (int k = 0; k < nf; ++k) {
        const FieldRef& s = fp.src[k];
        const FieldRef& d = fp.dst[k];
        if (d.size == 8) *(uint64_t*)ld.at(d) = *(const uint64_t*)ls.at(s);
        else *(uint32_t*)ld.at(d) = *(const uint32_t*)ls.at(s);
    }
}

struct KickFields {
    FieldRef f[15];   // x y z vx vy vz vhx vhy vhz ax ay az u uh u_dt
};

// The kick / drift / kick update of one record (every product and sum rounded
// on its own); P(k) addresses member k in the order of KickFields.
template <class Ptr>
__device__ __forceinline__ void kick_one(Ptr&& P, const Geom& g, double dt, double half, double half_prev,
                                         bool first)
{
    for (int d = 0; d < 3; ++d) {
        double a = *P(9 + d);
        double v = *P(3 + d);
        if (!first) v = __dadd_rn(*P(6 + d), __dmul_rn(a, half_prev));     // close the previous step
        double vh = __dadd_rn(v, __dmul_rn(a, half));                       // open this step
        double x = __dadd_rn(*P(d), __dmul_rn(vh, dt));                     // drift
        if (g.periodic[d]) {
            double hi = __dadd_rn(g.lo[d], g.len[d]);
            if (x >= hi) x = __dsub_rn(x, g.len[d]);
            else if (x < g.lo[d]) x = __dadd_rn(x, g.len[d]);
        }
        *P(d) = x;
        *P(6 + d) = vh;
        *P(3 + d) = __dadd_rn(vh, __dmul_rn(a, half));                      // predict
    }
    double du = *P(14);
    double u = *P(12);
    if (!first) u = __dadd_rn(*P(13), __dmul_rn(du, half_prev));
    double uh = __dadd_rn(u, __dmul_rn(du, half));
    *P(13) = uh;
    *P(12) = __dadd_rn(uh, __dmul_rn(du, half));
}

__global__ __launch_bounds__(kConvThreads) void k_kick_drift(KickFields kf, uint64_t stride, const uint64_t* ptrs,
                                                             Geom g, const DevState* st, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double dt = st->dt;
    const uint64_t rb = ptrs ? ptrs[i] : (uint64_t)i * stride;
    auto P = [&](int k) -> double* { return (double*)((uintptr_t)kf.f[k].base + kf.f[k].off + rb); };
    kick_one(P, g, dt, __dmul_rn(0.5, dt), __dmul_rn(0.5, st->dt_prev), st->nstep <= 1);
}

// The kick on records staged through LDS (stage_in / stage_out).
__global__ __launch_bounds__(kStageThreads) void k_kick_staged(KickFields kf, StagePlan sp, uint64_t stride, Geom g,
                                                               const DevState* st, int64_t n)
{
    extern __shared__ uint4 tile[];   // kStageThreads records x nch chunks
    const int64_t r0 = (int64_t)blockIdx.x * kStageThreads;
    char* const base = kf.f[0].base;
    const int nch = (int)sp.nch;
    stage_in(tile, base, stride, nullptr, r0, n, sp);
    const int64_t i = r0 + threadIdx.x;
    if (i < n) {
        char* const mine = (char*)&tile[threadIdx.x * nch] - (uint64_t)sp.c0 * 16;
        auto P = [&](int k) -> double* { return (double*)(mine + kf.f[k].off); };
        const double dt = st->dt;
        kick_one(P, g, dt, __dmul_rn(0.5, dt), __dmul_rn(0.5, st->dt_prev), st->nstep <= 1);
        for (uint32_t m = sp.direct; m; m &= m - 1) {
            const int k = __builtin_ctz(m);
            *(double*)(base + kf.f[k].off + (uint64_t)i * stride) = *P(k);
        }
    }
    stage_out(tile, base, stride, nullptr, r0, n, sp);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kConvThreads - 1) / kConvThreads); }

// Whole-record move: record (didx ? didx[p] : p) of dst = record (sidx ? sidx[p]
// : p) of src, as wpr words of W.  Consecutive threads take consecutive words
// of one record, so each record is one contiguous read and one contiguous
// write; a grid-stride loop covers n * wpr words.
template <typename W>
__global__ __launch_bounds__(kConvThreads) void k_rec_move(const W* __restrict__ src, W* __restrict__ dst,
                                                           const int32_t* sidx, const int32_t* didx,
                                                           uint32_t wpr, int64_t n)
{
    const int64_t total = n * (int64_t)wpr;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += step) {
        const int64_t p = t / wpr;
        const int64_t w = t - p * wpr;
        const int64_t rs = sidx ? (int64_t)sidx[p] : p;
        const int64_t rd = didx ? (int64_t)didx[p] : p;
        dst[rd * wpr + w] = src[rs * wpr + w];
    }
}

// After the records were moved into sorted order: perm is the identity and the
// key of record p is the cell of sorted position p.
__global__ __launch_bounds__(kConvThreads) void k_sorted_index(int32_t* perm, int32_t* key,
                                                               const int32_t* key_sorted, int64_t n)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    perm[p] = (int32_t)p;
    key[p] = key_sorted[p];
}

template <typename W>
hipError_t rec_move_as(const void* src, void* dst, const int32_t* sidx, const int32_t* didx, uint32_t stride,
                       int64_t n, hipStream_t s)
{
    const uint32_t wpr = stride / (uint32_t)sizeof(W);
    const int64_t total = n * (int64_t)wpr;
    const int64_t blocks = std::min<int64_t>((total + kConvThreads - 1) / kConvThreads, 1 << 20);
    hipLaunchKernelGGL(k_rec_move<W>, dim3((unsigned)blocks), dim3(kConvThreads), 0, s, (const W*)src, (W*)dst,
                       sidx, didx, wpr, n);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_rec_move(const void* src, void* dst, const int32_t* sidx, const int32_t* didx, uint32_t stride,
                           int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const uintptr_t al = (uintptr_t)src | (uintptr_t)dst | stride;
    if (al % 16 == 0) return rec_move_as<uint4>(src, dst, sidx, didx, stride, n, s);
    if (al % 8 == 0) return rec_move_as<uint2>(src, dst, sidx, didx, stride, n, s);
    return rec_move_as<uint32_t>(src, dst, sidx, didx, stride, n, s);
}

hipError_t launch_sorted_index(int32_t* perm, int32_t* key, const int32_t* key_sorted, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sorted_index, dim3(nblk(n)), dim3(kConvThreads), 0, s, perm, key, key_sorted, n);
    return hipGetLastError();
}

hipError_t launch_gather(const FieldRef* src, const FieldRef* dst, int nf, const Access& sa, const Access& da,
                         const int32_t* cell_key, const Geom& g, int64_t n, hipStream_t s)
{
    FieldPack fp;
    for (int k = 0; k < nf; ++k) {
        fp.src[k] = src[k];
        fp.dst[k] = dst[k];
    }
    StagePlan sp;
    if (n > 0 && nf > 0 && !sa.ptrs && plan_stage(fp.src, nf, 0u, sa.stride, &sp))
        hipLaunchKernelGGL(k_gather_staged, dim3((unsigned)((n + kStageThreads - 1) / kStageThreads)),
                           dim3(kStageThreads), kStageThreads * sp.nch * 16, s, fp, nf, sp, sa, da, cell_key, g, n);
    else
        hipLaunchKernelGGL(k_gather, dim3(nblk(n)), dim3(kConvThreads), 0, s, fp, nf, sa, da, cell_key, g, n);
    return hipGetLastError();
}

hipError_t launch_scatter(const FieldRef* src, const FieldRef* dst, int nf, const Access& sa, const Access& da,
                          int64_t n, hipStream_t s)
{
    FieldPack fp;
    for (int k = 0; k < nf; ++k) {
        fp.src[k] = src[k];
        fp.dst[k] = dst[k];
    }
    if (nf > 1)
        hipLaunchKernelGGL(k_scatter_lanes, dim3(nblk(n * nf)), dim3(kConvThreads), 0, s, fp, nf, sa, da, n);
    else
        hipLaunchKernelGGL(k_scatter, dim3(nblk(n)), dim3(kConvThreads), 0, s, fp, nf, sa, da, n);
    return hipGetLastError();
}

hipError_t launch_kick_drift(const FieldRef* f, const Access& rec, const Geom& g, const DevState* st, int64_t n,
                             hipStream_t s)
{
    KickFields kf;
    for (int k = 0; k < 15; ++k) kf.f[k] = f[k];
    // written: x y z vx vy vz vhx vhy vhz u uh (members 0-8, 12, 13)
    StagePlan sp;
    if (n > 0 && !rec.index && !rec.ptrs && plan_stage(kf.f, 15, 0x31FFu, rec.stride, &sp)) {
        const unsigned blocks = (unsigned)((n + kStageThreads - 1) / kStageThreads);
        hipLaunchKernelGGL(k_kick_staged, dim3(blocks), dim3(kStageThreads), kStageThreads * sp.nch * 16, s, kf, sp,
                           rec.stride, g, st, n);
    } else {
        hipLaunchKernelGGL(k_kick_drift, dim3(nblk(n)), dim3(kConvThreads), 0, s, kf, rec.stride, rec.ptrs, g, st,
                           n);
    }
    return hipGetLastError();
}

}  // namespace sphv
