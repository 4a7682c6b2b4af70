// Device helpers shared by the HIP kernels of libsphview.so (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace sphv {

// Locator of element p: a record byte offset (direct) or a block/slot pair (view).
template <bool DIRECT>
struct Loc;

template <>
struct Loc<false> {
    uint64_t blk, in;
    __device__ __forceinline__ char* at(const FieldRef& f) const { return f.base + f.off + blk + in * f.size; }
};

template <>
struct Loc<true> {
    uint64_t rb;   // record byte offset from the members' base, or the record's address (base null)
    __device__ __forceinline__ char* at(const FieldRef& f) const
    {
        return (char*)((uintptr_t)f.base + f.off + rb);
    }
};

template <bool DIRECT>
__device__ __forceinline__ Loc<DIRECT> locate(const Access& a, int64_t p);

template <>
__device__ __forceinline__ Loc<false> locate<false>(const Access& a, int64_t p)
{
    Loc<false> l;
    l.blk = (a.lw >= 63 ? 0ull : ((uint64_t)p >> a.lw) * a.block_bytes);
    l.in = (uint64_t)p & a.mask;
    return l;
}

template <>
__device__ __forceinline__ Loc<true> locate<true>(const Access& a, int64_t p)
{
    Loc<true> l;
    int64_t r = a.index ? (int64_t)a.index[p] : p;
    l.rb = a.ptrs ? a.ptrs[r] : (uint64_t)r * a.stride;
    return l;
}

template <class L>
__device__ __forceinline__ double ld_f64(const FieldRef& f, const L& l)
{
    return *(const double*)l.at(f);
}

template <class L>
__device__ __forceinline__ void st_f64(const FieldRef& f, const L& l, double v)
{
    *(double*)l.at(f) = v;
}

// A member read as float: a float member as stored, a double member rounded
// to nearest even; cell-relative coordinates use the origin of cell key k.
template <class L>
__device__ __forceinline__ float ld_as_f32(const FieldRef& f, const L& l, const Geom& g, int key)
{
    if (f.dtype == SPHV_F32) return *(const float*)l.at(f);
    double v = *(const double*)l.at(f);
    if (f.rel_axis >= 0) {
        int ax = f.rel_axis;
        int k = ax == 0 ? key % g.n[0] : (ax == 1 ? (key / g.n[0]) % g.n[1] : key / (g.n[0] * g.n[1]));
        double o = __dadd_rn(g.lo[ax], __dmul_rn((double)k, g.cell[ax]));
        return __double2float_rn(__dsub_rn(v, o));
    }
    return __double2float_rn(v);
}

// Decode a linear cell key.
__device__ __forceinline__ void cell_coords(int key, const Geom& g, int& kx, int& ky, int& kz)
{
    kx = key % g.n[0];
    int t = key / g.n[0];
    ky = t % g.n[1];
    kz = t / g.n[1];
}

__device__ __forceinline__ int cell_key(int kx, int ky, int kz, const Geom& g)
{
    return (kz * g.n[1] + ky) * g.n[0] + kx;
}

__device__ __forceinline__ void set_flag(DevState* st, uint32_t bit) { atomicOr(&st->flags, bit); }

// ---- records staged through LDS
//
// A block of kStageThreads threads takes kStageThreads records (consecutive
// from r0, or index[r0 + r]); the 16-byte chunks c0 .. c0+nch-1 of each (the
// byte span of the members a kernel touches) are read with consecutive
// threads on consecutive chunks, so a wave-wide load covers whole cache lines
// of a few records instead of one line per lane.  Thread r then finds its
// record's member at byte offset `off` at (char*)&tile[r * nch] + off - 16 c0.
constexpr int kStageThreads = 128;
constexpr uint32_t kStageMaxChunks = 16;

struct StagePlan {
    uint32_t c0, nch;
    uint32_t store_chunks;    // bit c: chunk c0 + c written back whole
    uint32_t direct;          // bit k: written member k stored on its own
};

// Plan over members f[0..nf) (8-byte members at 8-byte offsets of one base);
// `written` flags the members a kernel writes.  A chunk goes back whole when
// it holds only members (its bytes are read and rewritten, so a member that is
// only read gets its own bits back) and at least one written member; a
// written member in any other chunk is stored on its own.  False when the
// records do not allow staging (alignment, span over 16 chunks).
inline bool plan_stage(const FieldRef* f, int nf, uint32_t written, uint64_t stride, StagePlan* sp)
{
    const uintptr_t base = (uintptr_t)f[0].base;
    if (nf < 1 || nf > 32 || base % 16 || stride % 16) return false;
    uint64_t lo = ~0ull, hi = 0;
    for (int k = 0; k < nf; ++k) {
        if ((uintptr_t)f[k].base != base || f[k].size != 8 || f[k].off % 8) return false;
        lo = f[k].off < lo ? f[k].off : lo;
        hi = f[k].off + 8 > hi ? f[k].off + 8 : hi;
    }
    const uint64_t c0 = lo / 16, c1 = (hi + 15) / 16;
    if (c1 - c0 > kStageMaxChunks || c1 * 16 > stride) return false;
    uint32_t member = 0, wr = 0;   // 8-byte slots counted from byte 16 c0
    for (int k = 0; k < nf; ++k) {
        const uint32_t slot = (uint32_t)(f[k].off / 8 - 2 * c0);
        member |= 1u << slot;
        if ((written >> k) & 1u) wr |= 1u << slot;
    }
    sp->c0 = (uint32_t)c0;
    sp->nch = (uint32_t)(c1 - c0);
    sp->store_chunks = 0;
    for (uint32_t c = 0; c < sp->nch; ++c)
        if (((member >> (2 * c)) & 3u) == 3u && ((wr >> (2 * c)) & 3u)) sp->store_chunks |= 1u << c;
    sp->direct = 0;
    for (int k = 0; k < nf; ++k) {
        const uint32_t c = (uint32_t)(f[k].off / 16 - c0);
        if (((written >> k) & 1u) && !((sp->store_chunks >> c) & 1u)) sp->direct |= 1u << k;
    }
    return true;
}

// Loads the block's records into tile (kStageThreads x nch chunks) and waits
// for the whole block.  Records at or beyond n are skipped.
__device__ __forceinline__ void stage_in(uint4* tile, const char* base, uint64_t stride, const int32_t* index,
                                         int64_t r0, int64_t n, const StagePlan& sp)
{
    const int nch = (int)sp.nch;
    const int total = kStageThreads * nch;
    for (int q = threadIdx.x; q < total; q += kStageThreads) {
        const int r = q / nch;
        if (r0 + r < n) {
            const int64_t rec = index ? (int64_t)index[r0 + r] : r0 + r;
            tile[q] = *(const uint4*)(base + (uint64_t)rec * stride + (uint64_t)(sp.c0 + (q - r * nch)) * 16);
        }
    }
    __syncthreads();
}

// Waits for the whole block, then writes back the chunks the plan stores whole.
__device__ __forceinline__ void stage_out(const uint4* tile, char* base, uint64_t stride, const int32_t* index,
                                          int64_t r0, int64_t n, const StagePlan& sp)
{
    __syncthreads();
    const int nch = (int)sp.nch;
    const int total = kStageThreads * nch;
    for (int q = threadIdx.x; q < total; q += kStageThreads) {
        const int r = q / nch;
        const int c = q - r * nch;
        if (((sp.store_chunks >> c) & 1u) && r0 + r < n) {
            const int64_t rec = index ? (int64_t)index[r0 + r] : r0 + r;
            *(uint4*)(base + (uint64_t)rec * stride + (uint64_t)(sp.c0 + c) * 16) = tile[q];
        }
    }
}

// Locator of a member inside a staged record.
struct LocTile {
    char* p;   // the record's tile row minus 16 c0 bytes
    __device__ __forceinline__ char* at(const FieldRef& f) const { return p + f.off; }
};

// ---- runs of equal keys in consecutive lanes of a wave
//
// For a wave-wide key, the lane index of the first lane of this lane's run
// (a run is a maximal stretch of consecutive lanes with one key; `valid`
// false lanes form runs of their own).
__device__ __forceinline__ int run_head(int key, bool valid)
{
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int prev = __shfl_up(key, 1, kWave);
    const int pv = __shfl_up(valid ? 1 : 0, 1, kWave);
    const bool head = lane == 0 || !valid || !pv || prev != key;
    const uint64_t heads = __ballot(head) & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
    return 63 - __builtin_clzll(heads);
}

// True on the last lane of this lane's run.
__device__ __forceinline__ bool run_tail(int key, bool valid)
{
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int next = __shfl_down(key, 1, kWave);
    const int nv = __shfl_down(valid ? 1 : 0, 1, kWave);
    return lane == kWave - 1 || !valid || !nv || next != key;
}

// Largest v over the lanes of this lane's run up to this lane.
__device__ __forceinline__ uint32_t run_max_upto(uint32_t v, int head)
{
    const int lane = (int)(threadIdx.x & (kWave - 1));
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t o = __shfl_up(v, off, kWave);
        if (lane - off >= head) v = o > v ? o : v;
    }
    return v;
}

}  // namespace sphv
