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
    uint64_t rb;
    __device__ __forceinline__ char* at(const FieldRef& f) const { return f.base + f.off + rb; }
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
    l.rb = (uint64_t)r * a.stride;
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

}  // namespace sphv
