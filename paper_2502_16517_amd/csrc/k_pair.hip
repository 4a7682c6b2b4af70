// Pair loops of the SPH step over a converted view (or directly over the
// records): density with the smoothing-length iteration and the force, plus the
// fixed-order time-step / conservation reduction.
//
// Mapping onto gfx950 (wave64):
//  * One workgroup = one wave.  A persistent grid pulls work items from eight
//    queues, one per XCD (blockIdx % 8 runs on XCD blockIdx % 8), so that the
//    items of one XCD are a contiguous run of cells and share its L2; a wave
//    steals from the other queues when its own is empty.  The last wave to
//    leave resets the queue counters for the next launch.
//  * A work item is one local cell (<= 64 particles; larger cells are split).
//    Its active set is the (2R+1)^3 cells around it (paper Sec. 2.3: local vs
//    active particles); cells along x are contiguous in the sorted order, so
//    every (dy, dz) row is one or (wrapping) two or three contiguous spans.
//  * tpi lanes share one local particle i: lane (i, s) takes the staged
//    candidates s, s + tpi, ...; the tpi partial sums are added in a fixed
//    order.  Candidates are staged 64 at a time in LDS with the periodic image
//    shift applied; every candidate's slot and order depend only on the cell
//    structure, so results are deterministic.
//  * Out-of-range pairs either branch away or contribute the neutral element
//    (paper Sec. 5.6); both orders of evaluation are bit-identical.
//  * FP64: plain double arithmetic, fused only where fma() is written.
//    FP32: positions relative to the local cell's corner, pair arithmetic in
//    float, per-chunk float partial sums folded into Neumaier-compensated
//    float accumulators; Newton step and convergence test in double.
#include <atomic>
#include <type_traits>

#include "k_common.h"

namespace sphv {

namespace {

constexpr double kPi = 3.14159265358979323846;

// head[q * kQStride] counts the items taken from queue q.  A wave drains its
// own queue (q = its XCD), then looks at no more than kStealProbes of the
// others, in an order rotated per wave so that stealers spread over them, and
// stops at the first drained one it finds after those.  Every queue is some
// waves' own, so every item is taken.  Reads and takes of a head serialise at
// the device's point of coherence; bounding the probes keeps the end of a
// launch from queueing thousands of them.
constexpr int kStealProbes = 3;

__device__ int next_item(int32_t* head, int n_items, int xcd, int rot, int& qoff)
{
    while (qoff <= kStealProbes) {
        const int q = qoff == 0 ? xcd : (xcd + 1 + (rot + qoff - 1) % (kNumXcd - 1)) % kNumXcd;
        const int lo = (int)(((int64_t)n_items * q) / kNumXcd);
        const int hi = (int)(((int64_t)n_items * (q + 1)) / kNumXcd);
        if (lo < hi) {
            int32_t* hp = &head[q * kQStride];
            // heads only grow: a queue read as drained is drained
            if (lo + __hip_atomic_load(hp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < hi) {
                const int k = atomicAdd(hp, 1);
                if (lo + k < hi) return lo + k;
            }
        }
        ++qoff;
    }
    return -1;
}

// Lane 0 of every wave leaves its counters in its own slots (plain stores: no
// two waves share a cache line's worth of atomics at the end of the launch).
__device__ __forceinline__ void leave_part(int64_t* part, int64_t c0, int64_t c1, int64_t c2, int64_t c3)
{
    int64_t* p = part + (int64_t)blockIdx.x * kPartSlots;
    p[0] = c0;
    p[1] = c1;
    p[2] = c2;
    p[3] = c3;
}

__device__ __forceinline__ void neumaier(float& s, float& c, float x)
{
    float t = s + x;
    c += (fabsf(s) >= fabsf(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
}

// The smoothing kernels in truncated-power form, branch free; W = w(q)/(pi h^3).
// Cubic M4:
//   w(q)  = (2-q)_+^3 / 4 - (1-q)_+^3      (= 1 - 1.5 q^2 + 0.75 q^3 below 1)
//   w'(q) = 3 (1-q)_+^2 - 0.75 (2-q)_+^2
// Quartic M5 (Sec. 2.1), scaled to the same support 2h (its knots at q = 0.4,
// 1.2, 2), k = 1.25^4 / 10.24 = 15625/65536:
//   w(q)  = k ((2-q)_+^4 - 5 (1.2-q)_+^4 + 10 (0.4-q)_+^4)
//   w'(q) = -4 k ((2-q)_+^3 - 5 (1.2-q)_+^3 + 10 (0.4-q)_+^3)
// All pieces vanish identically for q >= 2, so no select is needed at the
// support edge and the pieces never diverge inside a wave.
template <int KERN, class R>
__device__ __forceinline__ void spline(R q, R& w, R& dw)
{
    const R a = fmax(R(2) - q, R(0));
    if constexpr (KERN == SPHV_KERNEL_QUARTIC) {
        const R b = fmax(R(1.2) - q, R(0));
        const R c = fmax(R(0.4) - q, R(0));
        const R a3 = a * a * a;
        const R b3 = b * b * b;
        const R c3 = c * c * c;
        const R k = R(15625.0 / 65536.0);
        w = k * fma(a3, a, fma(R(-5) * b3, b, R(10) * c3 * c));
        dw = (R(-4) * k) * fma(R(-5), b3, fma(R(10), c3, a3));
    } else {
        const R b = fmax(R(1) - q, R(0));
        const R a2 = a * a;
        const R b2 = b * b;
        w = fma(R(0.25) * a2, a, -(b2 * b));
        dw = fma(R(3), b2, R(-0.75) * a2);
    }
}

template <int KERN, class R>
__device__ __forceinline__ R spline_dw(R q)
{
    const R a = fmax(R(2) - q, R(0));
    if constexpr (KERN == SPHV_KERNEL_QUARTIC) {
        const R b = fmax(R(1.2) - q, R(0));
        const R c = fmax(R(0.4) - q, R(0));
        const R k = R(15625.0 / 65536.0);
        return (R(-4) * k) * fma(R(-5), b * b * b, fma(R(10), c * c * c, a * a * a));
    } else {
        const R b = fmax(R(1) - q, R(0));
        return fma(R(3), b * b, R(-0.75) * (a * a));
    }
}

// 1/sqrt(x) for normal x > 0: the hardware estimate refined by Newton-Raphson
// steps y <- y (3/2 - x y^2 / 2) (two in double, one in float).
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx, y * y, 1.5);
    y = y * fma(-hx, y * y, 1.5);
    return y;
}

__device__ __forceinline__ float rsqrt_nr(float x)
{
    float y = __builtin_amdgcn_rsqf(x);
    const float hx = 0.5f * x;
    return y * fmaf(-hx, y * y, 1.5f);
}

// 1/d: hardware estimate refined by Newton-Raphson steps y <- y + y (1 - d y).
__device__ __forceinline__ double rcp_nr(double d)
{
    double y = __builtin_amdgcn_rcp(d);
    double e = fma(-d, y, 1.0);
    y = fma(y, e, y);
    e = fma(-d, y, 1.0);
    return fma(y, e, y);
}

__device__ __forceinline__ float rcp_nr(float d)
{
    float y = __builtin_amdgcn_rcpf(d);
    return fmaf(y, fmaf(-d, y, 1.0f), y);
}

template <class R> struct Tiny;
template <> struct Tiny<double> { static constexpr double v = 1e-300; };
template <> struct Tiny<float> { static constexpr float v = 1e-30f; };

// Per-axis reach of a work item spanning gx cells along x, guarded against
// windows that wrap onto themselves.
__device__ __forceinline__ void axis_reach(const PairArgs& a, int R, int gx, int r[3])
{
    bool small = false;
    for (int d = 0; d < 3; ++d) {
        const int span = d == 0 ? gx : 1;
        r[d] = R;
        if (a.g.periodic[d] && 2 * R + span > a.g.n[d]) {
            r[d] = (a.g.n[d] - span) / 2;
            small = true;
        }
    }
    if (small && threadIdx.x == 0) set_flag(a.state, SPHV_F_GRID_TOO_SMALL);
}

// Walk the window of cells kx..kx+gx-1 of row (ky,kz): every contiguous span of candidates with
// its periodic image (ix,iy,iz in {-1,0,1}), staged 64 at a time into LDS slot
// 'lane'.  stage(j, ix, iy, iz) is called by the lane that owns the slot;
// compute(count, chunk) runs between barriers once 64 candidates (or the rest)
// are in; chunk numbers the batches 0, 1, ... in this fixed order.
template <class Stage, class Compute>
__device__ __forceinline__ void for_window(const PairArgs& a, int kx, int ky, int kz, int gx, const int r[3],
                                           int lane, Stage&& stage, Compute&& compute)
{
    const int nx = a.g.n[0], ny = a.g.n[1], nz = a.g.n[2];
    int fill = 0;
    int chunk = 0;
    for (int dz = -r[2]; dz <= r[2]; ++dz) {
        int z2 = kz + dz, iz = 0;
        if (z2 < 0 || z2 >= nz) {
            if (!a.g.periodic[2]) continue;
            iz = z2 < 0 ? -1 : 1;
            z2 -= iz * nz;
        }
        for (int dy = -r[1]; dy <= r[1]; ++dy) {
            int y2 = ky + dy, iy = 0;
            if (y2 < 0 || y2 >= ny) {
                if (!a.g.periodic[1]) continue;
                iy = y2 < 0 ? -1 : 1;
                y2 -= iy * ny;
            }
            const int row = (z2 * ny + y2) * nx;
            const int x0 = kx - r[0], x1 = kx + gx - 1 + r[0];
            const bool per = a.g.periodic[0] != 0;
            // up to three spans: wrapped left part, main part, wrapped right part
            for (int sgi = 0; sgi < 3; ++sgi) {
                int c0, c1, ix;
                if (sgi == 0) {
                    if (!(per && x0 < 0)) continue;
                    c0 = x0 + nx; c1 = nx - 1; ix = -1;
                } else if (sgi == 1) {
                    c0 = x0 < 0 ? 0 : x0; c1 = x1 >= nx ? nx - 1 : x1; ix = 0;
                } else {
                    if (!(per && x1 >= nx)) continue;
                    c0 = 0; c1 = x1 - nx; ix = 1;
                }
                int jb = a.cell_start[row + c0];
                const int je = a.cell_start[row + c1 + 1];
                while (jb < je) {
                    int take = je - jb;
                    if (take > kWave - fill) take = kWave - fill;
                    if (lane >= fill && lane < fill + take) stage(jb + lane - fill, ix, iy, iz);
                    fill += take;
                    jb += take;
                    if (fill == kWave) {
                        __syncthreads();
                        compute(kWave, chunk);
                        __syncthreads();
                        fill = 0;
                        ++chunk;
                    }
                }
            }
        }
    }
    if (fill) {
        __syncthreads();
        compute(fill, chunk);
        __syncthreads();
    }
}

// Raw members of one staged candidate (as loaded, before conversion).
template <class T, int K>
struct RawK {
    T v[K];
    int j, ix, iy, iz, key;
    uint64_t mask;
};
template <class T> using Raw4 = RawK<T, 4>;
template <class T> using Raw12 = RawK<T, 12>;

// Raw members of one staged force candidate and its per-particle constants.
template <class T, class R>
struct ForceRaw {
    T v[9];
    R fc[5];
    int j, ix, iy, iz, key;
    uint64_t mask;
};

template <class T, class L>
__device__ __forceinline__ T ld_raw(const FieldRef& f, const L& l)
{
    return *(const T*)l.at(f);
}

// Float coordinate relative to the corner of cell k along axis d: an FP32
// view stores it already; a record's double is converted exactly as the
// gather converts it.
__device__ __forceinline__ float rel32_of(float v, int, int, const Geom&) { return v; }
__device__ __forceinline__ float rel32_of(double v, int d, int k, const Geom& g)
{
    const double o = __dadd_rn(g.lo[d], __dmul_rn((double)k, g.cell[d]));
    return __double2float_rn(__dsub_rn(v, o));
}

// ------------------------------------------------------------------ spans
//
// The window of a work item as a table of spans built once per item: every
// (dy, dz) row contributes up to three contiguous spans of sorted positions
// (wrapped left part, main part, wrapped right part), in the order for_window
// visits them, so candidate q of the window (and chunk q / 64) is the same
// in both.  Rows are resolved by all lanes at once, and the staging of chunk
// c + 1 is issued before chunk c is evaluated.

constexpr int kMaxSpans = 160;     // windows of reach <= 3 (7 x 7 rows x 3 spans)
constexpr int kMaxChunksW = 128;   // candidates per window <= 8192
constexpr int kSpanPosBits = 27;   // sorted positions below 2^27 share a word with the image

struct SpanLds {
    uint32_t jbi[kMaxSpans];      // first sorted position of the span | image << 27, the periodic
                                  // image (ix+1) + 3 (iy+1) + 9 (iz+1) < 27
    uint16_t pre[kMaxSpans + 2];  // window index of its first candidate; pre[ns] = W
    uint8_t cstart[kMaxChunksW];  // span holding the first candidate of each chunk
};

__device__ __forceinline__ int wave_excl_scan(int v, int lane, int& total)
{
    int x = v;
    for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    total = __shfl(x, kWave - 1, kWave);
    return x - v;
}

// Fills L for the window of cells kx..kx+gx-1 of row (ky, kz) with per-axis reach r; returns
// false (for every lane) when the window exceeds the table, leaving the
// caller to walk it with for_window.
__device__ bool build_spans(const PairArgs& a, int kx, int ky, int kz, int gx, const int r[3], int lane, SpanLds& L,
                            int& ns_out, int& W_out)
{
    if (a.n >= (1ll << kSpanPosBits)) return false;
    const int nx = a.g.n[0], ny = a.g.n[1], nz = a.g.n[2];
    const int nyw = 2 * r[1] + 1;
    const int nrows = nyw * (2 * r[2] + 1);
    int ns = 0, W = 0;
    for (int r0 = 0; r0 < nrows; r0 += kWave) {
        const int rr = r0 + lane;
        // the row's spans in window order: wrapped left part, main part, wrapped
        // right part (each may be absent)
        int cnt = 0;
        int b0 = 0, n0 = 0, b1 = 0, n1 = 0, b2 = 0, n2 = 0;
        bool vl = false, vr = false;
        uint32_t img = 0;
        if (rr < nrows) {
            int z2 = kz + rr / nyw - r[2], iz = 0;
            int y2 = ky + rr % nyw - r[1], iy = 0;
            bool ok = true;
            if (z2 < 0 || z2 >= nz) {
                if (a.g.periodic[2]) { iz = z2 < 0 ? -1 : 1; z2 -= iz * nz; } else ok = false;
            }
            if (y2 < 0 || y2 >= ny) {
                if (a.g.periodic[1]) { iy = y2 < 0 ? -1 : 1; y2 -= iy * ny; } else ok = false;
            }
            if (ok) {
                const int row = (z2 * ny + y2) * nx;
                const int x0 = kx - r[0], x1 = kx + gx - 1 + r[0];
                const bool per = a.g.periodic[0] != 0;
                vl = per && x0 < 0;
                vr = per && x1 >= nx;
                const int m0 = x0 < 0 ? 0 : x0;
                const int m1 = x1 >= nx ? nx - 1 : x1;
                if (vl) {
                    b0 = a.cell_start[row + x0 + nx];
                    n0 = a.cell_start[row + nx] - b0;
                }
                b1 = a.cell_start[row + m0];
                n1 = a.cell_start[row + m1 + 1] - b1;
                if (vr) {
                    b2 = a.cell_start[row];
                    n2 = a.cell_start[row + x1 - nx + 1] - b2;
                }
                cnt = 1 + (vl ? 1 : 0) + (vr ? 1 : 0);
                img = (uint32_t)(3 * (iy + 1) + 9 * (iz + 1));
            }
        }
        int tot_s, tot_w;
        const int ps = wave_excl_scan(cnt, lane, tot_s);
        const int pw = wave_excl_scan(n0 + n1 + n2, lane, tot_w);
        if (ns + tot_s > kMaxSpans || W + tot_w >= 65536) return false;
        if (cnt) {
            int k = ns + ps;
            int w = W + pw;
            if (vl) {
                L.jbi[k] = (uint32_t)b0 | (img << kSpanPosBits);
                L.pre[k] = (uint16_t)w;
                ++k;
                w += n0;
            }
            L.jbi[k] = (uint32_t)b1 | ((img + 1u) << kSpanPosBits);
            L.pre[k] = (uint16_t)w;
            ++k;
            w += n1;
            if (vr) {
                L.jbi[k] = (uint32_t)b2 | ((img + 2u) << kSpanPosBits);
                L.pre[k] = (uint16_t)w;
            }
        }
        ns += tot_s;
        W += tot_w;
    }
    const int nch = (W + kWave - 1) / kWave;
    if (nch > kMaxChunksW) return false;
    if (lane == 0) L.pre[ns] = (uint16_t)W;
    __syncthreads();
    for (int c = lane; c < nch; c += kWave) {
        // the last span starting at or before the chunk's first candidate
        const int q = c * kWave;
        int lo = 0, hi = ns;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (L.pre[mid] <= q) lo = mid; else hi = mid;
        }
        L.cstart[c] = (uint8_t)lo;
    }
    __syncthreads();
    ns_out = ns;
    W_out = W;
    return true;
}

// Candidate q of chunk c for this lane: its sorted position and image.
__device__ __forceinline__ void span_lookup(const SpanLds& L, int c, int q, int& j, int& ix, int& iy, int& iz)
{
    int s = L.cstart[c];
    while (L.pre[s + 1] <= q) ++s;
    const uint32_t v = L.jbi[s];
    j = (int)(v & ((1u << kSpanPosBits) - 1u)) + (q - L.pre[s]);
    const int im = (int)(v >> kSpanPosBits);
    ix = im % 3 - 1;
    iy = (im / 3) % 3 - 1;
    iz = im / 9 - 1;
}

// Pipelined walk of a window described by L: fetch(valid, j, ix, iy, iz, c)
// issues the loads of this lane's candidate of chunk c and returns them,
// put(v, in_chunk) writes them to this lane's LDS slot, compute(count, chunk)
// evaluates a staged chunk.  The loads of chunk c + 1 are in flight while
// chunk c is evaluated.
template <class Fetch, class Put, class Compute>
__device__ __forceinline__ void run_window(const SpanLds& L, int W, int lane, Fetch&& fetch, Put&& put,
                                           Compute&& compute)
{
    const int nch = (W + kWave - 1) / kWave;
    auto get = [&](int c) {
        const int q = c * kWave + lane;
        int j = 0, ix = 0, iy = 0, iz = 0;
        const bool valid = q < W;
        if (valid) span_lookup(L, c, q, j, ix, iy, iz);
        return fetch(valid, j, ix, iy, iz, c);
    };
    auto cur = get(0);
    for (int c = 0; c < nch; ++c) {
        const int count = W - c * kWave < kWave ? W - c * kWave : kWave;
        put(cur, lane < count);
        if (c + 1 < nch) cur = get(c + 1);
        __syncthreads();
        compute(count, c);
        __syncthreads();
    }
}

// Bit k of the result is test(sl + k*tpi) for the candidates of this lane
// below count; four tests are packed per step.
template <class Test>
__device__ __forceinline__ uint64_t lane_mask(int count, int sl, int tpi, Test&& test)
{
    uint64_t hits = 0;
    int k = 0;
    int t = sl;
    for (; t + 3 * tpi < count; t += 4 * tpi, k += 4) {
        const uint32_t b0 = test(t) ? 1u : 0u;
        const uint32_t b1 = test(t + tpi) ? 2u : 0u;
        const uint32_t b2 = test(t + 2 * tpi) ? 4u : 0u;
        const uint32_t b3 = test(t + 3 * tpi) ? 8u : 0u;
        hits |= (uint64_t)(b0 | b1 | b2 | b3) << k;
    }
    for (; t < count; t += tpi, ++k) hits |= (test(t) ? 1ull : 0ull) << k;
    return hits;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ int wave_max_i(int v)
{
    for (int off = 32; off > 0; off >>= 1) {
        int o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// ================================================================ density
//
// Window-resident neighbour lists.  A first walk over a work item's window
// tests every candidate against a list radius per local particle, 2 h_l with
// h_l = min(h_cap, (1 + 1/16) h), and keeps the union of the hits (over the
// item's particles) compacted in LDS, position and mass, and per particle the
// list of its hits as indices into that union.  Every pass of the h iteration
// then walks its particle's list, split evenly over the particle's lanes,
// without touching global memory or the window again.  Should a Newton step
// take some h beyond its h_l, the item starts over with the chunk walk below;
// so does a window whose union or lists do not fit.  The chunk walk restages
// the window 64 candidates at a time in every pass and revisits the hits
// within twice the cell cap that its first pass cached.
// The walk that builds the lists also writes those cap hits for the force loop.

constexpr int kUMax = 320;     // union entries per work item
constexpr int kPool = 2304;    // list entries per work item, split evenly over its particles
constexpr double kListGrow = 1.0 + 1.0 / 16.0;

template <class R>
struct alignas(16) P4 {
    R x, y, z, m;
};

template <class R>
union DensStage {
    struct {
        R x[kWave], y[kWave], z[kWave], m[kWave];
        int j[kWave];
    } s;                       // one chunk of staged candidates
    struct {
        double t[3][kWave];
        int c[kWave];
    } r;                       // per-lane partial sums of a pass
};

template <class R>
union DensBig {
    uint64_t mcache[kMaskChunks][kWave];   // chunk walk: hit masks of the first pass
    P4<R> u[kUMax];                        // list walk: the union of the hits
};

// Bit k of lo (hi) is set when candidate sl + k*tpi lies within r2lo (r2hi);
// r^2 is fused, four candidates are tested per step.
template <class R>
__device__ __forceinline__ void lane_mask2(const R* sx, const R* sy, const R* sz, int count, int sl, int tpi, R xi,
                                           R yi, R zi, R r2lo, R r2hi, uint64_t& lo, uint64_t& hi)
{
    auto r2f = [&](int t) {
        const R dx = xi - sx[t];
        const R dy = yi - sy[t];
        const R dz = zi - sz[t];
        return fma(dz, dz, fma(dy, dy, dx * dx));
    };
    lo = 0;
    hi = 0;
    int k = 0;
    int t = sl;
    for (; t + 3 * tpi < count; t += 4 * tpi, k += 4) {
        const R q0 = r2f(t), q1 = r2f(t + tpi), q2 = r2f(t + 2 * tpi), q3 = r2f(t + 3 * tpi);
        const uint32_t l = (q0 < r2lo ? 1u : 0u) | (q1 < r2lo ? 2u : 0u) | (q2 < r2lo ? 4u : 0u) |
                           (q3 < r2lo ? 8u : 0u);
        const uint32_t h = (q0 < r2hi ? 1u : 0u) | (q1 < r2hi ? 2u : 0u) | (q2 < r2hi ? 4u : 0u) |
                           (q3 < r2hi ? 8u : 0u);
        lo |= (uint64_t)l << k;
        hi |= (uint64_t)h << k;
    }
    for (; t < count; t += tpi, ++k) {
        const R q = r2f(t);
        lo |= (q < r2lo ? 1ull : 0ull) << k;
        hi |= (q < r2hi ? 1ull : 0ull) << k;
    }
}

template <bool DIRECT, bool FP32, bool MASKED, int KERN>
__global__ __launch_bounds__(kWave) void k_density(PairArgs a)
{
    using R = typename std::conditional<FP32, float, double>::type;
    using RawT = typename std::conditional<FP32 && !DIRECT, float, double>::type;
    __shared__ DensStage<R> st;
    __shared__ SpanLds spans;
    __shared__ DensBig<R> big;
    __shared__ uint16_t s_list[kPool];
    __shared__ uint16_t s_uidx[kWave];
    __shared__ uint8_t s_flag[kWave];
    __shared__ int s_self[kWave];
    __shared__ int s_item;
    R* const sx = st.s.x;
    R* const sy = st.s.y;
    R* const sz = st.s.z;
    R* const sm = st.s.m;
    int* const sj = st.s.j;

    const int lane = threadIdx.x;
    const int n_items = a.meta[META_NITEMS];
    const int xcd = blockIdx.x % kNumXcd;
    const double eta3 = a.eta * a.eta * a.eta;
    if (blockIdx.x == 0 && lane == 0) a.meta[META_MASKS] = 1 + a.tpi + (FP32 ? 128 : 0);
    int qoff = 0;
    unsigned long long n_final = 0, n_evals = 0;
    int maxit = 0;
    uint32_t flags = 0;

    for (;;) {
        if (lane == 0) s_item = next_item(a.meta + a.qhead, n_items, xcd, (int)(blockIdx.x / kNumXcd), qoff);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);   // wave-uniform
        __syncthreads();
        if (item < 0) break;

        const int4 it = a.items[item];
        const int cell = it.x, first = it.y, ni = it.z, gx = it.w;
        int tpi = kWave / ni;
        if (a.tpi > 0 && a.tpi < tpi) tpi = a.tpi;
        const int il = lane / tpi, sl = lane - il * tpi;
        const bool act = il < ni;
        const int pi = first + (act ? il : 0);
        int kx, ky, kz;
        cell_coords(cell, a.g, kx, ky, kz);
        int Rg = 0;   // the item's reach: the largest of its cells (equal, empty cells aside)
        for (int k = 0; k < gx; ++k) Rg = a.reach[cell + k] > Rg ? a.reach[cell + k] : Rg;
        int r[3];
        axis_reach(a, Rg, gx, r);
        double hcap = 0.5 * (double)r[0] * a.g.cell[0];
        hcap = fmin(hcap, 0.5 * (double)r[1] * a.g.cell[1]);
        hcap = fmin(hcap, 0.5 * (double)r[2] * a.g.cell[2]);
        // no h of this item can exceed hcap, so no pair of any pass lies beyond 2 hcap
        const double Hcap = 2.0 * hcap;
        // widened so that a fused r^2 (a few ulp from the exact one) never misses a
        // candidate: the exact test decides each pair later
        constexpr double kWiden = FP32 ? 1.0 + 4e-6 : 1.0 + 1e-12;
        const R H2capw = (R)(Hcap * Hcap * kWiden);

        const Loc<DIRECT> li = locate<DIRECT>(a.acc, pi);
        R xi, yi, zi;
        double mi;
        if constexpr (FP32) {
            // relative to the corner of the item's first cell, as the candidates are staged
            const int own = a.key_sorted[pi];
            int ox, oy, oz;
            cell_coords(own, a.g, ox, oy, oz);
            xi = ld_as_f32(a.f[SPHV_X], li, a.g, own) + __double2float_rn((double)(ox - kx) * a.g.cell[0]);
            yi = ld_as_f32(a.f[SPHV_Y], li, a.g, own) + __double2float_rn((double)(oy - ky) * a.g.cell[1]);
            zi = ld_as_f32(a.f[SPHV_Z], li, a.g, own) + __double2float_rn((double)(oz - kz) * a.g.cell[2]);
            mi = (double)ld_as_f32(a.f[SPHV_M], li, a.g, own);
        } else {
            xi = ld_f64(a.f[SPHV_X], li);
            yi = ld_f64(a.f[SPHV_Y], li);
            zi = ld_f64(a.f[SPHV_Z], li);
            mi = ld_f64(a.f[SPHV_M], li);
        }
        const double h0 = ld_f64(a.f[SPHV_H], li);
        // list radius of this particle (its h may not leave [.., hl] while the lists serve it)
        const double hl = fmin(hcap, kListGrow * h0);
        const R Hl2w = (R)((2.0 * hl) * (2.0 * hl) * kWiden);
        int n_spans = 0, W = 0;
        const bool use_spans = build_spans(a, kx, ky, kz, gx, r, lane, spans, n_spans, W);

        // staging of one candidate: fetch issues the loads (raw members), put
        // converts them and writes this lane's LDS slot
        auto fetch = [&](bool valid, int j, int ix, int iy, int iz, int) {
            Raw4<RawT> v;
            v.j = j;
            v.ix = ix;
            v.iy = iy;
            v.iz = iz;
            if (valid) {
                const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
                v.v[0] = ld_raw<RawT>(a.f[SPHV_X], lj);
                v.v[1] = ld_raw<RawT>(a.f[SPHV_Y], lj);
                v.v[2] = ld_raw<RawT>(a.f[SPHV_Z], lj);
                v.v[3] = ld_raw<RawT>(a.f[SPHV_M], lj);
                if constexpr (FP32) v.key = a.key_sorted[j];
            }
            return v;
        };
        auto put = [&](const Raw4<RawT>& v, bool in_chunk) {
            if (!in_chunk) return;
            if constexpr (FP32) {
                int jx, jy, jz;
                cell_coords(v.key, a.g, jx, jy, jz);
                sx[lane] = rel32_of(v.v[0], 0, jx, a.g) +
                           __double2float_rn((double)(jx - kx + v.ix * a.g.n[0]) * a.g.cell[0]);
                sy[lane] = rel32_of(v.v[1], 1, jy, a.g) +
                           __double2float_rn((double)(jy - ky + v.iy * a.g.n[1]) * a.g.cell[1]);
                sz[lane] = rel32_of(v.v[2], 2, jz, a.g) +
                           __double2float_rn((double)(jz - kz + v.iz * a.g.n[2]) * a.g.cell[2]);
                sm[lane] = (R)v.v[3];
            } else {
                sx[lane] = v.v[0] + (double)v.ix * a.g.len[0];
                sy[lane] = v.v[1] + (double)v.iy * a.g.len[1];
                sz[lane] = v.v[2] + (double)v.iz * a.g.len[2];
                sm[lane] = v.v[3];
            }
            sj[lane] = v.j;
        };
        auto stage = [&](int j, int ix, int iy, int iz) { put(fetch(true, j, ix, iy, iz, 0), true); };

        // ---- list walk set-up: one walk over the window builds the union and the lists
        const int cap_i = kPool / ni;      // list entries per particle
        const int lbase = (act ? il : 0) * cap_i;
        int len = 0;                        // entries of this particle's list
        bool lists = false;
        if (use_spans) {
            s_self[lane] = -1;
            const int nch = (W + kWave - 1) / kWave;
            const int g0 = act ? il * tpi : 0;
            const int g1 = act ? g0 + tpi - 1 : 0;
            int nU = 0;
            bool fits = true;
            auto get = [&](int c) {
                const int q = c * kWave + lane;
                int j = 0, ix = 0, iy = 0, iz = 0;
                const bool valid = q < W;
                if (valid) span_lookup(spans, c, q, j, ix, iy, iz);
                return fetch(valid, j, ix, iy, iz, c);
            };
            auto cur = get(0);
            for (int c = 0; c < nch && fits; ++c) {
                const int count = W - c * kWave < kWave ? W - c * kWave : kWave;
                put(cur, lane < count);
                s_flag[lane] = 0;
                if (c + 1 < nch) cur = get(c + 1);
                __syncthreads();
                uint64_t hits = 0, caph = 0;
                if (act) lane_mask2<R>(sx, sy, sz, count, sl, tpi, xi, yi, zi, Hl2w, H2capw, hits, caph);
                if (c < kMaskChunks) a.item_masks[((int64_t)item * kMaskChunks + c) * kWave + lane] = caph;
                for (uint64_t m = hits; m; m &= m - 1) s_flag[sl + __builtin_ctzll(m) * tpi] = 1;
                __syncthreads();
                // compact the chunk's hits (over all particles) into the union
                const bool f = lane < count && s_flag[lane];
                const uint64_t bal = __ballot(f);
                const int u = nU + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                nU += __popcll(bal);
                if (f && u < kUMax) {
                    big.u[u] = P4<R>{sx[lane], sy[lane], sz[lane], sm[lane]};
                    s_uidx[lane] = (uint16_t)u;
                }
                // append this lane's hits to its particle's list, lanes in order
                const int hl_n = __popcll(hits);
                int tot;
                const int excl = wave_excl_scan(hl_n, lane, tot);
                const int e0 = __shfl(excl, g0, kWave);
                const int e1 = __shfl(excl + hl_n, g1, kWave);
                const int pos = len + excl - e0;
                const bool over = nU > kUMax || (act && pos + hl_n > cap_i);
                fits = !__any(over);
                __syncthreads();
                if (fits) {
                    int k = pos;
                    for (uint64_t m = hits; m; m &= m - 1) {
                        const int t = sl + __builtin_ctzll(m) * tpi;
                        const int u2 = s_uidx[t];
                        s_list[lbase + k] = (uint16_t)u2;
                        ++k;
                        if (sj[t] == pi) s_self[il] = u2;
                    }
                    len += e1 - e0;
                }
                __syncthreads();
            }
            lists = fits;
        }
        const int self_u = lists && act ? s_self[il] : -1;

        double h = h0;
        bool done = !act;
        unsigned long long it_final = 0, it_evals = 0;
        int it_maxit = 0;
        uint32_t it_flags = 0;
        for (int pass = 0;; ++pass) {
            const double Hd = 2.0 * h;
            const double H2d = Hd * Hd;
            const double hinv = 1.0 / h;
            const R H2 = (R)H2d;
            const R hin = (R)hinv;
            double t0 = 0.0, t1 = 0.0, t2 = 0.0;       // sum m w, sum w, sum m (3w + q w')
            float c0 = 0.f, c1 = 0.f, c2 = 0.f;         // FP32 compensation terms
            float f0 = 0.f, f1 = 0.f, f2 = 0.f;         // FP32 running sums
            int cnt = 0;

            // one candidate's contribution at the current h; in == false turns
            // it into the neutral element (zero w and w' add nothing)
            auto term = [&](R m, R r2, bool in, R& p0, R& p1, R& p2) {
                const R rr = r2 * rsqrt_nr(fmax(r2, Tiny<R>::v));
                const R q = rr * hin;
                R w, dw;
                spline<KERN>(q, w, dw);
                w = in ? w : (R)0;
                dw = in ? dw : (R)0;
                p0 = fma(m, w, p0);
                p1 = p1 + w;
                p2 = fma(m, fma(q, dw, (R)3 * w), p2);
            };
            auto fold = [&](R p0, R p1, R p2) {
                if constexpr (FP32) {
                    neumaier(f0, c0, p0);
                    neumaier(f1, c1, p1);
                    neumaier(f2, c2, p2);
                } else {
                    t0 += p0;
                    t1 += p1;
                    t2 += p2;
                }
            };

            if (lists) {
                if (!done) {
                    // entries sl, sl + tpi, ... of the list; float partial sums are
                    // folded into the compensated ones every 16 entries.  The index two
                    // entries ahead and the union entry one ahead are read while the
                    // current one is evaluated.
                    R p0 = 0, p1 = 0, p2 = 0;
                    int k = 0;
                    int u_nx = sl + tpi < len ? s_list[lbase + sl + tpi] : 0;
                    int u = sl < len ? s_list[lbase + sl] : 0;
                    P4<R> c_nx = big.u[u];
                    for (int e = sl; e < len; e += tpi) {
                        const P4<R> c = c_nx;
                        const int e2 = e + 2 * tpi;
                        const int u_n2 = e2 < len ? s_list[lbase + e2] : 0;
                        c_nx = big.u[u_nx];
                        const R dx = xi - c.x;
                        const R dy = yi - c.y;
                        const R dz = zi - c.z;
                        const R r2 = dx * dx + dy * dy + dz * dz;
                        const bool in = r2 < H2;
                        // list entries lie within the list radius, so nearly all are in
                        // range: the neutral-element select costs less than a divergent
                        // branch, and gives the same bits
                        term(c.m, r2, in, p0, p1, p2);
                        cnt += (in && u != self_u) ? 1 : 0;
                        if (FP32 && ++k == 16) {
                            fold(p0, p1, p2);
                            p0 = p1 = p2 = 0;
                            k = 0;
                        }
                        u = u_nx;
                        u_nx = u_n2;
                    }
                    fold(p0, p1, p2);
                }
            } else {
                auto compute = [&](int count, int chunk) {
                    if (done) return;
                    R p0 = 0, p1 = 0, p2 = 0;
                    if constexpr (MASKED) {
                        // the force loop's candidates within 2 hcap, cached as in the
                        // branching form
                        if (pass == 0 && chunk < kMaskChunks)
                            a.item_masks[((int64_t)item * kMaskChunks + chunk) * kWave + lane] =
                                lane_mask(count, sl, tpi, [&](int t) {
                                    const R dx = xi - sx[t];
                                    const R dy = yi - sy[t];
                                    const R dz = zi - sz[t];
                                    return fma(dz, dz, fma(dy, dy, dx * dx)) < H2capw;
                                });
                        // every candidate evaluated, out-of-range terms are the neutral element
                        for (int t = sl; t < count; t += tpi) {
                            const R dx = xi - sx[t];
                            const R dy = yi - sy[t];
                            const R dz = zi - sz[t];
                            const R r2 = dx * dx + dy * dy + dz * dz;
                            const bool in = r2 < H2;
                            term(sm[t], r2, in, p0, p1, p2);
                            // the self pair (r = 0) enters the sums but is not counted
                            cnt += (in && (r2 > (R)0 || sj[t] != pi)) ? 1 : 0;
                        }
                    } else {
                        // the first pass tests every candidate of this lane against 2 hcap
                        // and keeps the hits; later passes only revisit those.  Hits are
                        // evaluated in increasing order, in range at the current h only.
                        uint64_t hits = 0;
                        if (pass > 0 && chunk < kMaskChunks) {
                            hits = big.mcache[chunk][lane];
                        } else {
                            hits = lane_mask(count, sl, tpi, [&](int t) {
                                const R dx = xi - sx[t];
                                const R dy = yi - sy[t];
                                const R dz = zi - sz[t];
                                return fma(dz, dz, fma(dy, dy, dx * dx)) < H2capw;
                            });
                            if (pass == 0 && chunk < kMaskChunks) {
                                big.mcache[chunk][lane] = hits;
                                a.item_masks[((int64_t)item * kMaskChunks + chunk) * kWave + lane] = hits;
                            }
                        }
                        while (hits) {
                            const int kk = __builtin_ctzll(hits);
                            hits &= hits - 1;
                            const int t = sl + kk * tpi;
                            const R dx = xi - sx[t];
                            const R dy = yi - sy[t];
                            const R dz = zi - sz[t];
                            const R r2 = dx * dx + dy * dy + dz * dz;
                            if (r2 < H2) {
                                term(sm[t], r2, true, p0, p1, p2);
                                cnt += (r2 > (R)0 || sj[t] != pi) ? 1 : 0;
                            }
                        }
                    }
                    fold(p0, p1, p2);
                };
                if (use_spans) run_window(spans, W, lane, fetch, put, compute);
                else for_window(a, kx, ky, kz, gx, r, lane, stage, compute);
            }

            if constexpr (FP32) {
                t0 = (double)f0 + (double)c0;
                t1 = (double)f1 + (double)c1;
                t2 = (double)f2 + (double)c2;
            }
            if (tpi > 1) {
                st.r.t[0][lane] = t0;
                st.r.t[1][lane] = t1;
                st.r.t[2][lane] = t2;
                st.r.c[lane] = cnt;
                __syncthreads();
                if (act) {
                    const int b = il * tpi;
                    t0 = t1 = t2 = 0.0;
                    cnt = 0;
                    for (int k = 0; k < tpi; ++k) {
                        t0 += st.r.t[0][b + k];
                        t1 += st.r.t[1][b + k];
                        t2 += st.r.t[2][b + k];
                        cnt += st.r.c[b + k];
                    }
                }
                __syncthreads();
            }

            bool leave = false;   // an h outgrew its list radius
            if (!done) {
                const double h3 = h * h * h;
                const double norm = 1.0 / (kPi * h3);
                const double rho = norm * t0;
                const double nsum = norm * t1;
                const double drho = -(norm * hinv) * t2;
                const double mq = mi * eta3;
                const double f = rho - mq / h3;
                const double fp = drho + 3.0 * mq / (h3 * h);
                double hn;
                if (fp > 0.0) {
                    hn = h - f / fp;
                    if (hn < 0.5 * h) hn = 0.5 * h;
                    if (hn > 2.0 * h) hn = 2.0 * h;
                } else {
                    hn = a.eta * cbrt(mi / rho);
                }
                if (!isfinite(hn)) hn = a.eta * cbrt(mi / rho);
                if (hn > hcap) {
                    hn = hcap;
                    it_flags |= SPHV_F_H_CAP_HIT;
                }
                const bool conv = fabs(hn - h) <= a.tol * h;
                if (sl == 0) it_evals += (unsigned long long)cnt;
                if (conv || pass + 1 >= a.max_iter) {
                    if (!conv) it_flags |= SPHV_F_H_NOT_CONVERGED;
                    const double omega = 1.0 + h / (3.0 * rho) * drho;
                    const double wcount = (4.0 * kPi / 3.0) * (8.0 * h3) * nsum;
                    if (!(isfinite(rho) && isfinite(omega))) it_flags |= SPHV_F_NONFINITE_OUTPUT;
                    if (sl == 0) {
                        st_f64(a.f[SPHV_H], li, h);
                        st_f64(a.f[SPHV_RHO], li, rho);
                        st_f64(a.f[SPHV_OMEGA], li, omega);
                        st_f64(a.f[SPHV_WCOUNT], li, wcount);
                        it_final += (unsigned long long)cnt;
                    }
                    it_maxit = pass + 1 > it_maxit ? pass + 1 : it_maxit;
                    done = true;
                } else {
                    leave = lists && hn > hl;
                    h = hn;
                }
            }
            if (__any(leave)) {
                // start the item over with the chunk walk: its results replace
                // whatever the list walk stored
                lists = false;
                h = h0;
                done = !act;
                it_final = it_evals = 0;
                it_maxit = 0;
                it_flags = 0;
                pass = -1;
                continue;
            }
            if (__all(done)) break;
        }
        n_final += it_final;
        n_evals += it_evals;
        maxit = it_maxit > maxit ? it_maxit : maxit;
        flags |= it_flags;
    }

    n_final = wave_sum_u64(n_final);
    n_evals = wave_sum_u64(n_evals);
    maxit = wave_max_i(maxit);
    for (int off = 32; off > 0; off >>= 1) flags |= __shfl_xor(flags, off, kWave);
    if (lane == 0) leave_part(a.part, (int64_t)n_final, (int64_t)n_evals, maxit, flags);
}

// ================================================================== force

template <bool DIRECT, bool FP32, bool MASKED, int KERN>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3))) void k_force(PairArgs a)
{
    using R = typename std::conditional<FP32, float, double>::type;
    // staged j data
    __shared__ R sx[kWave], sy[kWave], sz[kWave], svx[kWave], svy[kWave], svz[kWave];
    __shared__ R sm[kWave], sH2[kWave], shinv[kWave], snorm[kWave], srho[kWave], sA[kWave], sc[kWave], sal[kWave];
    __shared__ SpanLds spans;
    using RawT = typename std::conditional<FP32 && !DIRECT, float, double>::type;
    __shared__ int sj[kWave];
    __shared__ double red[4][kWave];
    __shared__ double redv[kWave];
    __shared__ int redc[kWave];
    __shared__ int s_item;

    const int lane = threadIdx.x;
    const int n_items = a.meta[META_NITEMS];
    const int xcd = blockIdx.x % kNumXcd;
    const R gm = (R)a.gamma;
    const R gm1 = (R)(a.gamma - 1.0);
    const R ggm1 = (R)(a.gamma * (a.gamma - 1.0));
    const int masks_tag = a.meta[META_MASKS];
    int qoff = 0;
    unsigned long long n_pairs = 0;
    uint32_t flags = 0;
    (void)gm;

    for (;;) {
        if (lane == 0) s_item = next_item(a.meta + a.qhead, n_items, xcd, (int)(blockIdx.x / kNumXcd), qoff);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);   // wave-uniform
        __syncthreads();
        if (item < 0) break;

        const int4 it = a.items[item];
        const int cell = it.x, first = it.y, ni = it.z, gx = it.w;
        int tpi = kWave / ni;
        if (a.tpi > 0 && a.tpi < tpi) tpi = a.tpi;
        const int il = lane / tpi, sl = lane - il * tpi;
        const bool act = il < ni;
        const int pi = first + (act ? il : 0);
        int kx, ky, kz;
        cell_coords(cell, a.g, kx, ky, kz);
        // the item's force window, density reach and neighbours' bound: the
        // largest over its cells
        int Rf = 0, Rd = 0, Rs = 0;
        for (int k = 0; k < gx; ++k) {
            Rf = a.reach[cell + k] > Rf ? a.reach[cell + k] : Rf;
            Rd = a.reach_d[cell + k] > Rd ? a.reach_d[cell + k] : Rd;
            Rs = a.reach_s[cell + k] > Rs ? a.reach_s[cell + k] : Rs;
        }
        int r[3];
        axis_reach(a, Rf, gx, r);
        // the density loop cached the candidates within twice its cell cap for
        // this window; they hold every force pair when the windows agree and no
        // cell whose reach covers these has a larger own force reach (no
        // partner's support reaches further than the cap)
        const bool reuse = !MASKED && masks_tag == 1 + a.tpi + (FP32 ? 128 : 0) && Rf == Rd && Rs <= Rd;
        int n_spans = 0, W = 0;
        const bool use_spans = build_spans(a, kx, ky, kz, gx, r, lane, spans, n_spans, W);

        // local particle i and its derived quantities
        const Loc<DIRECT> li = locate<DIRECT>(a.acc, pi);
        R xi, yi, zi, vxi, vyi, vzi, hi, rhoi, omi, ui, ali;
        if constexpr (FP32) {
            // relative to the corner of the item's first cell, as the candidates are staged
            const int own = a.key_sorted[pi];
            int ox, oy, oz;
            cell_coords(own, a.g, ox, oy, oz);
            xi = ld_as_f32(a.f[SPHV_X], li, a.g, own) + __double2float_rn((double)(ox - kx) * a.g.cell[0]);
            yi = ld_as_f32(a.f[SPHV_Y], li, a.g, own) + __double2float_rn((double)(oy - ky) * a.g.cell[1]);
            zi = ld_as_f32(a.f[SPHV_Z], li, a.g, own) + __double2float_rn((double)(oz - kz) * a.g.cell[2]);
            vxi = ld_as_f32(a.f[SPHV_VX], li, a.g, cell);
            vyi = ld_as_f32(a.f[SPHV_VY], li, a.g, cell);
            vzi = ld_as_f32(a.f[SPHV_VZ], li, a.g, cell);
            hi = ld_as_f32(a.f[SPHV_H], li, a.g, cell);
            rhoi = ld_as_f32(a.f[SPHV_RHO], li, a.g, cell);
            omi = ld_as_f32(a.f[SPHV_OMEGA], li, a.g, cell);
            ui = ld_as_f32(a.f[SPHV_U], li, a.g, cell);
            ali = ld_as_f32(a.f[SPHV_ALPHA], li, a.g, cell);
        } else {
            xi = ld_f64(a.f[SPHV_X], li);
            yi = ld_f64(a.f[SPHV_Y], li);
            zi = ld_f64(a.f[SPHV_Z], li);
            vxi = ld_f64(a.f[SPHV_VX], li);
            vyi = ld_f64(a.f[SPHV_VY], li);
            vzi = ld_f64(a.f[SPHV_VZ], li);
            hi = ld_f64(a.f[SPHV_H], li);
            rhoi = ld_f64(a.f[SPHV_RHO], li);
            omi = ld_f64(a.f[SPHV_OMEGA], li);
            ui = ld_f64(a.f[SPHV_U], li);
            ali = ld_f64(a.f[SPHV_ALPHA], li);
        }
        const R Pi_ = gm1 * rhoi * ui;
        const R ci = sqrt(ggm1 * ui);
        const R Ai = Pi_ / (omi * rhoi * rhoi);
        const R hinvi = (R)1 / hi;
        const R hinv2 = hinvi * hinvi;
        const R normi = hinv2 * hinv2 / (R)kPi;
        const R hali = (R)0.5 * ali;

        double ax = 0.0, ay = 0.0, az = 0.0, du = 0.0;
        float fax = 0.f, cax = 0.f, fay = 0.f, cay = 0.f, faz = 0.f, caz = 0.f, fdu = 0.f, cdu = 0.f;
        R vsig = (R)2 * ci;
        int cnt = 0;

        // staging of one candidate: fetch issues the loads (raw members and, when
        // the density loop's masks apply, this lane's mask of the chunk), put
        // converts them, derives P, c, A, 1/h, and writes this lane's LDS slot
        uint64_t cmask = 0;
        // the per-particle constants (A, c, 1/h, norm, (2h)^2), computed once per
        // particle by the prep kernel that runs before this one
        const R* fcon = (const R*)a.fconst;
        auto fetch = [&](bool valid, int j, int ix, int iy, int iz, int c) {
            ForceRaw<RawT, R> v;
            v.j = j;
            v.ix = ix;
            v.iy = iy;
            v.iz = iz;
            v.mask = 0;
            if (reuse && c < kMaskChunks) v.mask = a.item_masks[((int64_t)item * kMaskChunks + c) * kWave + lane];
            if (valid) {
                const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
                const int roles[9] = {SPHV_X, SPHV_Y, SPHV_Z, SPHV_VX, SPHV_VY, SPHV_VZ, SPHV_M, SPHV_ALPHA,
                                      SPHV_RHO};
#pragma unroll
                for (int k = 0; k < 9; ++k) v.v[k] = ld_raw<RawT>(a.f[roles[k]], lj);
#pragma unroll
                for (int k = 0; k < 5; ++k) v.fc[k] = fcon[(int64_t)k * a.n + j];
                if constexpr (FP32) v.key = a.key_sorted[j];
            }
            return v;
        };
        auto put = [&](const ForceRaw<RawT, R>& v, bool in_chunk) {
            cmask = v.mask;
            if (!in_chunk) return;
            if constexpr (FP32) {
                int jx, jy, jz;
                cell_coords(v.key, a.g, jx, jy, jz);
                const int dk[3] = {jx - kx + v.ix * a.g.n[0], jy - ky + v.iy * a.g.n[1], jz - kz + v.iz * a.g.n[2]};
                const int kk[3] = {jx, jy, jz};
                R* dst[3] = {sx, sy, sz};
                for (int d = 0; d < 3; ++d)
                    dst[d][lane] = rel32_of(v.v[d], d, kk[d], a.g) + __double2float_rn((double)dk[d] * a.g.cell[d]);
            } else {
                sx[lane] = v.v[0] + (double)v.ix * a.g.len[0];
                sy[lane] = v.v[1] + (double)v.iy * a.g.len[1];
                sz[lane] = v.v[2] + (double)v.iz * a.g.len[2];
            }
            svx[lane] = (R)v.v[3];
            svy[lane] = (R)v.v[4];
            svz[lane] = (R)v.v[5];
            sm[lane] = (R)v.v[6];
            sal[lane] = (R)0.5 * (R)v.v[7];
            srho[lane] = (R)v.v[8];
            sA[lane] = v.fc[0];
            sc[lane] = v.fc[1];
            shinv[lane] = v.fc[2];
            snorm[lane] = v.fc[3];
            sH2[lane] = v.fc[4];
            sj[lane] = v.j;
        };
        auto stage = [&](int j, int ix, int iy, int iz) { put(fetch(true, j, ix, iy, iz, kMaskChunks), true); };

        // (2 max(h_i, h_j))^2 == max((2 h_i)^2, (2 h_j)^2): squaring and its
        // rounding are monotone, so the test is exact and per side
        const R Hi = (R)2 * hi;
        const R H2i = Hi * Hi;
        // the candidate test uses a fused r^2, shrunk so that it never rejects a pair
        // the exact test in the hit loop would accept
        const R shrink = (R)(FP32 ? 1.0 - 4e-6 : 1.0 - 1e-12);

        // one pair's contribution; live == false gives the neutral element
        auto term = [&](int t, R dx, R dy, R dz, R r2, bool live, R& pax, R& pay, R& paz, R& pdu) {
            const R y = rsqrt_nr(live ? r2 : (R)1);
            const R r = r2 * y;
            const R gi = spline_dw<KERN>(r * hinvi) * normi;
            const R gj = spline_dw<KERN>(r * shinv[t]) * snorm[t];
            const R gbar = (R)0.5 * (gi + gj);
            const R ex = dx * y, ey = dy * y, ez = dz * y;
            const R w = (vxi - svx[t]) * ex + (vyi - svy[t]) * ey + (vzi - svz[t]) * ez;
            const R mu = w < (R)0 ? w : (R)0;
            const R vs = ci + sc[t] - (R)3 * mu;
            // Pi = -(alpha_bar / 2) v_sig mu / rho_bar = -alpha_bar v_sig mu / (rho_i + rho_j)
            const R visc = -(hali + sal[t]) * vs * mu * rcp_nr(rhoi + srho[t]);
            const R mj = sm[t];
            const R Agi = Ai * gi;
            R coef = mj * fma(visc, gbar, fma(sA[t], gj, Agi));
            R dui = mj * fma((R)0.5 * visc, gbar, Agi) * w;
            coef = live ? coef : (R)0;
            dui = live ? dui : (R)0;
            pax = fma(-coef, ex, pax);
            pay = fma(-coef, ey, pay);
            paz = fma(-coef, ez, paz);
            pdu = pdu + dui;
            const R vcand = live ? vs : vsig;
            vsig = vcand > vsig ? vcand : vsig;
        };

        auto compute = [&](int count, int chunk) {
            if (!act) return;
            R pax = 0, pay = 0, paz = 0, pdu = 0;
            if constexpr (MASKED) {
                for (int t = sl; t < count; t += tpi) {
                    const R dx = xi - sx[t];
                    const R dy = yi - sy[t];
                    const R dz = zi - sz[t];
                    const R r2 = dx * dx + dy * dy + dz * dz;
                    const bool pair = r2 < fmax(H2i, sH2[t]) && (r2 > (R)0 || sj[t] != pi);
                    cnt += pair ? 1 : 0;
                    term(t, dx, dy, dz, r2, pair && r2 > (R)0, pax, pay, paz, pdu);
                }
            } else {
                // candidates of this lane that can be pairs: the density loop's hit
                // masks when they cover this window (a superset: every force pair lies
                // within twice the cell cap), else a test of every candidate
                uint64_t hits = 0;
                if (reuse && chunk < kMaskChunks) {
                    hits = use_spans ? cmask : a.item_masks[((int64_t)item * kMaskChunks + chunk) * kWave + lane];
                } else {
                    hits = lane_mask(count, sl, tpi, [&](int t) {
                        const R dx = xi - sx[t];
                        const R dy = yi - sy[t];
                        const R dz = zi - sz[t];
                        return fma(dz, dz, fma(dy, dy, dx * dx)) * shrink < fmax(H2i, sH2[t]);
                    });
                }
                while (hits) {
                    const int kk = __builtin_ctzll(hits);
                    hits &= hits - 1;
                    const int t = sl + kk * tpi;
                    const R dx = xi - sx[t];
                    const R dy = yi - sy[t];
                    const R dz = zi - sz[t];
                    const R r2 = dx * dx + dy * dy + dz * dz;
                    if (!(r2 < fmax(H2i, sH2[t]))) continue;
                    if (r2 > (R)0) {
                        ++cnt;
                        term(t, dx, dy, dz, r2, true, pax, pay, paz, pdu);
                    } else {
                        cnt += sj[t] != pi ? 1 : 0;   // coincident neighbour: counted, no force
                    }
                }
            }
            if constexpr (FP32) {
                neumaier(fax, cax, pax);
                neumaier(fay, cay, pay);
                neumaier(faz, caz, paz);
                neumaier(fdu, cdu, pdu);
            } else {
                ax += pax;
                ay += pay;
                az += paz;
                du += pdu;
            }
        };

        if (use_spans) run_window(spans, W, lane, fetch, put, compute);
        else for_window(a, kx, ky, kz, gx, r, lane, stage, compute);

        if constexpr (FP32) {
            ax = (double)fax + (double)cax;
            ay = (double)fay + (double)cay;
            az = (double)faz + (double)caz;
            du = (double)fdu + (double)cdu;
        }
        double vs_d = (double)vsig;
        if (tpi > 1) {
            red[0][lane] = ax;
            red[1][lane] = ay;
            red[2][lane] = az;
            red[3][lane] = du;
            redv[lane] = vs_d;
            redc[lane] = cnt;
            __syncthreads();
            if (act && sl == 0) {
                const int b = il * tpi;
                ax = ay = az = du = 0.0;
                cnt = 0;
                for (int k = 0; k < tpi; ++k) {
                    ax += red[0][b + k];
                    ay += red[1][b + k];
                    az += red[2][b + k];
                    du += red[3][b + k];
                    vs_d = redv[b + k] > vs_d ? redv[b + k] : vs_d;
                    cnt += redc[b + k];
                }
            }
            __syncthreads();
        }
        if (act && sl == 0) {
            st_f64(a.f[SPHV_AX], li, ax);
            st_f64(a.f[SPHV_AY], li, ay);
            st_f64(a.f[SPHV_AZ], li, az);
            st_f64(a.f[SPHV_UDT], li, du);
            st_f64(a.f[SPHV_VSIG], li, vs_d);
            n_pairs += (unsigned long long)cnt;
            if (!(isfinite(ax) && isfinite(ay) && isfinite(az) && isfinite(du))) flags |= SPHV_F_NONFINITE_OUTPUT;
        }
    }

    n_pairs = wave_sum_u64(n_pairs);
    for (int off = 32; off > 0; off >>= 1) flags |= __shfl_xor(flags, off, kWave);
    if (lane == 0) leave_part(a.part, (int64_t)n_pairs, 0, 0, flags);
}

// ============================================ time step and conservation sums

struct RedArgs {
    FieldRef in[6];     // m vx vy vz u h   (records through the index, or the view)
    FieldRef out[5];    // ax ay az u_dt v_sig (view or records)
    Access rec;
    Access outacc;
    DevState* state;
    double* part;       // [nblocks][16]
    int64_t n;
    double cfl;
};

constexpr int kRedThreads = 256;

template <bool DIRECT_OUT>
__global__ __launch_bounds__(kRedThreads) void k_reduce_part(RedArgs r)
{
    __shared__ double lds[9][kRedThreads];
    const int64_t base = (int64_t)blockIdx.x * kRedBlock;
    double s[9];
    for (int k = 0; k < 8; ++k) s[k] = 0.0;
    s[8] = INFINITY;                          // min h / v_sig
    for (int k = 0; k < kRedBlock / kRedThreads; ++k) {
        const int64_t p = base + (int64_t)threadIdx.x * (kRedBlock / kRedThreads) + k;
        if (p >= r.n) break;
        const Loc<true> lr = locate<true>(r.rec, p);
        const Loc<DIRECT_OUT> lo = locate<DIRECT_OUT>(r.outacc, p);
        const double m = ld_f64(r.in[0], lr);
        const double vx = ld_f64(r.in[1], lr), vy = ld_f64(r.in[2], lr), vz = ld_f64(r.in[3], lr);
        const double u = ld_f64(r.in[4], lr), h = ld_f64(r.in[5], lr);
        const double ax = ld_f64(r.out[0], lo), ay = ld_f64(r.out[1], lo), az = ld_f64(r.out[2], lo);
        const double du = ld_f64(r.out[3], lo), vs = ld_f64(r.out[4], lo);
        s[0] += m * vx;
        s[1] += m * vy;
        s[2] += m * vz;
        s[3] += m * (0.5 * (vx * vx + vy * vy + vz * vz) + u);
        s[4] += m * ax;
        s[5] += m * ay;
        s[6] += m * az;
        s[7] += m * (vx * ax + vy * ay + vz * az + du);
        const double q = h / vs;
        s[8] = q < s[8] ? q : s[8];
    }
    for (int k = 0; k < 9; ++k) lds[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int k = 0; k < 8; ++k) lds[k][threadIdx.x] += lds[k][threadIdx.x + w];
            const double o = lds[8][threadIdx.x + w];
            lds[8][threadIdx.x] = o < lds[8][threadIdx.x] ? o : lds[8][threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x < 9) r.part[(int64_t)blockIdx.x * 16 + threadIdx.x] = lds[threadIdx.x][0];
}

// k_reduce_part with the records' members staged through LDS: the block's
// kRedBlock particles in rounds of kStageThreads, thread t taking particles
// base + t, base + t + kStageThreads, ...; then the same tree as above.
template <bool DIRECT_OUT, bool IN_VIEW>
__global__ __launch_bounds__(kStageThreads) void k_reduce_staged(RedArgs r, StagePlan sp)
{
    extern __shared__ uint4 tile[];
    __shared__ double lds[9][kStageThreads];
    const int64_t base = (int64_t)blockIdx.x * kRedBlock;
    double s[9];
    for (int k = 0; k < 8; ++k) s[k] = 0.0;
    s[8] = INFINITY;                          // min h / v_sig
    for (int round = 0; round < kRedBlock / kStageThreads; ++round) {
        const int64_t r0 = base + (int64_t)round * kStageThreads;
        if (r0 >= r.n) break;                 // the same for the whole block
        if constexpr (!IN_VIEW) stage_in(tile, r.in[0].base, r.rec.stride, r.rec.index, r0, r.n, sp);
        const int64_t p = r0 + threadIdx.x;
        if (p < r.n) {
            const Loc<DIRECT_OUT> lo = locate<DIRECT_OUT>(r.outacc, p);
            double in6[6];
            if constexpr (IN_VIEW) {
                // the inputs are members of the view, in the outputs' slots
#pragma unroll
                for (int k = 0; k < 6; ++k) in6[k] = ld_f64(r.in[k], lo);
            } else {
                const LocTile lr{(char*)&tile[threadIdx.x * sp.nch] - (uint64_t)sp.c0 * 16};
#pragma unroll
                for (int k = 0; k < 6; ++k) in6[k] = ld_f64(r.in[k], lr);
            }
            const double m = in6[0], vx = in6[1], vy = in6[2], vz = in6[3], u = in6[4], h = in6[5];
            const double ax = ld_f64(r.out[0], lo), ay = ld_f64(r.out[1], lo), az = ld_f64(r.out[2], lo);
            const double du = ld_f64(r.out[3], lo), vs = ld_f64(r.out[4], lo);
            s[0] += m * vx;
            s[1] += m * vy;
            s[2] += m * vz;
            s[3] += m * (0.5 * (vx * vx + vy * vy + vz * vz) + u);
            s[4] += m * ax;
            s[5] += m * ay;
            s[6] += m * az;
            s[7] += m * (vx * ax + vy * ay + vz * az + du);
            const double q = h / vs;
            s[8] = q < s[8] ? q : s[8];
        }
        __syncthreads();                      // the tile is reloaded next round
    }
    for (int k = 0; k < 9; ++k) lds[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int w = kStageThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int k = 0; k < 8; ++k) lds[k][threadIdx.x] += lds[k][threadIdx.x + w];
            const double o = lds[8][threadIdx.x + w];
            lds[8][threadIdx.x] = o < lds[8][threadIdx.x] ? o : lds[8][threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x < 9) r.part[(int64_t)blockIdx.x * 16 + threadIdx.x] = lds[threadIdx.x][0];
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_final(RedArgs r, int64_t nb)
{
    __shared__ double lds[9][kRedThreads];
    double s[9];
    for (int k = 0; k < 8; ++k) s[k] = 0.0;
    s[8] = INFINITY;
    for (int64_t b = threadIdx.x; b < nb; b += kRedThreads) {
        for (int k = 0; k < 8; ++k) s[k] += r.part[b * 16 + k];
        const double q = r.part[b * 16 + 8];
        s[8] = q < s[8] ? q : s[8];
    }
    for (int k = 0; k < 9; ++k) lds[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int k = 0; k < 8; ++k) lds[k][threadIdx.x] += lds[k][threadIdx.x + w];
            const double o = lds[8][threadIdx.x + w];
            lds[8][threadIdx.x] = o < lds[8][threadIdx.x] ? o : lds[8][threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        DevState* st = r.state;
        for (int k = 0; k < 8; ++k) st->sums[k] = lds[k][0];
        const double dt = r.cfl * lds[8][0];
        st->t = st->t + st->dt;          // time of the current positions
        st->dt_prev = st->dt;
        st->dt = dt;
        st->nstep = st->nstep + 1;
        if (!(isfinite(dt) && dt > 0.0)) atomicOr(&st->flags, (uint32_t)SPHV_F_NONFINITE_OUTPUT);
    }
}

}  // namespace

// Folds the per-wave counters of the pair loop that ran just before on the same
// stream into the state block and rearms its queue for the next launch.  One
// workgroup; integer sums, maxima and ors do not depend on the order.
constexpr int kFoldThreads = 256;

__global__ __launch_bounds__(kFoldThreads) void k_pair_fold(int32_t* meta, int qhead, const int64_t* part,
                                                             int nblocks, DevState* st, int density)
{
    __shared__ unsigned long long s0[kFoldThreads / kWave], s1[kFoldThreads / kWave];
    __shared__ int s2[kFoldThreads / kWave];
    __shared__ uint32_t s3[kFoldThreads / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    unsigned long long c0 = 0, c1 = 0;
    int c2 = 0;
    uint32_t c3 = 0;
    for (int b = t; b < nblocks; b += kFoldThreads) {
        const int64_t* p = part + (int64_t)b * kPartSlots;
        c0 += (unsigned long long)p[0];
        c1 += (unsigned long long)p[1];
        c2 = (int)p[2] > c2 ? (int)p[2] : c2;
        c3 |= (uint32_t)p[3];
    }
    for (int off = 32; off > 0; off >>= 1) {
        c0 += __shfl_xor(c0, off, kWave);
        c1 += __shfl_xor(c1, off, kWave);
        const int o2 = __shfl_xor(c2, off, kWave);
        c2 = o2 > c2 ? o2 : c2;
        c3 |= __shfl_xor(c3, off, kWave);
    }
    if (lane == 0) {
        s0[w] = c0;
        s1[w] = c1;
        s2[w] = c2;
        s3[w] = c3;
    }
    __syncthreads();
    if (t == 0) {
        for (int k = 1; k < kFoldThreads / kWave; ++k) {
            c0 += s0[k];
            c1 += s1[k];
            c2 = s2[k] > c2 ? s2[k] : c2;
            c3 |= s3[k];
        }
        if (density) {
            st->pairs_density += c0;
            st->pair_evals_density += c1;
            if (c2 > st->max_iters) st->max_iters = c2;
        } else {
            st->pairs_force += c0;
        }
        st->pairs_total += c0;
        st->flags |= c3;
    }
    if (t < kNumXcd) meta[qhead + t * kQStride] = 0;
}

hipError_t launch_pair_fold(const PairArgs& a, int nblocks, int density, hipStream_t s)
{
    hipLaunchKernelGGL(k_pair_fold, dim3(1), dim3(kFoldThreads), 0, s, a.meta, a.qhead, (const int64_t*)a.part,
                       nblocks, a.state, density);
    return hipGetLastError();
}

int pair_grid_blocks(int64_t max_items)
{
    // persistent grid: at most enough single-wave workgroups to fill 256 CUs
    // several times over, a multiple of the 8 XCDs
    int64_t b = kMaxPairBlocks;
    if (max_items < b) b = (max_items + kNumXcd - 1) / kNumXcd * kNumXcd;
    if (b < kNumXcd) b = kNumXcd;
    return (int)b;
}

// Workgroups of a pair kernel that the device holds at once (its occupancy
// times the compute units), a multiple of the 8 XCDs; queried once per kernel.
template <class K>
int resident_blocks(K kernel, std::atomic<int>& cache)
{
    int v = cache.load(std::memory_order_relaxed);
    if (v > 0) return v;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || cus < 1)
        cus = 256;
    v = per_cu * cus / kNumXcd * kNumXcd;
    if (v < kNumXcd) v = kNumXcd;
    cache.store(v, std::memory_order_relaxed);
    return v;
}

// Launches one instance with no more workgroups than the device holds at once
// (a persistent grid gains nothing from waves that start after the queue has
// drained), then the fold of its counters.
template <class K>
hipError_t launch_pair(K kernel, std::atomic<int>& cache, const PairArgs& a0, int density, hipStream_t s)
{
    PairArgs a = a0;
    const int res = resident_blocks(kernel, cache);
    if (a.nblocks > res) a.nblocks = res;
    hipLaunchKernelGGL(kernel, dim3((unsigned)a.nblocks), dim3(kWave), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pair_fold, dim3(1), dim3(kFoldThreads), 0, s, a.meta, a.qhead, (const int64_t*)a.part,
                       a.nblocks, a.state, density);
    return hipGetLastError();
}

#define SPHV_PAIR_CASE(KERNEL, D, F, M, DENS)                                     \
    do {                                                                          \
        if (kern == SPHV_KERNEL_QUARTIC) {                                        \
            static std::atomic<int> cache_q{0};                                   \
            return launch_pair(KERNEL<D, F, M, SPHV_KERNEL_QUARTIC>, cache_q, a, DENS, s); \
        }                                                                         \
        static std::atomic<int> cache{0};                                         \
        return launch_pair(KERNEL<D, F, M, SPHV_KERNEL_CUBIC>, cache, a, DENS, s); \
    } while (0)

#define SPHV_PAIR_DISPATCH(KERNEL, DENS)                                          \
    do {                                                                          \
        if (direct) {                                                             \
            if (fp32) {                                                           \
                if (masked) SPHV_PAIR_CASE(KERNEL, true, true, true, DENS);       \
                SPHV_PAIR_CASE(KERNEL, true, true, false, DENS);                  \
            }                                                                     \
            if (masked) SPHV_PAIR_CASE(KERNEL, true, false, true, DENS);          \
            SPHV_PAIR_CASE(KERNEL, true, false, false, DENS);                     \
        }                                                                         \
        if (fp32) {                                                               \
            if (masked) SPHV_PAIR_CASE(KERNEL, false, true, true, DENS);          \
            SPHV_PAIR_CASE(KERNEL, false, true, false, DENS);                     \
        }                                                                         \
        if (masked) SPHV_PAIR_CASE(KERNEL, false, false, true, DENS);             \
        SPHV_PAIR_CASE(KERNEL, false, false, false, DENS);                        \
    } while (0)

hipError_t launch_density(const PairArgs& a, int direct, int fp32, int masked, int kern, hipStream_t s)
{
    SPHV_PAIR_DISPATCH(k_density, 1);
}

hipError_t launch_force(const PairArgs& a, int direct, int fp32, int masked, int kern, hipStream_t s)
{
    SPHV_PAIR_DISPATCH(k_force, 0);
}

hipError_t launch_force_reduce(const FieldRef* in6, const Access& rec, const FieldRef* out5, const Access& outacc,
                               int out_direct, int in_view, DevState* st, double cfl, int64_t n,
                               double* partials, hipStream_t s)
{
    RedArgs r;
    for (int k = 0; k < 6; ++k) r.in[k] = in6[k];
    for (int k = 0; k < 5; ++k) r.out[k] = out5[k];
    r.rec = rec;
    r.outacc = outacc;
    r.state = st;
    r.part = partials;
    r.n = n;
    r.cfl = cfl;
    int64_t nb = (n + kRedBlock - 1) / kRedBlock;
    if (nb < 1) nb = 1;
    StagePlan sp{};
    if (in_view && !out_direct) {
        // inputs and outputs in the view: the staged kernel's order, nothing staged
        hipLaunchKernelGGL((k_reduce_staged<false, true>), dim3((unsigned)nb), dim3(kStageThreads), 0, s, r, sp);
    } else if (n > 0 && !r.rec.ptrs && plan_stage(r.in, 6, 0u, r.rec.stride, &sp)) {
        const size_t lds = kStageThreads * sp.nch * 16;
        if (out_direct)
            hipLaunchKernelGGL((k_reduce_staged<true, false>), dim3((unsigned)nb), dim3(kStageThreads), lds, s, r,
                               sp);
        else
            hipLaunchKernelGGL((k_reduce_staged<false, false>), dim3((unsigned)nb), dim3(kStageThreads), lds, s, r,
                               sp);
    } else if (out_direct) {
        hipLaunchKernelGGL(k_reduce_part<true>, dim3((unsigned)nb), dim3(kRedThreads), 0, s, r);
    } else {
        hipLaunchKernelGGL(k_reduce_part<false>, dim3((unsigned)nb), dim3(kRedThreads), 0, s, r);
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, s, r, nb);
    return hipGetLastError();
}

}  // namespace sphv
