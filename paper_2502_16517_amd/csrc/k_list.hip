// Pair loops over per-particle neighbour lists (the list walk), an alternative
// to the item kernels of k_pair.hip selected by sphv_params.list_cap > 0.
//
// Mapping onto gfx950: one lane per local particle i (view element p = sorted
// position), 64 consecutive particles per wave, waves over the particles in a
// grid-stride loop.  Apart from the builds' coherent waves, no LDS and no
// barriers: every lane is independent, so the kernels hold many waves per
// SIMD to hide the latency of the candidate and list loads, which the L1/L2
// serve (neighbouring lanes read neighbouring cells).
//  * Build: the lane walks the active set of its particle -- the (2R+1)^3
//    cells around its own cell (paper Sec. 2.3: local vs active particles) --
//    in a fixed order (dz, dy, then the row's cells along x, wrapped part
//    first) and appends every candidate within its list radius to its list
//    (entry k of particle p at list[k n + p], so that a wave's k-th entries
//    are one contiguous 256-byte run).  A wave whose particles share one
//    dense cell walks that cell's window once for all of them, staging the
//    candidates in LDS (walk_wave).
//  * Evaluation: the lane walks its list in order, so every pair is evaluated
//    with no divergence between lanes other than list lengths.
//  * Density: one list (radius 2 h_l, h_l = min(h_cap, (1 + 1/16) h_0)) serves
//    every Newton pass.  Should h leave h_l, or the list overflow its capacity,
//    the lane evaluates its remaining passes over the whole window (the same
//    candidates in the same order, so the same sums), without the list.
//  * Force: the list holds exactly the pairs r < 2 max(h_i, h_j) at the
//    converged h; a lane whose pairs overflow the list evaluates them in a
//    second walk.  The per-particle constants that need a division or a root
//    (A = P / (Omega rho^2), c, 1/h, the kernel norm) are computed once per
//    particle by k_force_prep, not once per pair.
//  * Periodic images: minimum-image differences on the FP64 positions; in FP32
//    the candidate's cell-relative position is moved to the local cell's frame
//    by the nearest-image cell offset, exactly as the item kernels stage it.
//  * Every sum runs over the pairs in list (= window) order, so results are
//    deterministic; the outputs do not depend on the layout of the view.
#include <atomic>
#include <type_traits>

#include "k_common.h"

namespace sphv {

namespace {

constexpr double kPiL = 3.14159265358979323846;
constexpr double kGrowL = 1.0 + 1.0 / 16.0;   // list radius over the initial h

__device__ __forceinline__ void neumaier_l(float& s, float& c, float x)
{
    float t = s + x;
    c += (fabsf(s) >= fabsf(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
}

// The smoothing kernels (truncated-power form, branch free; W = w(q)/(pi h^3)):
// cubic M4 w = (2-q)_+^3/4 - (1-q)_+^3; quartic M5 w = k((2-q)_+^4 - 5(1.2-q)_+^4
// + 10(0.4-q)_+^4), k = 15625/65536, its knots scaled to the support 2h.
template <int KERN, class R>
__device__ __forceinline__ void spl(R q, R& w, R& dw)
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
__device__ __forceinline__ R spl_dw(R q)
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

// 1/sqrt(x) for normal x > 0: hardware estimate and Newton-Raphson steps
// y <- y (3/2 - x y^2 / 2) (two in double, one in float).
__device__ __forceinline__ double rsq_l(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx, y * y, 1.5);
    y = y * fma(-hx, y * y, 1.5);
    return y;
}

__device__ __forceinline__ float rsq_l(float x)
{
    float y = __builtin_amdgcn_rsqf(x);
    const float hx = 0.5f * x;
    return y * fmaf(-hx, y * y, 1.5f);
}

// 1/d: hardware estimate and Newton-Raphson steps y <- y + y (1 - d y).
__device__ __forceinline__ double rcp_l(double d)
{
    double y = __builtin_amdgcn_rcp(d);
    double e = fma(-d, y, 1.0);
    y = fma(y, e, y);
    e = fma(-d, y, 1.0);
    return fma(y, e, y);
}

__device__ __forceinline__ float rcp_l(float d)
{
    float y = __builtin_amdgcn_rcpf(d);
    return fmaf(y, fmaf(-d, y, 1.0f), y);
}

template <class R> struct TinyL;
template <> struct TinyL<double> { static constexpr double v = 1e-300; };
template <> struct TinyL<float> { static constexpr float v = 1e-30f; };

// Per-axis reach of one particle's window (reach R of its cell), narrowed on a
// periodic axis too short for 2R+1 cells (flagged).
__device__ __forceinline__ void lane_reach(const Geom& g, int R, int r[3], uint32_t& flags)
{
    for (int d = 0; d < 3; ++d) {
        r[d] = R;
        if (g.periodic[d] && 2 * R + 1 > g.n[d]) {
            r[d] = (g.n[d] - 1) / 2;
            flags |= SPHV_F_GRID_TOO_SMALL;
        }
    }
}

// Minimum-image difference a - b along axis d: the nearest periodic image on
// a periodic axis (within half a box length), the plain difference otherwise.
__device__ __forceinline__ double mi_diff(double a, double b, const Geom& g, int d)
{
    double dx = a - b;
    if (g.periodic[d]) {
        const double half = 0.5 * g.len[d];
        dx = dx > half ? dx - g.len[d] : (dx < -half ? dx + g.len[d] : dx);
    }
    return dx;
}

// Nearest-image cell offset k_j - k_i along axis d (|offset| <= n/2 on a
// periodic axis; within a window of reach r <= (n-1)/2 it is the window's).
__device__ __forceinline__ int mi_cell(int kj, int ki, const Geom& g, int d)
{
    int dk = kj - ki;
    if (g.periodic[d]) {
        const int n = g.n[d];
        dk = 2 * dk > n ? dk - n : (2 * dk < -n ? dk + n : dk);
    }
    return dk;
}

// FP32 position member of element l along axis d, relative to the corner of
// cell k_d: an FP32 view stores it so; a record's double is converted as the
// gather converts it.
template <class L>
__device__ __forceinline__ float ld_rel(const FieldRef& f, const L& l, const Geom& g, int d, int k)
{
    if (f.dtype == SPHV_F32) return *(const float*)l.at(f);
    const double v = *(const double*)l.at(f);
    const double o = __dadd_rn(g.lo[d], __dmul_rn((double)k, g.cell[d]));
    return __double2float_rn(__dsub_rn(v, o));
}

// Any other member as float (an FP32 view's float, or a double rounded).
template <class L>
__device__ __forceinline__ float ld_f32v(const FieldRef& f, const L& l)
{
    if (f.dtype == SPHV_F32) return *(const float*)l.at(f);
    return __double2float_rn(*(const double*)l.at(f));
}

template <class R, class L>
__device__ __forceinline__ R ld_r(const FieldRef& f, const L& l)
{
    if constexpr (std::is_same<R, float>::value) return ld_f32v(f, l);
    else return ld_f64(f, l);
}

// Candidate position relative to the local particle's frame: FP64 absolute
// (differences by minimum image), FP32 relative to the local cell's corner.
template <bool DIRECT, bool FP32>
struct Pos;

template <bool DIRECT>
struct Pos<DIRECT, false> {
    double x, y, z;
    __device__ __forceinline__ void load(const PairArgs& a, const Loc<DIRECT>& l, int, int, int)
    {
        x = ld_f64(a.f[SPHV_X], l);
        y = ld_f64(a.f[SPHV_Y], l);
        z = ld_f64(a.f[SPHV_Z], l);
    }
};

template <bool DIRECT>
struct Pos<DIRECT, true> {
    float x, y, z;
    // (ox, oy, oz): the candidate's nearest-image cell offset from the local cell
    __device__ __forceinline__ void load(const PairArgs& a, const Loc<DIRECT>& l, int jx, int jy, int jz, int ox,
                                         int oy, int oz)
    {
        x = ld_rel(a.f[SPHV_X], l, a.g, 0, jx) + __double2float_rn((double)ox * a.g.cell[0]);
        y = ld_rel(a.f[SPHV_Y], l, a.g, 1, jy) + __double2float_rn((double)oy * a.g.cell[1]);
        z = ld_rel(a.f[SPHV_Z], l, a.g, 2, jz) + __double2float_rn((double)oz * a.g.cell[2]);
    }
};

// Squared distance between the local particle (xi, yi, zi) and candidate c,
// and the components of x_i - x_j.
template <bool FP32, class P, class R>
__device__ __forceinline__ R diff(const PairArgs& a, R xi, R yi, R zi, const P& c, R& dx, R& dy, R& dz)
{
    if constexpr (FP32) {
        dx = xi - c.x;
        dy = yi - c.y;
        dz = zi - c.z;
    } else {
        dx = mi_diff(xi, c.x, a.g, 0);
        dy = mi_diff(yi, c.y, a.g, 1);
        dz = mi_diff(zi, c.z, a.g, 2);
    }
    return dx * dx + dy * dy + dz * dz;
}

// Bounds of each run of kBlock sorted positions (the last run may be
// shorter): the lower and upper corner of its particles' positions in the box
// frame (FP64; an FP32 view's cell-relative coordinates are moved back by
// their cell's corner and the box widened by their rounding) and its largest
// 2h.  A dense cell (more than kDense particles, ordered by sub-cell) holds
// compact runs, so the window walks skip runs that lie out of reach.
template <bool DIRECT, bool FP32>
__global__ __launch_bounds__(kWave) void k_block_bounds(PairArgs a, double* out)
{
    // one wave covers kWave / kBlock runs, each reduced over its own kBlock lanes
    static_assert(kWave % kBlock == 0, "runs tile a wave");
    const int64_t p = (int64_t)blockIdx.x * kWave + threadIdx.x;
    const bool valid = p < a.n;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, H = 0.0;
    if (valid) {
        const Loc<DIRECT> l = locate<DIRECT>(a.acc, p);
        double x[3];
        if constexpr (FP32) {
            int k[3];
            cell_coords(a.key_sorted[p], a.g, k[0], k[1], k[2]);
            const int roles[3] = {SPHV_X, SPHV_Y, SPHV_Z};
            for (int d = 0; d < 3; ++d) {
                const double o = __dadd_rn(a.g.lo[d], __dmul_rn((double)k[d], a.g.cell[d]));
                const double v = (double)ld_rel(a.f[roles[d]], l, a.g, d, k[d]) + o;
                const double e = a.g.cell[d] * 0x1p-20;      // far above the float rounding of the offset
                lo[d] = v - e;
                hi[d] = v + e;
            }
        } else {
            x[0] = ld_f64(a.f[SPHV_X], l);
            x[1] = ld_f64(a.f[SPHV_Y], l);
            x[2] = ld_f64(a.f[SPHV_Z], l);
            for (int d = 0; d < 3; ++d) lo[d] = hi[d] = x[d];
        }
        H = 2.0 * (FP32 ? (double)ld_f32v(a.f[SPHV_H], l) : ld_f64(a.f[SPHV_H], l));
    }
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(lo[d], __shfl_xor(lo[d], off, kWave));
            hi[d] = fmax(hi[d], __shfl_xor(hi[d], off, kWave));
        }
        H = fmax(H, __shfl_xor(H, off, kWave));
    }
    if (valid && threadIdx.x % kBlock == 0) {
        double* o = out + (p / kBlock) * kBlockWords;
        for (int d = 0; d < 3; ++d) {
            o[d] = lo[d];
            o[3 + d] = hi[d];
        }
        o[6] = H;
        o[7] = 0.0;
    }
}

// Distance from coordinate p to the slab of cell index k (not wrapped: the
// window's own image) along axis d.
__device__ __forceinline__ double slab_dist(double p, int k, const Geom& g, int d)
{
    const double lo = g.lo[d] + (double)k * g.cell[d];
    return fmax(fmax(lo - p, p - (lo + g.cell[d])), 0.0);
}

// The window's offsets -r..r along an axis, taken from index t0 on (wrapping
// round), visit the cells in ascending order of their wrapped index: on a
// periodic axis whose window wraps, the offsets that wrap come last (low
// wrap) or first (high wrap).
__device__ __forceinline__ int rot_start(int k, int r, int n, int periodic)
{
    if (!periodic) return 0;
    if (k - r < 0) return r - k;              // offset -k has cell 0
    if (k + r >= n) return n - k + r;         // offset n-k wraps to cell 0
    return 0;
}

__device__ __forceinline__ int rot_offset(int t, int t0, int r)
{
    int q = t + t0;
    if (q > 2 * r) q -= 2 * r + 1;
    return q - r;
}

// Walks the window of cell (kx, ky, kz) with per-axis reach r in a fixed
// order, ascending in the cells' keys and so in sorted position (z, then y,
// then x, each from the lowest wrapped index up), and calls
// visit(j, jx, jy, jz, ox, oy, oz) for every candidate j
// (sorted position) of cell (jx, jy, jz), (ox, oy, oz) being that cell's
// offset from the local cell in the window.  Candidates that cannot be within
// reach of the local particle at (px, py, pz) (box frame) are skipped, in the
// same way for every walk of that particle: a row of cells whose (y, z)
// distance d2 fails keep_cell(d2, -1), a cell whose box distance fails
// keep_cell(d2, key), and, in a cell of more than kDense particles with block
// bounds given, a run of kBlock sorted positions whose bounds fail
// keep_block(bounds, sx, sy, sz), (sx, sy, sz) being the periodic shift of the
// cell's image.
// walk_window_runs hands visit_run(j0, j1, jx, jy, jz, ox, oy, oz) each run of
// consecutive sorted positions [j0, j1) it keeps, in the same order.
//
// With SEG (for visits that do not need the candidates' cells) the cells of a
// row that the row's bound keeps, keep_cell(d2, -1), are consecutive in x
// (the box distance falls, then rises, along the row) and so are their
// candidates in sorted position: the row's kept range of cells (two pieces
// when it wraps round a periodic x axis) is then one run, read from two cell
// offsets instead of two per cell, whenever it holds at most kSeg candidates
// (so no cell of it is dense).  A longer range is walked cell by cell as
// without SEG.  The run's candidates are a superset of those the cells would
// give (all those within the row bound), in the same order; such a run is
// handed over with jx = -1 and ox the window offset of the row's cell 0
// (run_cell gives each candidate's cell and offset).  In sparse regions,
// where a window spans many cells with few particles, this replaces most of
// the walk's dependent loads.
constexpr int kSeg = kDense;

template <bool SEG, class KC, class KB, class V>
__device__ __forceinline__ void walk_window_runs(const PairArgs& a, int kx, int ky, int kz, const int r[3],
                                                 double px, double py, double pz, KC&& keep_cell, KB&& keep_block,
                                                 V&& visit_run)
{
    const int nx = a.g.n[0], ny = a.g.n[1], nz = a.g.n[2];
    // offsets in the order that visits cells (so sorted positions) ascending
    const int t0z = rot_start(kz, r[2], nz, a.g.periodic[2]);
    const int t0y = rot_start(ky, r[1], ny, a.g.periodic[1]);
    for (int tz = 0; tz <= 2 * r[2]; ++tz) {
        const int dz = rot_offset(tz, t0z, r[2]);
        int z2 = kz + dz;
        if (z2 < 0 || z2 >= nz) {
            if (!a.g.periodic[2]) continue;
            z2 += z2 < 0 ? nz : -nz;
        }
        const double ez = slab_dist(pz, kz + dz, a.g, 2);
        for (int ty = 0; ty <= 2 * r[1]; ++ty) {
            const int dy = rot_offset(ty, t0y, r[1]);
            int y2 = ky + dy;
            if (y2 < 0 || y2 >= ny) {
                if (!a.g.periodic[1]) continue;
                y2 += y2 < 0 ? ny : -ny;
            }
            const double ey = slab_dist(py, ky + dy, a.g, 1);
            const double dyz = fma(ey, ey, ez * ez);
            if (!keep_cell(dyz, -1)) continue;
            const int row = (z2 * ny + y2) * nx;
            // the row's offsets [da, db]: the whole window row, or with SEG the
            // offsets the row bound keeps, grown from a kept offset next to the
            // local cell (the one holding the particle, at distance 0) or found
            // by a scan of the window row
            int da = -r[0], db = r[0];
            if constexpr (SEG) {
                auto row_keeps = [&](int dx) {
                    const double ex = slab_dist(px, kx + dx, a.g, 0);
                    return keep_cell(fma(ex, ex, dyz), -1);
                };
                int d0 = 0;
                bool found = row_keeps(0);
                if (!found && r[0] >= 1) {
                    if (row_keeps(-1)) d0 = -1, found = true;
                    else if (row_keeps(1)) d0 = 1, found = true;
                }
                if (found) {
                    da = db = d0;
                    while (da > -r[0] && row_keeps(da - 1)) --da;
                    while (db < r[0] && row_keeps(db + 1)) ++db;
                } else {
                    int lo_k = r[0] + 1, hi_k = -r[0] - 1;
                    for (int dx = -r[0]; dx <= r[0]; ++dx)
                        if (row_keeps(dx)) {
                            lo_k = dx < lo_k ? dx : lo_k;
                            hi_k = dx;
                        }
                    if (lo_k > hi_k) continue;
                    da = lo_k;
                    db = hi_k;
                }
            }
            // those cells in unwrapped x, in at most two pieces of ascending
            // wrapped index, each with its shift s = unwrapped - wrapped
            int ua = kx + da, ub = kx + db;
            if (!a.g.periodic[0]) {
                ua = ua < 0 ? 0 : ua;
                ub = ub > nx - 1 ? nx - 1 : ub;
                if (ua > ub) continue;
            }
            int a0 = ua, b0 = ub, s0 = 0, a1 = 0, b1 = -1, s1 = 0;
            if (ub < 0) {
                a0 = ua + nx, b0 = ub + nx, s0 = -nx;
            } else if (ua >= nx) {
                a0 = ua - nx, b0 = ub - nx, s0 = nx;
            } else if (ua < 0) {
                a0 = 0, b0 = ub;
                a1 = ua + nx, b1 = nx - 1, s1 = -nx;
            } else if (ub >= nx) {
                a0 = 0, b0 = ub - nx, s0 = nx;
                a1 = ua, b1 = nx - 1;
            }
            for (int q = 0; q < 2; ++q) {
                const int xa = q ? a1 : a0, xb = q ? b1 : b0, sq = q ? s1 : s0;
                if (xa > xb) break;
                // with SEG, a piece of at most kSeg candidates is one run
                bool whole = false;
                int wb = 0, we = 0;
                if constexpr (SEG) {
                    wb = a.cell_start[row + xa];
                    we = a.cell_start[row + xb + 1];
                    whole = we - wb <= kSeg;
                }
                for (int x2 = xa; x2 <= xb; ++x2) {
                    const int dx = x2 + sq - kx;
                    int jb = wb, je = we;
                    bool dense = false;
                    if (!whole) {
                        const double ex = slab_dist(px, kx + dx, a.g, 0);
                        if (!keep_cell(fma(ex, ex, dyz), row + x2)) continue;
                        jb = a.cell_start[row + x2];
                        je = a.cell_start[row + x2 + 1];
                        dense = a.blocks && je - jb > kDense;
                    }
                    // the cell's runs of kBlock sorted positions when dense, else
                    // the cell (or the whole piece) as one run
                    for (int j0 = jb; j0 < je;) {
                        int j1 = je;
                        bool keep = true;
                        if (dense) {
                            const int bk = j0 / kBlock;
                            j1 = (bk + 1) * kBlock < je ? (bk + 1) * kBlock : je;
                            const double sx = sq > 0 ? a.g.len[0] : (sq < 0 ? -a.g.len[0] : 0.0);
                            const double sy = ky + dy - y2 > 0 ? a.g.len[1] : (ky + dy - y2 < 0 ? -a.g.len[1] : 0.0);
                            const double sz = kz + dz - z2 > 0 ? a.g.len[2] : (kz + dz - z2 < 0 ? -a.g.len[2] : 0.0);
                            keep = keep_block(a.blocks + (int64_t)bk * kBlockWords, sx, sy, sz);
                        }
                        if (keep) visit_run(j0, j1, whole ? -1 : x2, y2, z2, whole ? sq - kx : dx, dy, dz);
                        j0 = j1;
                    }
                    if (whole) break;
                }
            }
        }
    }
}

template <bool SEG, class KC, class KB, class V>
__device__ __forceinline__ void walk_window(const PairArgs& a, int kx, int ky, int kz, const int r[3], double px,
                                            double py, double pz, KC&& keep_cell, KB&& keep_block, V&& visit)
{
    walk_window_runs<SEG>(a, kx, ky, kz, r, px, py, pz, keep_cell, keep_block,
                     [&](int j0, int j1, int jx, int jy, int jz, int ox, int oy, int oz) {
                         for (int j = j0; j < j1; ++j) visit(j, jx, jy, jz, ox, oy, oz);
                     });
}

// Candidate j of a run handed over by walk_window_runs: its cell x index jx
// and window offset ox, read from its key when the run spans several cells of
// its row (jx < 0, ox the offset of the row's cell 0).
__device__ __forceinline__ void run_cell(const PairArgs& a, int j, int jy, int jz, int& jx, int& ox)
{
    if (jx >= 0) return;
    jx = a.key_sorted[j] - (jz * a.g.n[1] + jy) * a.g.n[0];
    ox += jx;
}

// The candidates j0 .. j1-1 of a run, their members loaded B at a time (all
// loads of a batch issued before any is used, so that a lane has several
// gathers in flight), then used one after the other in order.
template <int B, class Load, class Use>
__device__ __forceinline__ void batched(int j0, int j1, Load&& load, Use&& use)
{
    int j = j0;
    for (; j + B <= j1; j += B) {
        decltype(load(j)) v[B];
#pragma unroll
        for (int k = 0; k < B; ++k) v[k] = load(j + k);
#pragma unroll
        for (int k = 0; k < B; ++k) use(j + k, v[k]);
    }
    for (; j < j1; ++j) use(j, load(j));
}

// Squared distance from (px, py, pz) minus the shift to the box of a run's bounds.
__device__ __forceinline__ double box_d2(const double* bnd, double px, double py, double pz, double sx, double sy,
                                         double sz)
{
    const double p[3] = {px - sx, py - sy, pz - sz};
    double d2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double e = fmax(fmax(bnd[d] - p[d], p[d] - bnd[3 + d]), 0.0);
        d2 = fma(e, e, d2);
    }
    return d2;
}

// The local particle's position in the box frame, FP64: as stored, or an FP32
// view's cell-relative coordinate moved back by its cell's corner.
template <bool FP32, class R>
__device__ __forceinline__ double box_pos(R v, const Geom& g, int d, int k)
{
    if constexpr (FP32) return (double)v + __dadd_rn(g.lo[d], __dmul_rn((double)k, g.cell[d]));
    else return v;
}

// ------------------------------------------------------- coherent waves
//
// The 64 lanes of a list build are 64 consecutive sorted positions.  When they
// all lie in one dense cell (the core of a clustered distribution), each
// lane's own walk keeps a slightly different set of runs, and the wave pays
// for the union of them with one gather per candidate and lane.  Such a wave
// instead walks its shared window once: a row, cell or run of kBlock positions
// is kept when it can lie within reach of the lanes' bounding box (never
// closer than any lane, with the largest of their radii: a superset of every
// lane's own culling), its candidates are staged into LDS 64 at a time by the
// whole wave (one gather per candidate), and every lane tests every staged
// candidate in order.  A lane's hits are those of its own walk, in the same
// order.  (A wave that straddles two dense cells holds the last sub-cells of
// one, its far corner in sub-cell order, and the first of the next, its near
// corner: its box spans the cells' whole y and z extent, and walking the union
// of its lanes' windows together cost more than their own walks.)

struct WaveBox {
    double lo[3], hi[3];
};

__device__ __forceinline__ double wave_min_d(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, kWave));
    return v;
}

__device__ __forceinline__ double wave_max_d(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}

// The lanes' box-frame positions spanned (every lane active).
__device__ __forceinline__ WaveBox wave_box(double bx, double by, double bz)
{
    WaveBox w;
    const double b[3] = {bx, by, bz};
    for (int d = 0; d < 3; ++d) {
        w.lo[d] = wave_min_d(b[d]);
        w.hi[d] = wave_max_d(b[d]);
    }
    return w;
}

// A wave of the list builds is coherent when its 64 positions are particles of
// one cell of more than kDense particles (with run bounds built) whose window
// offsets fit the staging's 10-bit fields.
__device__ __forceinline__ bool wave_coherent(const PairArgs& a, int64_t p)
{
    const bool active = p < a.n;
    const int cell = active ? a.key_sorted[p] : -1;
    const int c0 = __builtin_amdgcn_readfirstlane(cell);
    if (!a.blocks || !__all(active && cell == c0)) return false;
    return a.cell_start[c0 + 1] - a.cell_start[c0] > kDense && a.reach[c0] < 512;
}

// Distance from the wave box's interval along axis d to the slab of cell k.
__device__ __forceinline__ double slab_dist_box(const WaveBox& w, int k, const Geom& g, int d)
{
    const double lo = g.lo[d] + (double)k * g.cell[d];
    return fmax(fmax(lo - w.hi[d], w.lo[d] - (lo + g.cell[d])), 0.0);
}

// Squared distance from the wave box, moved by minus the shift, to a run's bounds.
__device__ __forceinline__ double box_box_d2(const double* bnd, const WaveBox& w, double sx, double sy, double sz)
{
    const double s[3] = {sx, sy, sz};
    double d2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double e = fmax(fmax(bnd[d] - (w.hi[d] - s[d]), (w.lo[d] - s[d]) - bnd[3 + d]), 0.0);
        d2 = fma(e, e, d2);
    }
    return d2;
}

// The coherent wave's walk of the window of cell (kx, ky, kz): the same rows,
// cells and runs as walk_window_runs, in the same order, kept by the wave box:
// a row when its (y, z) distance is below rr_row, a cell when its distance is
// below cell_rr(key), a run of a dense cell when its bounds' distance is below
// run_rr(bounds) (the lanes test 64 runs at a time).  add_run(j0, j1, jx, jy,
// jz, ox, oy, oz) takes each kept run, j1 - j0 <= kWave.
template <class CR, class RR, class Add>
__device__ __forceinline__ void walk_wave(const PairArgs& a, int kx, int ky, int kz, const int r[3],
                                          const WaveBox& w, double rr_row, CR&& cell_rr, RR&& run_rr,
                                          Add&& add_run)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int nx = a.g.n[0], ny = a.g.n[1], nz = a.g.n[2];
    const int t0z = rot_start(kz, r[2], nz, a.g.periodic[2]);
    const int t0y = rot_start(ky, r[1], ny, a.g.periodic[1]);
    const int t0x = rot_start(kx, r[0], nx, a.g.periodic[0]);
    for (int tz = 0; tz <= 2 * r[2]; ++tz) {
        const int dz = rot_offset(tz, t0z, r[2]);
        int z2 = kz + dz;
        if (z2 < 0 || z2 >= nz) {
            if (!a.g.periodic[2]) continue;
            z2 += z2 < 0 ? nz : -nz;
        }
        const double ez = slab_dist_box(w, kz + dz, a.g, 2);
        for (int ty = 0; ty <= 2 * r[1]; ++ty) {
            const int dy = rot_offset(ty, t0y, r[1]);
            int y2 = ky + dy;
            if (y2 < 0 || y2 >= ny) {
                if (!a.g.periodic[1]) continue;
                y2 += y2 < 0 ? ny : -ny;
            }
            const double ey = slab_dist_box(w, ky + dy, a.g, 1);
            const double dyz = fma(ey, ey, ez * ez);
            if (!(dyz < rr_row * rr_row)) continue;
            const int row = (z2 * ny + y2) * nx;
            for (int tx = 0; tx <= 2 * r[0]; ++tx) {
                const int dx = rot_offset(tx, t0x, r[0]);
                int x2 = kx + dx;
                if (x2 < 0 || x2 >= nx) {
                    if (!a.g.periodic[0]) continue;
                    x2 += x2 < 0 ? nx : -nx;
                }
                const double ex = slab_dist_box(w, kx + dx, a.g, 0);
                const double rc = cell_rr(row + x2);
                if (!(fma(ex, ex, dyz) < rc * rc)) continue;
                const int jb = __builtin_amdgcn_readfirstlane(a.cell_start[row + x2]);
                const int je = __builtin_amdgcn_readfirstlane(a.cell_start[row + x2 + 1]);
                if (jb >= je) continue;
                if (je - jb <= kDense) {
                    add_run(jb, je, x2, y2, z2, dx, dy, dz);
                    continue;
                }
                const double sx = kx + dx - x2 > 0 ? a.g.len[0] : (kx + dx - x2 < 0 ? -a.g.len[0] : 0.0);
                const double sy = ky + dy - y2 > 0 ? a.g.len[1] : (ky + dy - y2 < 0 ? -a.g.len[1] : 0.0);
                const double sz = kz + dz - z2 > 0 ? a.g.len[2] : (kz + dz - z2 < 0 ? -a.g.len[2] : 0.0);
                const int bfirst = jb / kBlock, blast = (je - 1) / kBlock;
                for (int b0 = bfirst; b0 <= blast; b0 += kWave) {
                    const int b = b0 + lane;
                    bool keep = false;
                    if (b <= blast) {
                        const double* bnd = a.blocks + (int64_t)b * kBlockWords;
                        const double rb = run_rr(bnd);
                        keep = box_box_d2(bnd, w, sx, sy, sz) < rb * rb;
                    }
                    for (uint64_t m = __ballot(keep); m; m &= m - 1) {
                        const int bb = b0 + __builtin_ctzll(m);
                        const int j0 = bb * kBlock > jb ? bb * kBlock : jb;
                        const int j1 = (bb + 1) * kBlock < je ? (bb + 1) * kBlock : je;
                        add_run(j0, j1, x2, y2, z2, dx, dy, dz);
                    }
                }
            }
        }
    }
}

// The staging of a coherent wave's candidates: runs are appended to a chunk of
// at most kWave candidates (their sorted positions, and for an FP32 view their
// cell and window offset); a full chunk, and the last one, is staged by the
// wave (stage(t, j, jx, jy, jz, ox, oy, oz) by lane t) and then taken by every
// lane in order (use(t, j)).
struct WaveChunk {
    int j[kWave];
    int key[kWave];
    int off[kWave];
};

template <bool FP32, class Stage, class Use>
struct WaveRuns {
    const PairArgs& a;
    WaveChunk& c;
    Stage& stage;
    Use& use;
    int fill = 0;

    __device__ __forceinline__ WaveRuns(const PairArgs& a_, WaveChunk& c_, Stage& s_, Use& u_)
        : a(a_), c(c_), stage(s_), use(u_)
    {
    }

    __device__ __forceinline__ void flush()
    {
        if (fill == 0) return;
        const int lane = threadIdx.x & (kWave - 1);
        __syncthreads();
        if (lane < fill) {
            int jx = 0, jy = 0, jz = 0, ox = 0, oy = 0, oz = 0;
            if constexpr (FP32) {
                cell_coords(c.key[lane], a.g, jx, jy, jz);
                const int o = c.off[lane];
                ox = (o & 1023) - 512;
                oy = ((o >> 10) & 1023) - 512;
                oz = ((o >> 20) & 1023) - 512;
            }
            stage(lane, c.j[lane], jx, jy, jz, ox, oy, oz);
        }
        __syncthreads();
        for (int t = 0; t < fill; ++t) use(t, c.j[t]);
        __syncthreads();
        fill = 0;
    }

    __device__ __forceinline__ void add(int j0, int j1, int jx, int jy, int jz, int ox, int oy, int oz)
    {
        const int lane = threadIdx.x & (kWave - 1);
        const int len = j1 - j0;
        if (fill + len > kWave) flush();
        if (lane < len) {
            c.j[fill + lane] = j0 + lane;
            if constexpr (FP32) {
                c.key[fill + lane] = (jz * a.g.n[1] + jy) * a.g.n[0] + jx;
                c.off[fill + lane] = (ox + 512) | ((oy + 512) << 10) | ((oz + 512) << 20);
            }
        }
        fill += len;
    }
};

// ================================================================ density

// The density list walk runs in three launches, each holding only the
// registers of its own part:
//  k_density_list_build   every particle's list: the candidates of its window
//                         within its list radius h_l = min(h_cap, (1 + 1/16) h0)
//                         (widened diameter), in window order, and their number;
//  k_density_list_pass    the Newton passes over the list while h stays within
//                         h_l; a particle whose list overflowed, or whose h
//                         leaves h_l before a pass, leaves its h, pass number and
//                         evaluation count (in the force constants' storage,
//                         which the force loop fills only later) for
//  k_density_list_window  its remaining passes over the whole window (it
//                         returns at once when no particle was left over).
// Every particle runs the same passes in the same order as in one walk.

// Particle p of the density list walk.
template <bool DIRECT, bool FP32>
struct DensListLane {
    using R = typename std::conditional<FP32, float, double>::type;
    Loc<DIRECT> li;
    int kx, ky, kz;
    int r[3];
    R xi, yi, zi;
    double mi, h0, hl, hcap;
    R Hl2w;

    __device__ __forceinline__ void load(const PairArgs& a, int64_t p, uint32_t& flags)
    {
        const int cell = a.key_sorted[p];
        cell_coords(cell, a.g, kx, ky, kz);
        lane_reach(a.g, a.reach[cell], r, flags);
        hcap = 0.5 * (double)r[0] * a.g.cell[0];
        hcap = fmin(hcap, 0.5 * (double)r[1] * a.g.cell[1]);
        hcap = fmin(hcap, 0.5 * (double)r[2] * a.g.cell[2]);
        // a fused r^2 is a few ulp from the exact one: the list radius is widened
        // so that it never drops a candidate the exact test would take
        constexpr double kWiden = FP32 ? 1.0 + 4e-6 : 1.0 + 1e-12;
        li = locate<DIRECT>(a.acc, p);
        if constexpr (FP32) {
            xi = ld_rel(a.f[SPHV_X], li, a.g, 0, kx);
            yi = ld_rel(a.f[SPHV_Y], li, a.g, 1, ky);
            zi = ld_rel(a.f[SPHV_Z], li, a.g, 2, kz);
            mi = (double)ld_f32v(a.f[SPHV_M], li);
        } else {
            xi = ld_f64(a.f[SPHV_X], li);
            yi = ld_f64(a.f[SPHV_Y], li);
            zi = ld_f64(a.f[SPHV_Z], li);
            mi = ld_f64(a.f[SPHV_M], li);
        }
        h0 = ld_f64(a.f[SPHV_H], li);
        hl = fmin(hcap, kGrowL * h0);
        Hl2w = (R)((2.0 * hl) * (2.0 * hl) * kWiden);
    }

    // the window's candidates that can lie within the cull radius 2 hh, run by
    // run, in window order
    template <class VisitRun>
    __device__ __forceinline__ void walk_runs(const PairArgs& a, double hh, VisitRun&& visit_run) const
    {
        const double bx = box_pos<FP32>(xi, a.g, 0, kx), by = box_pos<FP32>(yi, a.g, 1, ky),
                     bz = box_pos<FP32>(zi, a.g, 2, kz);
        const double rr = 2.0 * hh * (1.0 + 1e-6) + (FP32 ? a.g.cmin * 0x1p-18 : 0.0);
        const double rc2 = rr * rr;
        auto keep = [&](const double* bnd, double sx, double sy, double sz) {
            return box_d2(bnd, bx, by, bz, sx, sy, sz) < rc2;
        };
        auto keep_cell = [&](double d2, int) { return d2 < rc2; };
        walk_window_runs<true>(a, kx, ky, kz, r, bx, by, bz, keep_cell, keep, visit_run);
    }
};

// The sums of one Newton pass at smoothing length h: sum m w, sum w and
// sum m (3w + q w'); a candidate out of range adds the neutral element.
template <bool FP32, int KERN>
struct DensPassSums {
    using R = typename std::conditional<FP32, float, double>::type;
    R H2, hin;
    float f0 = 0.f, f1 = 0.f, f2 = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
    R p0 = 0, p1 = 0, p2 = 0;
    int kf = 0;
    int cnt = 0;

    __device__ __forceinline__ explicit DensPassSums(double h)
    {
        H2 = (R)((2.0 * h) * (2.0 * h));
        hin = (R)(1.0 / h);
    }

    __device__ __forceinline__ void term(R m, R r2, bool in)
    {
        const R rr = r2 * rsq_l(fmax(r2, TinyL<R>::v));
        const R q = rr * hin;
        R w, dw;
        spl<KERN>(q, w, dw);
        w = in ? w : (R)0;
        dw = in ? dw : (R)0;
        p0 = fma(m, w, p0);
        p1 = p1 + w;
        p2 = fma(m, fma(q, dw, (R)3 * w), p2);
        if constexpr (FP32) {
            // float partial sums folded into the compensated ones every 16 terms
            if (++kf == 16) {
                neumaier_l(f0, c0, p0);
                neumaier_l(f1, c1, p1);
                neumaier_l(f2, c2, p2);
                p0 = p1 = p2 = 0;
                kf = 0;
            }
        }
    }

    __device__ __forceinline__ void totals(double& t0, double& t1, double& t2)
    {
        if constexpr (FP32) {
            neumaier_l(f0, c0, p0);
            neumaier_l(f1, c1, p1);
            neumaier_l(f2, c2, p2);
            t0 = (double)f0 + (double)c0;
            t1 = (double)f1 + (double)c1;
            t2 = (double)f2 + (double)c2;
        } else {
            t0 = p0;
            t1 = p1;
            t2 = p2;
        }
    }
};

// The Newton step of the h iteration after a pass at h with totals t0..t2:
// true when the particle is done (converged, or its last pass), its outputs
// then stored; else hn is the next h.
template <bool DIRECT>
__device__ __forceinline__ bool dens_newton(const PairArgs& a, const Loc<DIRECT>& li, double mi, double hcap,
                                            double h, double t0, double t1, double t2, int pass, double& hn,
                                            uint32_t& flags)
{
    const double eta3 = a.eta * a.eta * a.eta;
    const double hinv = 1.0 / h;
    const double h3 = h * h * h;
    const double norm = 1.0 / (kPiL * h3);
    const double rho = norm * t0;
    const double nsum = norm * t1;
    const double drho = -(norm * hinv) * t2;
    const double mq = mi * eta3;
    const double f = rho - mq / h3;
    const double fp = drho + 3.0 * mq / (h3 * h);
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
        flags |= SPHV_F_H_CAP_HIT;
    }
    const bool conv = fabs(hn - h) <= a.tol * h;
    if (!(conv || pass + 1 >= a.max_iter)) return false;
    if (!conv) flags |= SPHV_F_H_NOT_CONVERGED;
    const double omega = 1.0 + h / (3.0 * rho) * drho;
    const double wcount = (4.0 * kPiL / 3.0) * (8.0 * h3) * nsum;
    if (!(isfinite(rho) && isfinite(omega))) flags |= SPHV_F_NONFINITE_OUTPUT;
    st_f64(a.f[SPHV_H], li, h);
    st_f64(a.f[SPHV_RHO], li, rho);
    st_f64(a.f[SPHV_OMEGA], li, omega);
    st_f64(a.f[SPHV_WCOUNT], li, wcount);
    return true;
}

// per-wave counters of a density launch into its fold slots
__device__ __forceinline__ void dens_leave(const PairArgs& a, unsigned long long n_final, unsigned long long n_evals,
                                           int maxit, uint32_t flags)
{
    for (int off = 32; off > 0; off >>= 1) {
        n_final += __shfl_xor(n_final, off, kWave);
        n_evals += __shfl_xor(n_evals, off, kWave);
        const int o = __shfl_xor(maxit, off, kWave);
        maxit = o > maxit ? o : maxit;
        flags |= __shfl_xor(flags, off, kWave);
    }
    if (threadIdx.x == 0) {
        int64_t* pp = a.part + (int64_t)blockIdx.x * kPartSlots;
        pp[0] = (int64_t)n_final;
        pp[1] = (int64_t)n_evals;
        pp[2] = maxit;
        pp[3] = flags;
    }
}

template <bool DIRECT, bool FP32, int KERN>
__global__ __launch_bounds__(kWave) void k_density_list_build(PairArgs a)
{
    using R = typename std::conditional<FP32, float, double>::type;
    const int lane = threadIdx.x;
    const int64_t n = a.n;
    const int cap = a.list_cap;
    if (blockIdx.x == 0 && lane == 0) a.meta[META_MASKS] = 0;   // the item kernels' mask cache is not written
    __shared__ WaveChunk chunk;
    __shared__ R s_x[kWave], s_y[kWave], s_z[kWave];
    uint32_t flags = 0;
    for (int64_t base = (int64_t)blockIdx.x * kWave; base < n; base += (int64_t)gridDim.x * kWave) {
        const int64_t p = base + lane;
        auto take = [&](const DensListLane<DIRECT, FP32>& I, int j, const Pos<DIRECT, FP32>& c, int& len) {
            R dx, dy, dz;
            if constexpr (FP32) {
                dx = I.xi - c.x;
                dy = I.yi - c.y;
                dz = I.zi - c.z;
            } else {
                dx = mi_diff(I.xi, c.x, a.g, 0);
                dy = mi_diff(I.yi, c.y, a.g, 1);
                dz = mi_diff(I.zi, c.z, a.g, 2);
            }
            if (fma(dz, dz, fma(dy, dy, dx * dx)) < I.Hl2w) {
                if (len < cap) a.list[p + (int64_t)len * n] = j;
                ++len;
            }
        };
        if (wave_coherent(a, p)) {
            // one walk for the wave, within the largest list diameter of its lanes
            DensListLane<DIRECT, FP32> I;
            I.load(a, p, flags);
            const WaveBox w = wave_box(box_pos<FP32>(I.xi, a.g, 0, I.kx), box_pos<FP32>(I.yi, a.g, 1, I.ky),
                                       box_pos<FP32>(I.zi, a.g, 2, I.kz));
            const double rr = wave_max_d(2.0 * I.hl * (1.0 + 1e-6) + (FP32 ? a.g.cmin * 0x1p-18 : 0.0));
            int len = 0;
            auto stage = [&](int t, int j, int jx, int jy, int jz, int ox, int oy, int oz) {
                Pos<DIRECT, FP32> c;
                const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
                if constexpr (FP32) c.load(a, lj, jx, jy, jz, ox, oy, oz);
                else c.load(a, lj, jx, jy, jz);
                s_x[t] = c.x;
                s_y[t] = c.y;
                s_z[t] = c.z;
            };
            auto use = [&](int t, int j) {
                Pos<DIRECT, FP32> c;
                c.x = s_x[t];
                c.y = s_y[t];
                c.z = s_z[t];
                take(I, j, c, len);
            };
            WaveRuns<FP32, decltype(stage), decltype(use)> runs(a, chunk, stage, use);
            walk_wave(
                a, I.kx, I.ky, I.kz, I.r, w, rr, [&](int) { return rr; }, [&](const double*) { return rr; },
                [&](int j0, int j1, int jx, int jy, int jz, int ox, int oy, int oz) {
                    runs.add(j0, j1, jx, jy, jz, ox, oy, oz);
                });
            runs.flush();
            a.list_len[p] = len;
            continue;
        }
        if (p >= n) continue;
        DensListLane<DIRECT, FP32> I;
        I.load(a, p, flags);
        int len = 0;
        I.walk_runs(a, I.hl, [&](int j0, int j1, int jx, int jy, int jz, int ox, int oy, int oz) {
            batched<4>(
                j0, j1,
                [&](int j) {
                    Pos<DIRECT, FP32> c;
                    const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
                    if constexpr (FP32) {
                        int cx = jx, co = ox;
                        run_cell(a, j, jy, jz, cx, co);
                        c.load(a, lj, cx, jy, jz, co, oy, oz);
                    } else {
                        c.load(a, lj, jx, jy, jz);
                    }
                    return c;
                },
                [&](int j, const Pos<DIRECT, FP32>& c) { take(I, j, c, len); });
        });
        a.list_len[p] = len;
    }
    for (int off = 32; off > 0; off >>= 1) flags |= __shfl_xor(flags, off, kWave);
    if (lane == 0 && flags) atomicOr(&a.state->flags, flags);
}

template <bool DIRECT, bool FP32, int KERN>
__global__ __launch_bounds__(kWave) void k_density_list_pass(PairArgs a)
{
    using R = typename std::conditional<FP32, float, double>::type;
    const int lane = threadIdx.x;
    const int64_t n = a.n;
    const int cap = a.list_cap;
    double* left_h = (double*)a.fconst;
    unsigned long long* left_evals = (unsigned long long*)a.fconst + n;
    int64_t* left_pass = (int64_t*)a.fconst + 2 * n;
    unsigned long long n_final = 0, n_evals = 0;
    int maxit = 0;
    uint32_t flags = 0;
    bool any_left = false;
    for (int64_t base = (int64_t)blockIdx.x * kWave; base < n; base += (int64_t)gridDim.x * kWave) {
        const int64_t p = base + lane;
        if (p >= n) continue;
        DensListLane<DIRECT, FP32> I;
        I.load(a, p, flags);
        const int len = a.list_len[p];
        const int32_t* L = a.list + p;
        double h = I.h0;
        unsigned long long it_evals = 0;
        int64_t leave_at = -1;
        for (int pass = 0;; ++pass) {
            if (len > cap || h > I.hl) {
                leave_at = pass;
                break;
            }
            DensPassSums<FP32, KERN> S(h);
            struct Cand {
                Pos<DIRECT, FP32> c;
                R m;
            };
            auto cand = [&](int j) {
                Cand v;
                const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
                if constexpr (FP32) {
                    int jx, jy, jz;
                    cell_coords(a.key_sorted[j], a.g, jx, jy, jz);
                    v.c.load(a, lj, jx, jy, jz, mi_cell(jx, I.kx, a.g, 0), mi_cell(jy, I.ky, a.g, 1),
                             mi_cell(jz, I.kz, a.g, 2));
                } else {
                    v.c.load(a, lj, 0, 0, 0);
                }
                v.m = ld_r<R>(a.f[SPHV_M], lj);
                return v;
            };
            auto use = [&](int j, const Cand& v) {
                R dx, dy, dz;
                const R r2 = diff<FP32>(a, I.xi, I.yi, I.zi, v.c, dx, dy, dz);
                const bool in = r2 < S.H2;
                S.term(v.m, r2, in);
                S.cnt += (in && (r2 > (R)0 || j != (int)p)) ? 1 : 0;
            };
            // the list, four entries at a time: their indices, then their
            // neighbours' loads all in flight together, then the terms in order
            int e = 0;
            for (; e + 4 <= len; e += 4) {
                int jj[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) jj[k] = L[(int64_t)(e + k) * n];
                Cand vv[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) vv[k] = cand(jj[k]);
#pragma unroll
                for (int k = 0; k < 4; ++k) use(jj[k], vv[k]);
            }
            for (; e < len; ++e) {
                const int j = L[(int64_t)e * n];
                use(j, cand(j));
            }
            double t0, t1, t2;
            S.totals(t0, t1, t2);
            it_evals += (unsigned long long)S.cnt;
            double hn;
            if (dens_newton<DIRECT>(a, I.li, I.mi, I.hcap, h, t0, t1, t2, pass, hn, flags)) {
                n_final += (unsigned long long)S.cnt;
                maxit = pass + 1 > maxit ? pass + 1 : maxit;
                n_evals += it_evals;
                break;
            }
            h = hn;
        }
        left_pass[p] = leave_at;
        if (leave_at >= 0) {
            left_h[p] = h;
            left_evals[p] = it_evals;
            any_left = true;
        }
    }
    if (__any(any_left) && lane == 0) atomicOr((unsigned int*)&a.meta[META_LIST_OVF], 1u);
    dens_leave(a, n_final, n_evals, maxit, flags);
}

template <bool DIRECT, bool FP32, int KERN>
__global__ __launch_bounds__(kWave) void k_density_list_window(PairArgs a)
{
    using R = typename std::conditional<FP32, float, double>::type;
    const int lane = threadIdx.x;
    const int64_t n = a.n;
    const double* left_h = (const double*)a.fconst;
    const unsigned long long* left_evals = (const unsigned long long*)a.fconst + n;
    const int64_t* left_pass = (const int64_t*)a.fconst + 2 * n;
    const bool any = a.meta[META_LIST_OVF] != 0;
    unsigned long long n_final = 0, n_evals = 0;
    int maxit = 0;
    uint32_t flags = 0;
    for (int64_t base = (int64_t)blockIdx.x * kWave; any && base < n; base += (int64_t)gridDim.x * kWave) {
        const int64_t p = base + lane;
        if (p >= n) continue;
        const int64_t first = left_pass[p];
        if (first < 0) continue;
        DensListLane<DIRECT, FP32> I;
        uint32_t unused = 0;
        I.load(a, p, unused);
        double h = left_h[p];
        unsigned long long it_evals = left_evals[p];
        for (int pass = (int)first;; ++pass) {
            DensPassSums<FP32, KERN> S(h);
            // the whole window: every candidate the list would hold (while h
            // stays within h_l, those are exactly the list's entries, in its
            // order, so the FP32 partial sums are grouped as in the list walk)
            // and every candidate in range at the current h
            I.walk_runs(a, fmax(I.hl, h), [&](int j0, int j1, int jx, int jy, int jz, int ox, int oy, int oz) {
                for (int j = j0; j < j1; ++j) {
                    Pos<DIRECT, FP32> c;
                    const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
                    if constexpr (FP32) {
                        int cx = jx, co = ox;
                        run_cell(a, j, jy, jz, cx, co);
                        c.load(a, lj, cx, jy, jz, co, oy, oz);
                    } else {
                        c.load(a, lj, jx, jy, jz);
                    }
                    const R m = ld_r<R>(a.f[SPHV_M], lj);
                    R dx, dy, dz;
                    const R r2 = diff<FP32>(a, I.xi, I.yi, I.zi, c, dx, dy, dz);
                    const bool in = r2 < S.H2;
                    if (in || fma(dz, dz, fma(dy, dy, dx * dx)) < I.Hl2w) {
                        S.term(m, r2, in);
                        S.cnt += (in && (r2 > (R)0 || j != (int)p)) ? 1 : 0;
                    }
                }
            });
            double t0, t1, t2;
            S.totals(t0, t1, t2);
            it_evals += (unsigned long long)S.cnt;
            double hn;
            if (dens_newton<DIRECT>(a, I.li, I.mi, I.hcap, h, t0, t1, t2, pass, hn, flags)) {
                n_final += (unsigned long long)S.cnt;
                maxit = pass + 1 > maxit ? pass + 1 : maxit;
                n_evals += it_evals;
                break;
            }
            h = hn;
        }
    }
    dens_leave(a, n_final, n_evals, maxit, flags);
}

// ================================================================== force

// Per-particle constants of the force loop, once per particle: A = P/(Omega
// rho^2) with P = (gamma-1) rho u, c = sqrt(gamma (gamma-1) u), 1/h, the
// kernel gradient's norm 1/(pi h^4) and (2h)^2, at fconst[k n + p], k = 0..4,
// in the pair precision (both force loops read them instead of deriving them
// again for every pair or staged candidate).
template <bool DIRECT, bool FP32>
__global__ void k_force_prep(PairArgs a)
{
    using R = typename std::conditional<FP32, float, double>::type;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const Loc<DIRECT> l = locate<DIRECT>(a.acc, p);
    const R gm1 = (R)(a.gamma - 1.0);
    const R ggm1 = (R)(a.gamma * (a.gamma - 1.0));
    const R h = ld_r<R>(a.f[SPHV_H], l), rho = ld_r<R>(a.f[SPHV_RHO], l);
    const R om = ld_r<R>(a.f[SPHV_OMEGA], l), u = ld_r<R>(a.f[SPHV_U], l);
    const R P = gm1 * rho * u;
    const R hv = (R)1 / h;
    const R hv2 = hv * hv;
    R* fc = (R*)a.fconst;
    fc[p] = P / (om * rho * rho);
    fc[a.n + p] = sqrt(ggm1 * u);
    fc[2 * a.n + p] = hv;
    fc[3 * a.n + p] = hv2 * hv2 / (R)kPiL;
    const R H = (R)2 * h;
    fc[4 * a.n + p] = H * H;
}

// The force list walk runs in three launches, each holding only the registers
// of its own part, so that more waves share a SIMD and hide the latency of the
// per-lane gathers:
//  k_force_list_build   every particle's pairs (r < 2 max(h_i, h_j), r > 0) in
//                       window order into its list, and their number; the pair
//                       counts (coincident neighbours included); a list too
//                       short for its pairs raises a flag;
//  k_force_list_eval    the particles whose pairs fit their list: the pairs
//                       from the list;
//  k_force_list_window  only when the flag is up, the other particles: the
//                       same pairs in the same order from their window.

// Particle i of a force list walk: its position in the frame of the pair
// differences and the window's culling bounds.
template <bool DIRECT, bool FP32>
struct ForceListPos {
    using R = typename std::conditional<FP32, float, double>::type;
    Loc<DIRECT> li;
    int kx, ky, kz;
    int r[3];
    R xi, yi, zi, Hi, H2i;
    double bx, by, bz;

    __device__ __forceinline__ void load(const PairArgs& a, int64_t p, uint32_t& flags)
    {
        const int cell = a.key_sorted[p];
        cell_coords(cell, a.g, kx, ky, kz);
        lane_reach(a.g, a.reach[cell], r, flags);
        li = locate<DIRECT>(a.acc, p);
        if constexpr (FP32) {
            xi = ld_rel(a.f[SPHV_X], li, a.g, 0, kx);
            yi = ld_rel(a.f[SPHV_Y], li, a.g, 1, ky);
            zi = ld_rel(a.f[SPHV_Z], li, a.g, 2, kz);
        } else {
            xi = ld_f64(a.f[SPHV_X], li);
            yi = ld_f64(a.f[SPHV_Y], li);
            zi = ld_f64(a.f[SPHV_Z], li);
        }
        Hi = (R)2 * ld_r<R>(a.f[SPHV_H], li);
        H2i = Hi * Hi;
        bx = box_pos<FP32>(xi, a.g, 0, kx);
        by = box_pos<FP32>(yi, a.g, 1, ky);
        bz = box_pos<FP32>(zi, a.g, 2, kz);
    }

    // every candidate of the window that can be a pair, in window order: the
    // runs and cells within reach of max(2 h_i, their largest 2h)
    template <class Visit>
    __device__ __forceinline__ void walk(const PairArgs& a, Visit&& visit) const
    {
        const double mrg = FP32 ? a.g.cmin * 0x1p-18 : 0.0;
        auto keep = [&](const double* bnd, double sx, double sy, double sz) {
            const double rr = fmax((double)Hi, bnd[6]) * (1.0 + 1e-6) + mrg;
            return box_d2(bnd, bx, by, bz, sx, sy, sz) < rr * rr;
        };
        // a row is kept within the largest 2h any force partner of the cell's
        // particles can have (the cover of the own force reaches)
        const double Hg = (double)a.reach_s[cell_key(kx, ky, kz, a.g)] * a.g.cmin;
        auto keep_cell = [&](double d2, int key) {
            const double Hc = key < 0 ? Hg : (double)__uint_as_float(a.cell_h[key]);
            const double rr = fmax((double)Hi, Hc) * (1.0 + 1e-6) + mrg;
            return d2 < rr * rr;
        };
        walk_window<true>(a, kx, ky, kz, r, bx, by, bz, keep_cell, keep, visit);
    }

    template <class VisitRun>
    __device__ __forceinline__ void walk_runs(const PairArgs& a, VisitRun&& visit_run) const
    {
        const double mrg = FP32 ? a.g.cmin * 0x1p-18 : 0.0;
        auto keep = [&](const double* bnd, double sx, double sy, double sz) {
            const double rr = fmax((double)Hi, bnd[6]) * (1.0 + 1e-6) + mrg;
            return box_d2(bnd, bx, by, bz, sx, sy, sz) < rr * rr;
        };
        // a row is kept within the largest 2h any force partner of the cell's
        // particles can have (the cover of the own force reaches)
        const double Hg = (double)a.reach_s[cell_key(kx, ky, kz, a.g)] * a.g.cmin;
        auto keep_cell = [&](double d2, int key) {
            const double Hc = key < 0 ? Hg : (double)__uint_as_float(a.cell_h[key]);
            const double rr = fmax((double)Hi, Hc) * (1.0 + 1e-6) + mrg;
            return d2 < rr * rr;
        };
        walk_window_runs<true>(a, kx, ky, kz, r, bx, by, bz, keep_cell, keep, visit_run);
    }

    // candidate j placed in i's frame; true when (i, j) is a pair or j coincides with i
    __device__ __forceinline__ bool pair_test(const PairArgs& a, int j, int jx, int jy, int jz, int ox, int oy,
                                              int oz, R& dx, R& dy, R& dz, R& r2, Loc<DIRECT>& lj) const
    {
        const R* fc = (const R*)a.fconst;
        Pos<DIRECT, FP32> c;
        lj = locate<DIRECT>(a.acc, j);
        if constexpr (FP32) {
            int cx = jx, co = ox;
            run_cell(a, j, jy, jz, cx, co);
            c.load(a, lj, cx, jy, jz, co, oy, oz);
        } else {
            c.load(a, lj, jx, jy, jz);
        }
        r2 = diff<FP32>(a, xi, yi, zi, c, dx, dy, dz);
        return r2 < fmax(H2i, fc[4 * a.n + j]);
    }
};

// The sums of particle i over its pairs, in the order the pairs are added.
template <bool DIRECT, bool FP32, int KERN>
struct ForceListSums {
    using R = typename std::conditional<FP32, float, double>::type;
    R vxi, vyi, vzi, rhoi, hali, Ai, ci, hinvi, normi;
    float fax = 0.f, cax = 0.f, fay = 0.f, cay = 0.f, faz = 0.f, caz = 0.f, fdu = 0.f, cdu = 0.f;
    R pax = 0, pay = 0, paz = 0, pdu = 0;
    int kf = 0;
    R vsig;

    __device__ __forceinline__ void load(const PairArgs& a, int64_t p, const Loc<DIRECT>& li)
    {
        const R* fc = (const R*)a.fconst;
        const int64_t n = a.n;
        vxi = ld_r<R>(a.f[SPHV_VX], li);
        vyi = ld_r<R>(a.f[SPHV_VY], li);
        vzi = ld_r<R>(a.f[SPHV_VZ], li);
        rhoi = ld_r<R>(a.f[SPHV_RHO], li);
        hali = (R)0.5 * ld_r<R>(a.f[SPHV_ALPHA], li);
        Ai = fc[p];
        ci = fc[n + p];
        hinvi = fc[2 * n + p];
        normi = fc[3 * n + p];
        vsig = (R)2 * ci;
    }

    // the members of neighbour j a pair term reads
    struct Nb {
        R vxj, vyj, vzj, mj, rhoj, halj, Aj, cj, hinvj, normj;
    };
    __device__ __forceinline__ static Nb nb_of(const PairArgs& a, int j, const Loc<DIRECT>& lj)
    {
        const R* fc = (const R*)a.fconst;
        const int64_t n = a.n;
        Nb b;
        b.vxj = ld_r<R>(a.f[SPHV_VX], lj);
        b.vyj = ld_r<R>(a.f[SPHV_VY], lj);
        b.vzj = ld_r<R>(a.f[SPHV_VZ], lj);
        b.mj = ld_r<R>(a.f[SPHV_M], lj);
        b.rhoj = ld_r<R>(a.f[SPHV_RHO], lj);
        b.halj = (R)0.5 * ld_r<R>(a.f[SPHV_ALPHA], lj);
        b.Aj = fc[j];
        b.cj = fc[n + j];
        b.hinvj = fc[2 * n + j];
        b.normj = fc[3 * n + j];
        return b;
    }

    // one pair's contribution (r > 0)
    __device__ __forceinline__ void term(const PairArgs& a, int j, const Loc<DIRECT>& lj, R dx, R dy, R dz, R r2)
    {
        term_nb(nb_of(a, j, lj), dx, dy, dz, r2);
    }

    __device__ __forceinline__ void term_nb(const Nb& b, R dx, R dy, R dz, R r2)
    {
        const R vxj = b.vxj, vyj = b.vyj, vzj = b.vzj, mj = b.mj, rhoj = b.rhoj, halj = b.halj;
        const R Aj = b.Aj, cj = b.cj, hinvj = b.hinvj, normj = b.normj;
        const R y = rsq_l(r2);
        const R rr = r2 * y;
        const R gi = spl_dw<KERN>(rr * hinvi) * normi;
        const R gj = spl_dw<KERN>(rr * hinvj) * normj;
        const R gbar = (R)0.5 * (gi + gj);
        const R ex = dx * y, ey = dy * y, ez = dz * y;
        const R w = (vxi - vxj) * ex + (vyi - vyj) * ey + (vzi - vzj) * ez;
        const R mu = w < (R)0 ? w : (R)0;
        const R vs = ci + cj - (R)3 * mu;
        // Pi = -(alpha_bar / 2) v_sig mu / rho_bar = -alpha_bar v_sig mu / (rho_i + rho_j)
        const R visc = -(hali + halj) * vs * mu * rcp_l(rhoi + rhoj);
        const R Agi = Ai * gi;
        const R coef = mj * fma(visc, gbar, fma(Aj, gj, Agi));
        const R dui = mj * fma((R)0.5 * visc, gbar, Agi) * w;
        pax = fma(-coef, ex, pax);
        pay = fma(-coef, ey, pay);
        paz = fma(-coef, ez, paz);
        pdu = pdu + dui;
        vsig = vs > vsig ? vs : vsig;
        if constexpr (FP32) {
            if (++kf == 16) {
                neumaier_l(fax, cax, pax);
                neumaier_l(fay, cay, pay);
                neumaier_l(faz, caz, paz);
                neumaier_l(fdu, cdu, pdu);
                pax = pay = paz = pdu = 0;
                kf = 0;
            }
        }
    }

    // the outputs of particle i
    __device__ __forceinline__ void store(const PairArgs& a, const Loc<DIRECT>& li, uint32_t& flags)
    {
        double ax, ay, az, du;
        if constexpr (FP32) {
            neumaier_l(fax, cax, pax);
            neumaier_l(fay, cay, pay);
            neumaier_l(faz, caz, paz);
            neumaier_l(fdu, cdu, pdu);
            ax = (double)fax + (double)cax;
            ay = (double)fay + (double)cay;
            az = (double)faz + (double)caz;
            du = (double)fdu + (double)cdu;
        } else {
            ax = pax;
            ay = pay;
            az = paz;
            du = pdu;
        }
        st_f64(a.f[SPHV_AX], li, ax);
        st_f64(a.f[SPHV_AY], li, ay);
        st_f64(a.f[SPHV_AZ], li, az);
        st_f64(a.f[SPHV_UDT], li, du);
        st_f64(a.f[SPHV_VSIG], li, (double)vsig);
        if (!(isfinite(ax) && isfinite(ay) && isfinite(az) && isfinite(du))) flags |= SPHV_F_NONFINITE_OUTPUT;
    }
};

template <bool DIRECT, bool FP32, int KERN>
__global__ __launch_bounds__(kWave) void k_force_list_build(PairArgs a)
{
    using R = typename std::conditional<FP32, float, double>::type;
    const int lane = threadIdx.x;
    const int64_t n = a.n;
    const int cap = a.list_cap;
    __shared__ WaveChunk chunk;
    __shared__ R s_x[kWave], s_y[kWave], s_z[kWave], s_h[kWave];
    unsigned long long n_pairs = 0;
    uint32_t flags = 0;
    bool over = false;
    const R* fc = (const R*)a.fconst;
    for (int64_t base = (int64_t)blockIdx.x * kWave; base < n; base += (int64_t)gridDim.x * kWave) {
        const int64_t p = base + lane;
        int len = 0;
        int coinc = 0;   // coincident neighbours: counted as pairs, no force
        auto take = [&](const ForceListPos<DIRECT, FP32>& I, int j, const Pos<DIRECT, FP32>& c, R H2j) {
            R dx, dy, dz;
            const R r2 = diff<FP32>(a, I.xi, I.yi, I.zi, c, dx, dy, dz);
            if (r2 < fmax(I.H2i, H2j)) {
                if (r2 > (R)0) {
                    if (len < cap) a.list[p + (int64_t)len * n] = j;
                    ++len;
                } else if (j != (int)p) {
                    ++coinc;
                }
            }
        };
        if (wave_coherent(a, p)) {
            // one walk for the wave, within the largest support of its lanes
            ForceListPos<DIRECT, FP32> I;
            I.load(a, p, flags);
            const WaveBox w = wave_box(I.bx, I.by, I.bz);
            const double Hmax = wave_max_d((double)I.Hi);
            const double mrg = FP32 ? a.g.cmin * 0x1p-18 : 0.0;
            const double Hg = (double)a.reach_s[cell_key(I.kx, I.ky, I.kz, a.g)] * a.g.cmin;
            const double rr_row = fmax(Hmax, Hg) * (1.0 + 1e-6) + mrg;
            auto stage = [&](int t, int j, int jx, int jy, int jz, int ox, int oy, int oz) {
                Pos<DIRECT, FP32> c;
                const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
                if constexpr (FP32) c.load(a, lj, jx, jy, jz, ox, oy, oz);
                else c.load(a, lj, jx, jy, jz);
                s_x[t] = c.x;
                s_y[t] = c.y;
                s_z[t] = c.z;
                s_h[t] = fc[4 * n + j];
            };
            auto use = [&](int t, int j) {
                Pos<DIRECT, FP32> c;
                c.x = s_x[t];
                c.y = s_y[t];
                c.z = s_z[t];
                take(I, j, c, s_h[t]);
            };
            WaveRuns<FP32, decltype(stage), decltype(use)> runs(a, chunk, stage, use);
            walk_wave(
                a, I.kx, I.ky, I.kz, I.r, w, rr_row,
                [&](int key) { return fmax(Hmax, (double)__uint_as_float(a.cell_h[key])) * (1.0 + 1e-6) + mrg; },
                [&](const double* bnd) { return fmax(Hmax, bnd[6]) * (1.0 + 1e-6) + mrg; },
                [&](int j0, int j1, int jx, int jy, int jz, int ox, int oy, int oz) {
                    runs.add(j0, j1, jx, jy, jz, ox, oy, oz);
                });
            runs.flush();
        } else {
            if (p >= n) continue;
            ForceListPos<DIRECT, FP32> I;
            I.load(a, p, flags);
            // candidates two at a time (four cost this kernel more in occupancy
            // than they gain in loads in flight)
            struct Cand {
                Pos<DIRECT, FP32> c;
                R H2;
            };
            I.walk_runs(a, [&](int j0, int j1, int jx, int jy, int jz, int ox, int oy, int oz) {
                batched<2>(
                    j0, j1,
                    [&](int j) {
                        Cand v;
                        const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
                        if constexpr (FP32) {
                            int cx = jx, co = ox;
                            run_cell(a, j, jy, jz, cx, co);
                            v.c.load(a, lj, cx, jy, jz, co, oy, oz);
                        } else {
                            v.c.load(a, lj, jx, jy, jz);
                        }
                        v.H2 = fc[4 * n + j];
                        return v;
                    },
                    [&](int j, const Cand& v) { take(I, j, v.c, v.H2); });
            });
        }
        a.list_len[p] = len;
        over |= len > cap;
        n_pairs += (unsigned long long)(len + coinc);
    }
    if (__any(over) && lane == 0) atomicOr((unsigned int*)&a.meta[META_LIST_OVF], 1u);
    for (int off = 32; off > 0; off >>= 1) {
        n_pairs += __shfl_xor(n_pairs, off, kWave);
        flags |= __shfl_xor(flags, off, kWave);
    }
    if (lane == 0) {
        int64_t* pp = a.part + (int64_t)blockIdx.x * kPartSlots;
        pp[0] = (int64_t)n_pairs;
        pp[1] = 0;
        pp[2] = 0;
        pp[3] = flags;
    }
}

template <bool DIRECT, bool FP32, int KERN>
__global__ __launch_bounds__(kWave) void k_force_list_eval(PairArgs a)
{
    using R = typename std::conditional<FP32, float, double>::type;
    const int lane = threadIdx.x;
    const int64_t n = a.n;
    const int cap = a.list_cap;
    uint32_t flags = 0;
    for (int64_t base = (int64_t)blockIdx.x * kWave; base < n; base += (int64_t)gridDim.x * kWave) {
        const int64_t p = base + lane;
        if (p >= n) continue;
        const int len = a.list_len[p];
        if (len > cap) continue;
        const Loc<DIRECT> li = locate<DIRECT>(a.acc, p);
        int kx = 0, ky = 0, kz = 0;
        R xi, yi, zi;
        if constexpr (FP32) {
            cell_coords(a.key_sorted[p], a.g, kx, ky, kz);
            xi = ld_rel(a.f[SPHV_X], li, a.g, 0, kx);
            yi = ld_rel(a.f[SPHV_Y], li, a.g, 1, ky);
            zi = ld_rel(a.f[SPHV_Z], li, a.g, 2, kz);
        } else {
            xi = ld_f64(a.f[SPHV_X], li);
            yi = ld_f64(a.f[SPHV_Y], li);
            zi = ld_f64(a.f[SPHV_Z], li);
        }
        using Sums = ForceListSums<DIRECT, FP32, KERN>;
        Sums S;
        S.load(a, p, li);
        const int32_t* L = a.list + p;
        // a neighbour's members, loaded before they are used
        struct Cand {
            Pos<DIRECT, FP32> c;
            typename Sums::Nb b;
        };
        auto cand = [&](int j) {
            Cand v;
            const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
            if constexpr (FP32) {
                int jx, jy, jz;
                cell_coords(a.key_sorted[j], a.g, jx, jy, jz);
                v.c.load(a, lj, jx, jy, jz, mi_cell(jx, kx, a.g, 0), mi_cell(jy, ky, a.g, 1), mi_cell(jz, kz, a.g, 2));
            } else {
                v.c.load(a, lj, 0, 0, 0);
            }
            v.b = Sums::nb_of(a, j, lj);
            return v;
        };
        auto use = [&](const Cand& v) {
            R dx, dy, dz;
            const R r2 = diff<FP32>(a, xi, yi, zi, v.c, dx, dy, dz);
            S.term_nb(v.b, dx, dy, dz, r2);
        };
        // two entries at a time: both neighbours' loads in flight together, the
        // next two entries' indices read meanwhile
        int e = 0;
        int jn0 = len > 0 ? L[0] : 0, jn1 = len > 1 ? L[n] : 0;
        for (; e + 2 <= len; e += 2) {
            const int j0 = jn0, j1 = jn1;
            if (e + 2 < len) jn0 = L[(int64_t)(e + 2) * n];
            if (e + 3 < len) jn1 = L[(int64_t)(e + 3) * n];
            const Cand v0 = cand(j0);
            const Cand v1 = cand(j1);
            use(v0);
            use(v1);
        }
        if (e < len) use(cand(jn0));
        S.store(a, li, flags);
    }
    for (int off = 32; off > 0; off >>= 1) flags |= __shfl_xor(flags, off, kWave);
    if (lane == 0 && flags) atomicOr(&a.state->flags, flags);
}

template <bool DIRECT, bool FP32, int KERN>
__global__ __launch_bounds__(kWave) void k_force_list_window(PairArgs a)
{
    using R = typename std::conditional<FP32, float, double>::type;
    const int lane = threadIdx.x;
    const int64_t n = a.n;
    const int cap = a.list_cap;
    if (a.meta[META_LIST_OVF] == 0) return;
    uint32_t flags = 0;
    for (int64_t base = (int64_t)blockIdx.x * kWave; base < n; base += (int64_t)gridDim.x * kWave) {
        const int64_t p = base + lane;
        if (p >= n) continue;
        if (a.list_len[p] <= cap) continue;
        ForceListPos<DIRECT, FP32> I;
        uint32_t unused = 0;
        I.load(a, p, unused);
        ForceListSums<DIRECT, FP32, KERN> S;
        S.load(a, p, I.li);
        I.walk(a, [&](int j, int jx, int jy, int jz, int ox, int oy, int oz) {
            R dx, dy, dz, r2;
            Loc<DIRECT> lj;
            if (I.pair_test(a, j, jx, jy, jz, ox, oy, oz, dx, dy, dz, r2, lj) && r2 > (R)0)
                S.term(a, j, lj, dx, dy, dz, r2);
        });
        S.store(a, I.li, flags);
    }
    for (int off = 32; off > 0; off >>= 1) flags |= __shfl_xor(flags, off, kWave);
    if (lane == 0 && flags) atomicOr(&a.state->flags, flags);
}

// ======================================================= symmetric force
//
// Each pair evaluated once (paper Sec. 5.3: F(p1, p2) = -F(p2, p1)), FP64,
// in three launches with a fixed order of every sum:
//  1. k_force_sym_build: every particle's force list, ascending in sorted
//     position (the window walk's order), and its length;
//  2. k_force_sym_upper: for each pair (i, j) with i < j, the owner i evaluates
//     it, adds its own side in list order, and stores j's side -- m_i B r_hat
//     (B the pair's bracket A_i g_i + A_j g_j + Pi gbar), m_i (A_j g_j + Pi
//     gbar / 2) w and the pair's v_sig -- in slot e of j, e being i's position
//     in j's list (found by bisection); i's own sums go to its outputs;
//  3. k_force_sym_lower: each particle adds the slots of its partners below
//     it (the head of its list) in list order to what pass 2 left.
// Should any list overflow (flagged by pass 1), pass 2 does nothing and pass
// 3 evaluates every particle's pairs twice from its window.

// Common set-up of one particle of the force loop (FP64).
template <bool DIRECT>
struct ForceLane {
    double xi, yi, zi, vxi, vyi, vzi, hi, rhoi, hali, mi, Ai, ci, hinvi, normi, Hi, H2i, bx, by, bz;
    int kx, ky, kz;
    int r[3];
    Loc<DIRECT> li;

    __device__ __forceinline__ void load(const PairArgs& a, int64_t p, uint32_t& flags)
    {
        const int cell = a.key_sorted[p];
        cell_coords(cell, a.g, kx, ky, kz);
        lane_reach(a.g, a.reach[cell], r, flags);
        li = locate<DIRECT>(a.acc, p);
        xi = ld_f64(a.f[SPHV_X], li);
        yi = ld_f64(a.f[SPHV_Y], li);
        zi = ld_f64(a.f[SPHV_Z], li);
        vxi = ld_f64(a.f[SPHV_VX], li);
        vyi = ld_f64(a.f[SPHV_VY], li);
        vzi = ld_f64(a.f[SPHV_VZ], li);
        hi = ld_f64(a.f[SPHV_H], li);
        rhoi = ld_f64(a.f[SPHV_RHO], li);
        mi = ld_f64(a.f[SPHV_M], li);
        hali = 0.5 * ld_f64(a.f[SPHV_ALPHA], li);
        const double* fc = (const double*)a.fconst;
        const int64_t n = a.n;
        Ai = fc[p];
        ci = fc[n + p];
        hinvi = fc[2 * n + p];
        normi = fc[3 * n + p];
        Hi = 2.0 * hi;
        H2i = Hi * Hi;
        bx = xi;
        by = yi;
        bz = zi;
    }
};

// One pair's terms from i's side (r > 0): B, the unit vector, w, gbar, visc,
// g_i, g_j, vs.
template <int KERN, bool DIRECT>
struct PairTerms {
    double B, ex, ey, ez, w, gbar, visc, gi, gj, vs, mj, Aj;

    __device__ __forceinline__ void eval(const PairArgs& a, const ForceLane<DIRECT>& L, int j,
                                         const Loc<DIRECT>& lj, double dx, double dy, double dz, double r2)
    {
        const double* fc = (const double*)a.fconst;
        const int64_t n = a.n;
        const double vxj = ld_f64(a.f[SPHV_VX], lj), vyj = ld_f64(a.f[SPHV_VY], lj), vzj = ld_f64(a.f[SPHV_VZ], lj);
        mj = ld_f64(a.f[SPHV_M], lj);
        const double rhoj = ld_f64(a.f[SPHV_RHO], lj);
        const double halj = 0.5 * ld_f64(a.f[SPHV_ALPHA], lj);
        Aj = fc[j];
        const double cj = fc[n + j], hinvj = fc[2 * n + j], normj = fc[3 * n + j];
        const double y = rsq_l(r2);
        const double rr = r2 * y;
        gi = spl_dw<KERN>(rr * L.hinvi) * L.normi;
        gj = spl_dw<KERN>(rr * hinvj) * normj;
        gbar = 0.5 * (gi + gj);
        ex = dx * y;
        ey = dy * y;
        ez = dz * y;
        w = (L.vxi - vxj) * ex + (L.vyi - vyj) * ey + (L.vzi - vzj) * ez;
        const double mu = w < 0.0 ? w : 0.0;
        vs = L.ci + cj - 3.0 * mu;
        visc = -(L.hali + halj) * vs * mu * rcp_l(L.rhoi + rhoj);
        B = fma(visc, gbar, fma(Aj, gj, L.Ai * gi));
    }
};

template <bool DIRECT, int KERN>
__global__ __launch_bounds__(kWave) void k_force_sym_build(PairArgs a)
{
    const int lane = threadIdx.x;
    const int64_t n = a.n;
    const int cap = a.list_cap;
    const double* fc = (const double*)a.fconst;
    unsigned long long n_pairs = 0;
    uint32_t flags = 0;
    bool over = false;
    for (int64_t base = (int64_t)blockIdx.x * kWave; base < n; base += (int64_t)gridDim.x * kWave) {
        const int64_t p = base + lane;
        if (p >= n) continue;
        ForceLane<DIRECT> L;
        L.load(a, p, flags);
        auto keep = [&](const double* bnd, double sx, double sy, double sz) {
            const double rr = fmax(L.Hi, bnd[6]) * (1.0 + 1e-6);
            return box_d2(bnd, L.bx, L.by, L.bz, sx, sy, sz) < rr * rr;
        };
        // a row is kept within the largest 2h any force partner of the cell's
        // particles can have (the cover of the own force reaches)
        const double Hg = (double)a.reach_s[cell_key(L.kx, L.ky, L.kz, a.g)] * a.g.cmin;
        auto keep_cell = [&](double d2, int key) {
            const double Hc = key < 0 ? Hg : (double)__uint_as_float(a.cell_h[key]);
            const double rr = fmax(L.Hi, Hc) * (1.0 + 1e-6);
            return d2 < rr * rr;
        };
        int32_t* Ls = a.list + p;
        int len = 0, coinc = 0;
        walk_window<true>(a, L.kx, L.ky, L.kz, L.r, L.bx, L.by, L.bz, keep_cell, keep,
                    [&](int j, int, int, int, int, int, int) {
                        const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
                        const double dx = mi_diff(L.xi, ld_f64(a.f[SPHV_X], lj), a.g, 0);
                        const double dy = mi_diff(L.yi, ld_f64(a.f[SPHV_Y], lj), a.g, 1);
                        const double dz = mi_diff(L.zi, ld_f64(a.f[SPHV_Z], lj), a.g, 2);
                        const double r2 = dx * dx + dy * dy + dz * dz;
                        if (r2 < fmax(L.H2i, fc[4 * n + j])) {
                            if (r2 > 0.0) {
                                if (len < cap) Ls[(int64_t)len * n] = j;
                                ++len;
                            } else if (j != (int)p) {
                                ++coinc;
                            }
                        }
                    });
        a.list_len[p] = len;
        over |= len > cap;
        n_pairs += (unsigned long long)(len + coinc);
    }
    if (__any(over) && lane == 0) atomicOr((unsigned int*)&a.meta[META_LIST_OVF], 1u);
    for (int off = 32; off > 0; off >>= 1) {
        n_pairs += __shfl_xor(n_pairs, off, kWave);
        flags |= __shfl_xor(flags, off, kWave);
    }
    if (lane == 0) {
        int64_t* pp = a.part + (int64_t)blockIdx.x * kPartSlots;
        pp[0] = (int64_t)n_pairs;
        pp[1] = 0;
        pp[2] = 0;
        pp[3] = flags;
    }
}

template <bool DIRECT, int KERN>
__global__ __launch_bounds__(kWave) void k_force_sym_upper(PairArgs a)
{
    const int lane = threadIdx.x;
    const int64_t n = a.n;
    const int64_t cn = (int64_t)a.list_cap * n;
    if (a.meta[META_LIST_OVF]) return;
    uint32_t flags = 0;
    for (int64_t base = (int64_t)blockIdx.x * kWave; base < n; base += (int64_t)gridDim.x * kWave) {
        const int64_t p = base + lane;
        if (p >= n) continue;
        ForceLane<DIRECT> L;
        L.load(a, p, flags);
        const int32_t* Li = a.list + p;
        const int len = a.list_len[p];
        double pax = 0.0, pay = 0.0, paz = 0.0, pdu = 0.0, vsig = 2.0 * L.ci;
        // the list ascends: the partners above p are its tail
        for (int e = 0; e < len; ++e) {
            const int j = Li[(int64_t)e * n];
            if (j < (int)p) continue;
            const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
            const double dx = mi_diff(L.xi, ld_f64(a.f[SPHV_X], lj), a.g, 0);
            const double dy = mi_diff(L.yi, ld_f64(a.f[SPHV_Y], lj), a.g, 1);
            const double dz = mi_diff(L.zi, ld_f64(a.f[SPHV_Z], lj), a.g, 2);
            const double r2 = dx * dx + dy * dy + dz * dz;
            PairTerms<KERN, DIRECT> t;
            t.eval(a, L, j, lj, dx, dy, dz, r2);
            const double coef = t.mj * t.B;
            pax = fma(-coef, t.ex, pax);
            pay = fma(-coef, t.ey, pay);
            paz = fma(-coef, t.ez, paz);
            pdu = pdu + t.mj * fma(0.5 * t.visc, t.gbar, L.Ai * t.gi) * t.w;
            vsig = t.vs > vsig ? t.vs : vsig;
            // j's side, in j's slot for p: p's position in j's (ascending) list
            const int32_t* Lj = a.list + j;
            const int lenj = a.list_len[j];
            int lo = 0, hi = lenj;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (Lj[(int64_t)mid * n] < (int)p) lo = mid + 1;
                else hi = mid;
            }
            // the pair relation is symmetric, so p is in j's list; a miss is a
            // fault of the lists, flagged, its slot left alone
            if (lo >= lenj || Lj[(int64_t)lo * n] != (int)p) {
                flags |= SPHV_F_LIST_MISMATCH;
                continue;
            }
            const double cj = L.mi * t.B;
            double* sl = a.slots + (int64_t)lo * n + j;
            sl[0] = cj * t.ex;
            sl[cn] = cj * t.ey;
            sl[2 * cn] = cj * t.ez;
            sl[3 * cn] = L.mi * fma(0.5 * t.visc, t.gbar, t.Aj * t.gj) * t.w;
            sl[4 * cn] = t.vs;
        }
        st_f64(a.f[SPHV_AX], L.li, pax);
        st_f64(a.f[SPHV_AY], L.li, pay);
        st_f64(a.f[SPHV_AZ], L.li, paz);
        st_f64(a.f[SPHV_UDT], L.li, pdu);
        st_f64(a.f[SPHV_VSIG], L.li, vsig);
    }
    for (int off = 32; off > 0; off >>= 1) flags |= __shfl_xor(flags, off, kWave);
    if (lane == 0 && flags) atomicOr(&a.state->flags, flags);
}

template <bool DIRECT, int KERN>
__global__ __launch_bounds__(kWave) void k_force_sym_lower(PairArgs a)
{
    const int lane = threadIdx.x;
    const int64_t n = a.n;
    const int64_t cn = (int64_t)a.list_cap * n;
    const bool twice = a.meta[META_LIST_OVF] != 0;
    const double* fc = (const double*)a.fconst;
    uint32_t flags = 0;
    for (int64_t base = (int64_t)blockIdx.x * kWave; base < n; base += (int64_t)gridDim.x * kWave) {
        const int64_t p = base + lane;
        if (p >= n) continue;
        ForceLane<DIRECT> L;
        L.load(a, p, flags);
        double ax, ay, az, du, vsig;
        if (!twice) {
            // the upper sums pass 2 left, then the stored sides of the partners below
            const int32_t* Li = a.list + p;
            const int len = a.list_len[p];
            double lax = 0.0, lay = 0.0, laz = 0.0, ldu = 0.0;
            vsig = ld_f64(a.f[SPHV_VSIG], L.li);
            for (int e = 0; e < len; ++e) {
                if (Li[(int64_t)e * n] > (int)p) break;
                const double* sl = a.slots + (int64_t)e * n + p;
                lax += sl[0];
                lay += sl[cn];
                laz += sl[2 * cn];
                ldu += sl[3 * cn];
                vsig = sl[4 * cn] > vsig ? sl[4 * cn] : vsig;
            }
            ax = ld_f64(a.f[SPHV_AX], L.li) + lax;
            ay = ld_f64(a.f[SPHV_AY], L.li) + lay;
            az = ld_f64(a.f[SPHV_AZ], L.li) + laz;
            du = ld_f64(a.f[SPHV_UDT], L.li) + ldu;
        } else {
            // some list overflowed: every pair of p from its window, evaluated here
            auto keep = [&](const double* bnd, double sx, double sy, double sz) {
                const double rr = fmax(L.Hi, bnd[6]) * (1.0 + 1e-6);
                return box_d2(bnd, L.bx, L.by, L.bz, sx, sy, sz) < rr * rr;
            };
            // a row is kept within the largest 2h any force partner of the cell's
            // particles can have (the cover of the own force reaches)
            const double Hg = (double)a.reach_s[cell_key(L.kx, L.ky, L.kz, a.g)] * a.g.cmin;
            auto keep_cell = [&](double d2, int key) {
                const double Hc = key < 0 ? Hg : (double)__uint_as_float(a.cell_h[key]);
                const double rr = fmax(L.Hi, Hc) * (1.0 + 1e-6);
                return d2 < rr * rr;
            };
            ax = ay = az = du = 0.0;
            vsig = 2.0 * L.ci;
            walk_window<true>(a, L.kx, L.ky, L.kz, L.r, L.bx, L.by, L.bz, keep_cell, keep,
                        [&](int j, int, int, int, int, int, int) {
                            const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
                            const double dx = mi_diff(L.xi, ld_f64(a.f[SPHV_X], lj), a.g, 0);
                            const double dy = mi_diff(L.yi, ld_f64(a.f[SPHV_Y], lj), a.g, 1);
                            const double dz = mi_diff(L.zi, ld_f64(a.f[SPHV_Z], lj), a.g, 2);
                            const double r2 = dx * dx + dy * dy + dz * dz;
                            if (!(r2 < fmax(L.H2i, fc[4 * n + j]) && r2 > 0.0)) return;
                            PairTerms<KERN, DIRECT> t;
                            t.eval(a, L, j, lj, dx, dy, dz, r2);
                            const double coef = t.mj * t.B;
                            ax = fma(-coef, t.ex, ax);
                            ay = fma(-coef, t.ey, ay);
                            az = fma(-coef, t.ez, az);
                            du = du + t.mj * fma(0.5 * t.visc, t.gbar, L.Ai * t.gi) * t.w;
                            vsig = t.vs > vsig ? t.vs : vsig;
                        });
        }
        st_f64(a.f[SPHV_AX], L.li, ax);
        st_f64(a.f[SPHV_AY], L.li, ay);
        st_f64(a.f[SPHV_AZ], L.li, az);
        st_f64(a.f[SPHV_UDT], L.li, du);
        st_f64(a.f[SPHV_VSIG], L.li, vsig);
        if (!(isfinite(ax) && isfinite(ay) && isfinite(az) && isfinite(du))) flags |= SPHV_F_NONFINITE_OUTPUT;
    }
    for (int off = 32; off > 0; off >>= 1) flags |= __shfl_xor(flags, off, kWave);
    if (lane == 0 && flags) atomicOr(&a.state->flags, flags);
}

// Workgroups (one wave each) that the device holds at once for a kernel, a
// multiple of the 8 XCDs, at most kMaxPairBlocks; queried once per kernel.
template <class K>
int list_blocks(K kernel, std::atomic<int>& cache, int64_t n)
{
    int v = cache.load(std::memory_order_relaxed);
    if (v <= 0) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        v = per_cu * cus / kNumXcd * kNumXcd;
        if (v < kNumXcd) v = kNumXcd;
        if (v > kMaxPairBlocks) v = kMaxPairBlocks;
        cache.store(v, std::memory_order_relaxed);
    }
    const int64_t need = (n + kWave - 1) / kWave;
    return (int)(need < v ? (need > 0 ? need : 1) : v);
}

}  // namespace

template <class K>
static hipError_t run_list(K kernel, std::atomic<int>& cache, const PairArgs& a0, int density, hipStream_t s)
{
    PairArgs a = a0;
    a.nblocks = list_blocks(kernel, cache, a.n);
    hipLaunchKernelGGL(kernel, dim3((unsigned)a.nblocks), dim3(kWave), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_pair_fold(a, a.nblocks, density, s);
}

#define SPHV_LIST_CASE(KERNEL, D, F, DENS)                                                  \
    do {                                                                                    \
        if (kern == SPHV_KERNEL_QUARTIC) {                                                  \
            static std::atomic<int> cache_q{0};                                             \
            return run_list(KERNEL<D, F, SPHV_KERNEL_QUARTIC>, cache_q, a, DENS, s);        \
        }                                                                                   \
        static std::atomic<int> cache{0};                                                   \
        return run_list(KERNEL<D, F, SPHV_KERNEL_CUBIC>, cache, a, DENS, s);                \
    } while (0)

template <bool DIRECT, bool FP32, int KERN>
static hipError_t run_density_list(std::atomic<int>* caches, const PairArgs& a0, hipStream_t s)
{
    PairArgs a = a0;
    hipError_t e = launch_fill_u32(a.meta + META_LIST_OVF, 0u, 1, s);
    if (e != hipSuccess) return e;
    const int nb1 = list_blocks(k_density_list_build<DIRECT, FP32, KERN>, caches[0], a.n);
    hipLaunchKernelGGL((k_density_list_build<DIRECT, FP32, KERN>), dim3((unsigned)nb1), dim3(kWave), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // each of the two launches that run passes leaves per-wave counters, folded after it
    a.nblocks = list_blocks(k_density_list_pass<DIRECT, FP32, KERN>, caches[1], a.n);
    hipLaunchKernelGGL((k_density_list_pass<DIRECT, FP32, KERN>), dim3((unsigned)a.nblocks), dim3(kWave), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_pair_fold(a, a.nblocks, 1, s)) != hipSuccess) return e;
    a.nblocks = list_blocks(k_density_list_window<DIRECT, FP32, KERN>, caches[2], a.n);
    hipLaunchKernelGGL((k_density_list_window<DIRECT, FP32, KERN>), dim3((unsigned)a.nblocks), dim3(kWave), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_pair_fold(a, a.nblocks, 1, s);
}

#define SPHV_DENSITY_LIST_CASE(D, F)                                                        \
    do {                                                                                    \
        if (kern == SPHV_KERNEL_QUARTIC) {                                                  \
            static std::atomic<int> cq[3];                                                  \
            return run_density_list<D, F, SPHV_KERNEL_QUARTIC>(cq, a, s);                   \
        }                                                                                   \
        static std::atomic<int> cc[3];                                                      \
        return run_density_list<D, F, SPHV_KERNEL_CUBIC>(cc, a, s);                         \
    } while (0)

hipError_t launch_density_list(const PairArgs& a, int direct, int fp32, int kern, hipStream_t s)
{
    if (direct) {
        if (fp32) SPHV_DENSITY_LIST_CASE(true, true);
        SPHV_DENSITY_LIST_CASE(true, false);
    }
    if (fp32) SPHV_DENSITY_LIST_CASE(false, true);
    SPHV_DENSITY_LIST_CASE(false, false);
}

hipError_t launch_block_bounds(const PairArgs& a, double* blocks, int direct, int fp32, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((a.n + kWave - 1) / kWave);
    if (direct) {
        if (fp32) hipLaunchKernelGGL((k_block_bounds<true, true>), dim3(nb), dim3(kWave), 0, s, a, blocks);
        else hipLaunchKernelGGL((k_block_bounds<true, false>), dim3(nb), dim3(kWave), 0, s, a, blocks);
    } else {
        if (fp32) hipLaunchKernelGGL((k_block_bounds<false, true>), dim3(nb), dim3(kWave), 0, s, a, blocks);
        else hipLaunchKernelGGL((k_block_bounds<false, false>), dim3(nb), dim3(kWave), 0, s, a, blocks);
    }
    return hipGetLastError();
}

hipError_t launch_force_prep(const PairArgs& a, int direct, int fp32, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((a.n + 255) / 256);
    if (direct) {
        if (fp32) hipLaunchKernelGGL((k_force_prep<true, true>), dim3(nb), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_force_prep<true, false>), dim3(nb), dim3(256), 0, s, a);
    } else {
        if (fp32) hipLaunchKernelGGL((k_force_prep<false, true>), dim3(nb), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_force_prep<false, false>), dim3(nb), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

template <bool DIRECT, int KERN>
static hipError_t run_force_sym(std::atomic<int>* caches, const PairArgs& a0, hipStream_t s)
{
    PairArgs a = a0;
    hipError_t e = launch_fill_u32(a.meta + META_LIST_OVF, 0u, 1, s);
    if (e != hipSuccess) return e;
    a.nblocks = list_blocks(k_force_sym_build<DIRECT, KERN>, caches[0], a.n);
    hipLaunchKernelGGL((k_force_sym_build<DIRECT, KERN>), dim3((unsigned)a.nblocks), dim3(kWave), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_pair_fold(a, a.nblocks, 0, s)) != hipSuccess) return e;
    const int nb2 = list_blocks(k_force_sym_upper<DIRECT, KERN>, caches[1], a.n);
    hipLaunchKernelGGL((k_force_sym_upper<DIRECT, KERN>), dim3((unsigned)nb2), dim3(kWave), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nb3 = list_blocks(k_force_sym_lower<DIRECT, KERN>, caches[2], a.n);
    hipLaunchKernelGGL((k_force_sym_lower<DIRECT, KERN>), dim3((unsigned)nb3), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_force_sym(const PairArgs& a, int direct, int kern, hipStream_t s)
{
    if (direct) {
        if (kern == SPHV_KERNEL_QUARTIC) {
            static std::atomic<int> c[3];
            return run_force_sym<true, SPHV_KERNEL_QUARTIC>(c, a, s);
        }
        static std::atomic<int> c[3];
        return run_force_sym<true, SPHV_KERNEL_CUBIC>(c, a, s);
    }
    if (kern == SPHV_KERNEL_QUARTIC) {
        static std::atomic<int> c[3];
        return run_force_sym<false, SPHV_KERNEL_QUARTIC>(c, a, s);
    }
    static std::atomic<int> c[3];
    return run_force_sym<false, SPHV_KERNEL_CUBIC>(c, a, s);
}

template <bool DIRECT, bool FP32, int KERN>
static hipError_t run_force_list(std::atomic<int>* caches, const PairArgs& a0, hipStream_t s)
{
    PairArgs a = a0;
    hipError_t e = launch_fill_u32(a.meta + META_LIST_OVF, 0u, 1, s);
    if (e != hipSuccess) return e;
    a.nblocks = list_blocks(k_force_list_build<DIRECT, FP32, KERN>, caches[0], a.n);
    hipLaunchKernelGGL((k_force_list_build<DIRECT, FP32, KERN>), dim3((unsigned)a.nblocks), dim3(kWave), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_pair_fold(a, a.nblocks, 0, s)) != hipSuccess) return e;
    const int nb2 = list_blocks(k_force_list_eval<DIRECT, FP32, KERN>, caches[1], a.n);
    hipLaunchKernelGGL((k_force_list_eval<DIRECT, FP32, KERN>), dim3((unsigned)nb2), dim3(kWave), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nb3 = list_blocks(k_force_list_window<DIRECT, FP32, KERN>, caches[2], a.n);
    hipLaunchKernelGGL((k_force_list_window<DIRECT, FP32, KERN>), dim3((unsigned)nb3), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

#define SPHV_FORCE_LIST_CASE(D, F)                                                          \
    do {                                                                                    \
        if (kern == SPHV_KERNEL_QUARTIC) {                                                  \
            static std::atomic<int> cq[3];                                                  \
            return run_force_list<D, F, SPHV_KERNEL_QUARTIC>(cq, a, s);                     \
        }                                                                                   \
        static std::atomic<int> cc[3];                                                      \
        return run_force_list<D, F, SPHV_KERNEL_CUBIC>(cc, a, s);                           \
    } while (0)

hipError_t launch_force_list(const PairArgs& a, int direct, int fp32, int kern, hipStream_t s)
{
    if (direct) {
        if (fp32) SPHV_FORCE_LIST_CASE(true, true);
        SPHV_FORCE_LIST_CASE(true, false);
    }
    if (fp32) SPHV_FORCE_LIST_CASE(false, true);
    SPHV_FORCE_LIST_CASE(false, false);
}

}  // namespace sphv
