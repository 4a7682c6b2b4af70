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
#include <type_traits>

#include "k_common.h"

namespace sphv {

namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ int next_item(int32_t* head, int n_items, int xcd, int& qoff)
{
    while (qoff < kNumXcd) {
        int q = (xcd + qoff) % kNumXcd;
        int lo = (int)(((int64_t)n_items * q) / kNumXcd);
        int hi = (int)(((int64_t)n_items * (q + 1)) / kNumXcd);
        if (lo < hi) {
            int k = atomicAdd(&head[q], 1);
            if (lo + k < hi) return lo + k;
        }
        ++qoff;
    }
    return -1;
}

// Called by every lane 0 once its wave is done with the queue.
__device__ void queue_exit(int32_t* meta, int qhead, int qexit)
{
    __threadfence();
    int done = atomicAdd(&meta[qexit], 1);
    if (done == (int)gridDim.x - 1) {
        for (int q = 0; q < kNumXcd; ++q) atomicExch(&meta[qhead + q], 0);
        atomicExch(&meta[qexit], 0);
        __threadfence();
    }
}

__device__ __forceinline__ void neumaier(float& s, float& c, float x)
{
    float t = s + x;
    c += (fabsf(s) >= fabsf(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
}

// Cubic M4 spline in its truncated-power form, branch free:
//   w(q)  = (2-q)_+^3 / 4 - (1-q)_+^3      (= 1 - 1.5 q^2 + 0.75 q^3 below 1)
//   w'(q) = 3 (1-q)_+^2 - 0.75 (2-q)_+^2
// Both vanish identically for q >= 2, so no select is needed at the support
// edge and the two pieces never diverge inside a wave.
template <class R>
__device__ __forceinline__ void spline(R q, R& w, R& dw)
{
    const R a = fmax(R(2) - q, R(0));
    const R b = fmax(R(1) - q, R(0));
    const R a2 = a * a;
    const R b2 = b * b;
    w = fma(R(0.25) * a2, a, -(b2 * b));
    dw = fma(R(3), b2, R(-0.75) * a2);
}

template <class R>
__device__ __forceinline__ R spline_dw(R q)
{
    const R a = fmax(R(2) - q, R(0));
    const R b = fmax(R(1) - q, R(0));
    return fma(R(3), b * b, R(-0.75) * (a * a));
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

// Per-axis reach of a cell, guarded against windows that wrap onto themselves.
__device__ __forceinline__ void axis_reach(const PairArgs& a, int R, int r[3])
{
    bool small = false;
    for (int d = 0; d < 3; ++d) {
        r[d] = R;
        if (a.g.periodic[d] && 2 * R + 1 > a.g.n[d]) {
            r[d] = (a.g.n[d] - 1) / 2;
            small = true;
        }
    }
    if (small && threadIdx.x == 0) set_flag(a.state, SPHV_F_GRID_TOO_SMALL);
}

// Walk the window of cell (kx,ky,kz): every contiguous span of candidates with
// its periodic image (ix,iy,iz in {-1,0,1}), staged 64 at a time into LDS slot
// 'lane'.  stage(j, ix, iy, iz) is called by the lane that owns the slot;
// compute(count) runs between barriers once 64 candidates (or the rest) are in.
template <class Stage, class Compute>
__device__ __forceinline__ void for_window(const PairArgs& a, int kx, int ky, int kz, const int r[3], int lane,
                                           Stage&& stage, Compute&& compute)
{
    const int nx = a.g.n[0], ny = a.g.n[1], nz = a.g.n[2];
    int fill = 0;
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
            int x0 = kx - r[0], x1 = kx + r[0];
            // up to three spans: wrapped left part, main part, wrapped right part
            int sc0[3], sc1[3], six[3], ns = 0;
            if (a.g.periodic[0]) {
                if (x0 < 0) { sc0[ns] = x0 + nx; sc1[ns] = nx - 1; six[ns] = -1; ++ns; x0 = 0; }
                int xr = x1 >= nx ? nx - 1 : x1;
                sc0[ns] = x0; sc1[ns] = xr; six[ns] = 0; ++ns;
                if (x1 >= nx) { sc0[ns] = 0; sc1[ns] = x1 - nx; six[ns] = 1; ++ns; }
            } else {
                sc0[0] = x0 < 0 ? 0 : x0;
                sc1[0] = x1 >= nx ? nx - 1 : x1;
                six[0] = 0;
                ns = 1;
            }
            for (int sgi = 0; sgi < ns; ++sgi) {
                int jb = a.cell_start[row + sc0[sgi]];
                const int je = a.cell_start[row + sc1[sgi] + 1];
                while (jb < je) {
                    int take = je - jb;
                    if (take > kWave - fill) take = kWave - fill;
                    if (lane >= fill && lane < fill + take) stage(jb + lane - fill, six[sgi], iy, iz);
                    fill += take;
                    jb += take;
                    if (fill == kWave) {
                        __syncthreads();
                        compute(kWave);
                        __syncthreads();
                        fill = 0;
                    }
                }
            }
        }
    }
    if (fill) {
        __syncthreads();
        compute(fill);
        __syncthreads();
    }
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

template <bool DIRECT, bool FP32, bool MASKED>
__global__ __launch_bounds__(kWave) void k_density(PairArgs a)
{
    using R = typename std::conditional<FP32, float, double>::type;
    __shared__ R sx[kWave], sy[kWave], sz[kWave], sm[kWave];
    __shared__ int sj[kWave];
    __shared__ double red[3][kWave];
    __shared__ int redc[kWave];
    __shared__ int s_item;

    const int lane = threadIdx.x;
    const int n_items = a.meta[META_NITEMS];
    const int xcd = blockIdx.x % kNumXcd;
    const double eta3 = a.eta * a.eta * a.eta;
    int qoff = 0;
    unsigned long long n_final = 0, n_evals = 0;
    int maxit = 0;
    uint32_t flags = 0;

    for (;;) {
        if (lane == 0) s_item = next_item(a.meta + a.qhead, n_items, xcd, qoff);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);   // wave-uniform
        __syncthreads();
        if (item < 0) break;

        const int4 it = a.items[item];
        const int cell = it.x, first = it.y, ni = it.z;
        int tpi = kWave / ni;
        if (a.tpi > 0 && a.tpi < tpi) tpi = a.tpi;
        const int il = lane / tpi, sl = lane - il * tpi;
        const bool act = il < ni;
        const int pi = first + (act ? il : 0);
        int kx, ky, kz;
        cell_coords(cell, a.g, kx, ky, kz);
        int r[3];
        axis_reach(a, a.reach[cell], r);
        double hcap = 0.5 * (double)r[0] * a.g.cell[0];
        hcap = fmin(hcap, 0.5 * (double)r[1] * a.g.cell[1]);
        hcap = fmin(hcap, 0.5 * (double)r[2] * a.g.cell[2]);

        const Loc<DIRECT> li = locate<DIRECT>(a.acc, pi);
        R xi, yi, zi;
        double mi;
        if constexpr (FP32) {
            xi = ld_as_f32(a.f[SPHV_X], li, a.g, cell);
            yi = ld_as_f32(a.f[SPHV_Y], li, a.g, cell);
            zi = ld_as_f32(a.f[SPHV_Z], li, a.g, cell);
            mi = (double)ld_as_f32(a.f[SPHV_M], li, a.g, cell);
        } else {
            xi = ld_f64(a.f[SPHV_X], li);
            yi = ld_f64(a.f[SPHV_Y], li);
            zi = ld_f64(a.f[SPHV_Z], li);
            mi = ld_f64(a.f[SPHV_M], li);
        }
        double h = ld_f64(a.f[SPHV_H], li);
        bool done = !act;

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

            auto stage = [&](int j, int ix, int iy, int iz) {
                const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
                if constexpr (FP32) {
                    const int kj = a.key_sorted[j];
                    int jx, jy, jz;
                    cell_coords(kj, a.g, jx, jy, jz);
                    const int dkx = jx - kx + ix * a.g.n[0];
                    const int dky = jy - ky + iy * a.g.n[1];
                    const int dkz = jz - kz + iz * a.g.n[2];
                    sx[lane] = ld_as_f32(a.f[SPHV_X], lj, a.g, kj) + __double2float_rn((double)dkx * a.g.cell[0]);
                    sy[lane] = ld_as_f32(a.f[SPHV_Y], lj, a.g, kj) + __double2float_rn((double)dky * a.g.cell[1]);
                    sz[lane] = ld_as_f32(a.f[SPHV_Z], lj, a.g, kj) + __double2float_rn((double)dkz * a.g.cell[2]);
                    sm[lane] = ld_as_f32(a.f[SPHV_M], lj, a.g, kj);
                } else {
                    sx[lane] = ld_f64(a.f[SPHV_X], lj) + (double)ix * a.g.len[0];
                    sy[lane] = ld_f64(a.f[SPHV_Y], lj) + (double)iy * a.g.len[1];
                    sz[lane] = ld_f64(a.f[SPHV_Z], lj) + (double)iz * a.g.len[2];
                    sm[lane] = ld_f64(a.f[SPHV_M], lj);
                }
                sj[lane] = j;
            };

            // one candidate's contribution at the current h; in == false turns
            // it into the neutral element (zero w and w' add nothing)
            auto term = [&](int t, R r2, bool in, R& p0, R& p1, R& p2) {
                const R r = r2 * rsqrt_nr(fmax(r2, Tiny<R>::v));
                const R q = r * hin;
                R w, dw;
                spline(q, w, dw);
                w = in ? w : (R)0;
                dw = in ? dw : (R)0;
                const R m = sm[t];
                p0 = fma(m, w, p0);
                p1 = p1 + w;
                p2 = fma(m, fma(q, dw, (R)3 * w), p2);
                // the self pair (r = 0) enters the sums but is not counted
                cnt += (in && (r2 > (R)0 || sj[t] != pi)) ? 1 : 0;
            };

            auto compute = [&](int count) {
                if (done) return;
                R p0 = 0, p1 = 0, p2 = 0;
                if constexpr (MASKED) {
                    // every candidate evaluated, out-of-range terms are the neutral element
                    for (int t = sl; t < count; t += tpi) {
                        const R dx = xi - sx[t];
                        const R dy = yi - sy[t];
                        const R dz = zi - sz[t];
                        const R r2 = dx * dx + dy * dy + dz * dz;
                        term(t, r2, r2 < H2, p0, p1, p2);
                    }
                } else {
                    // test every candidate of this lane, then evaluate only the hits,
                    // in the same increasing order
                    uint64_t hits = 0;
                    int k = 0;
#pragma unroll 4
                    for (int t = sl; t < count; t += tpi, ++k) {
                        const R dx = xi - sx[t];
                        const R dy = yi - sy[t];
                        const R dz = zi - sz[t];
                        const R r2 = dx * dx + dy * dy + dz * dz;
                        hits |= (r2 < H2 ? 1ull : 0ull) << k;
                    }
                    while (hits) {
                        const int kk = __builtin_ctzll(hits);
                        hits &= hits - 1;
                        const int t = sl + kk * tpi;
                        const R dx = xi - sx[t];
                        const R dy = yi - sy[t];
                        const R dz = zi - sz[t];
                        const R r2 = dx * dx + dy * dy + dz * dz;
                        term(t, r2, true, p0, p1, p2);
                    }
                }
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

            for_window(a, kx, ky, kz, r, lane, stage, compute);

            if constexpr (FP32) {
                t0 = (double)f0 + (double)c0;
                t1 = (double)f1 + (double)c1;
                t2 = (double)f2 + (double)c2;
            }
            if (tpi > 1) {
                red[0][lane] = t0;
                red[1][lane] = t1;
                red[2][lane] = t2;
                redc[lane] = cnt;
                __syncthreads();
                if (act) {
                    const int b = il * tpi;
                    t0 = t1 = t2 = 0.0;
                    cnt = 0;
                    for (int k = 0; k < tpi; ++k) {
                        t0 += red[0][b + k];
                        t1 += red[1][b + k];
                        t2 += red[2][b + k];
                        cnt += redc[b + k];
                    }
                }
                __syncthreads();
            }

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
                    flags |= SPHV_F_H_CAP_HIT;
                }
                const bool conv = fabs(hn - h) <= a.tol * h;
                if (sl == 0) n_evals += (unsigned long long)cnt;
                if (conv || pass + 1 >= a.max_iter) {
                    if (!conv) flags |= SPHV_F_H_NOT_CONVERGED;
                    const double omega = 1.0 + h / (3.0 * rho) * drho;
                    const double wcount = (4.0 * kPi / 3.0) * (8.0 * h3) * nsum;
                    if (!(isfinite(rho) && isfinite(omega))) flags |= SPHV_F_NONFINITE_OUTPUT;
                    if (sl == 0) {
                        st_f64(a.f[SPHV_H], li, h);
                        st_f64(a.f[SPHV_RHO], li, rho);
                        st_f64(a.f[SPHV_OMEGA], li, omega);
                        st_f64(a.f[SPHV_WCOUNT], li, wcount);
                        n_final += (unsigned long long)cnt;
                    }
                    maxit = pass + 1 > maxit ? pass + 1 : maxit;
                    done = true;
                } else {
                    h = hn;
                }
            }
            if (__all(done)) break;
        }
    }

    n_final = wave_sum_u64(n_final);
    n_evals = wave_sum_u64(n_evals);
    maxit = wave_max_i(maxit);
    for (int off = 32; off > 0; off >>= 1) flags |= __shfl_xor(flags, off, kWave);
    if (lane == 0) {
        if (n_final) {
            atomicAdd(&a.state->pairs_density, n_final);
            atomicAdd(&a.state->pairs_total, n_final);
        }
        if (n_evals) atomicAdd(&a.state->pair_evals_density, n_evals);
        if (maxit) atomicMax(&a.state->max_iters, maxit);
        if (flags) atomicOr(&a.state->flags, flags);
        queue_exit(a.meta, a.qhead, a.qexit);
    }
}

// ================================================================== force

template <bool DIRECT, bool FP32, bool MASKED>
__global__ __launch_bounds__(kWave) void k_force(PairArgs a)
{
    using R = typename std::conditional<FP32, float, double>::type;
    // staged j data
    __shared__ R sx[kWave], sy[kWave], sz[kWave], svx[kWave], svy[kWave], svz[kWave];
    __shared__ R sm[kWave], sH2[kWave], shinv[kWave], snorm[kWave], srho[kWave], sA[kWave], sc[kWave], sal[kWave];
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
    int qoff = 0;
    unsigned long long n_pairs = 0;
    uint32_t flags = 0;
    (void)gm;

    for (;;) {
        if (lane == 0) s_item = next_item(a.meta + a.qhead, n_items, xcd, qoff);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);   // wave-uniform
        __syncthreads();
        if (item < 0) break;

        const int4 it = a.items[item];
        const int cell = it.x, first = it.y, ni = it.z;
        int tpi = kWave / ni;
        if (a.tpi > 0 && a.tpi < tpi) tpi = a.tpi;
        const int il = lane / tpi, sl = lane - il * tpi;
        const bool act = il < ni;
        const int pi = first + (act ? il : 0);
        int kx, ky, kz;
        cell_coords(cell, a.g, kx, ky, kz);
        int r[3];
        axis_reach(a, a.reach[cell], r);

        // local particle i and its derived quantities
        const Loc<DIRECT> li = locate<DIRECT>(a.acc, pi);
        R xi, yi, zi, vxi, vyi, vzi, hi, rhoi, omi, ui, ali;
        if constexpr (FP32) {
            xi = ld_as_f32(a.f[SPHV_X], li, a.g, cell);
            yi = ld_as_f32(a.f[SPHV_Y], li, a.g, cell);
            zi = ld_as_f32(a.f[SPHV_Z], li, a.g, cell);
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

        auto stage = [&](int j, int ix, int iy, int iz) {
            const Loc<DIRECT> lj = locate<DIRECT>(a.acc, j);
            R u_, rho_, om_, h_;
            if constexpr (FP32) {
                const int kj = a.key_sorted[j];
                int jx, jy, jz;
                cell_coords(kj, a.g, jx, jy, jz);
                const int dkx = jx - kx + ix * a.g.n[0];
                const int dky = jy - ky + iy * a.g.n[1];
                const int dkz = jz - kz + iz * a.g.n[2];
                sx[lane] = ld_as_f32(a.f[SPHV_X], lj, a.g, kj) + __double2float_rn((double)dkx * a.g.cell[0]);
                sy[lane] = ld_as_f32(a.f[SPHV_Y], lj, a.g, kj) + __double2float_rn((double)dky * a.g.cell[1]);
                sz[lane] = ld_as_f32(a.f[SPHV_Z], lj, a.g, kj) + __double2float_rn((double)dkz * a.g.cell[2]);
                svx[lane] = ld_as_f32(a.f[SPHV_VX], lj, a.g, kj);
                svy[lane] = ld_as_f32(a.f[SPHV_VY], lj, a.g, kj);
                svz[lane] = ld_as_f32(a.f[SPHV_VZ], lj, a.g, kj);
                sm[lane] = ld_as_f32(a.f[SPHV_M], lj, a.g, kj);
                sal[lane] = (R)0.5 * ld_as_f32(a.f[SPHV_ALPHA], lj, a.g, kj);
                h_ = ld_as_f32(a.f[SPHV_H], lj, a.g, kj);
                rho_ = ld_as_f32(a.f[SPHV_RHO], lj, a.g, kj);
                om_ = ld_as_f32(a.f[SPHV_OMEGA], lj, a.g, kj);
                u_ = ld_as_f32(a.f[SPHV_U], lj, a.g, kj);
            } else {
                sx[lane] = ld_f64(a.f[SPHV_X], lj) + (double)ix * a.g.len[0];
                sy[lane] = ld_f64(a.f[SPHV_Y], lj) + (double)iy * a.g.len[1];
                sz[lane] = ld_f64(a.f[SPHV_Z], lj) + (double)iz * a.g.len[2];
                svx[lane] = ld_f64(a.f[SPHV_VX], lj);
                svy[lane] = ld_f64(a.f[SPHV_VY], lj);
                svz[lane] = ld_f64(a.f[SPHV_VZ], lj);
                sm[lane] = ld_f64(a.f[SPHV_M], lj);
                sal[lane] = (R)0.5 * ld_f64(a.f[SPHV_ALPHA], lj);
                h_ = ld_f64(a.f[SPHV_H], lj);
                rho_ = ld_f64(a.f[SPHV_RHO], lj);
                om_ = ld_f64(a.f[SPHV_OMEGA], lj);
                u_ = ld_f64(a.f[SPHV_U], lj);
            }
            const R P_ = gm1 * rho_ * u_;
            const R hv = (R)1 / h_;
            const R hv2 = hv * hv;
            const R H_ = (R)2 * h_;
            sH2[lane] = H_ * H_;
            shinv[lane] = hv;
            snorm[lane] = hv2 * hv2 / (R)kPi;
            srho[lane] = rho_;
            sA[lane] = P_ / (om_ * rho_ * rho_);
            sc[lane] = sqrt(ggm1 * u_);
            sj[lane] = j;
        };

        // (2 max(h_i, h_j))^2 == max((2 h_i)^2, (2 h_j)^2): squaring and its
        // rounding are monotone, so the test is exact and per side
        const R Hi = (R)2 * hi;
        const R H2i = Hi * Hi;

        // one pair's contribution; live == false gives the neutral element
        auto term = [&](int t, R dx, R dy, R dz, R r2, bool live, R& pax, R& pay, R& paz, R& pdu) {
            const R y = rsqrt_nr(live ? r2 : (R)1);
            const R r = r2 * y;
            const R gi = spline_dw(r * hinvi) * normi;
            const R gj = spline_dw(r * shinv[t]) * snorm[t];
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

        auto compute = [&](int count) {
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
                uint64_t hits = 0;
                int k = 0;
#pragma unroll 4
                for (int t = sl; t < count; t += tpi, ++k) {
                    const R dx = xi - sx[t];
                    const R dy = yi - sy[t];
                    const R dz = zi - sz[t];
                    const R r2 = dx * dx + dy * dy + dz * dz;
                    hits |= (r2 < fmax(H2i, sH2[t]) ? 1ull : 0ull) << k;
                }
                while (hits) {
                    const int kk = __builtin_ctzll(hits);
                    hits &= hits - 1;
                    const int t = sl + kk * tpi;
                    const R dx = xi - sx[t];
                    const R dy = yi - sy[t];
                    const R dz = zi - sz[t];
                    const R r2 = dx * dx + dy * dy + dz * dz;
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

        for_window(a, kx, ky, kz, r, lane, stage, compute);

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
    if (lane == 0) {
        if (n_pairs) {
            atomicAdd(&a.state->pairs_force, n_pairs);
            atomicAdd(&a.state->pairs_total, n_pairs);
        }
        if (flags) atomicOr(&a.state->flags, flags);
        queue_exit(a.meta, a.qhead, a.qexit);
    }
}

// ============================================ time step and conservation sums

struct RedArgs {
    FieldRef in[6];     // m vx vy vz u h   (records, through the index)
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

int pair_grid_blocks(int64_t max_items)
{
    // persistent grid: enough single-wave workgroups to fill 256 CUs several
    // times over, a multiple of the 8 XCDs
    int64_t b = 256 * 20;
    if (max_items < b) b = (max_items + kNumXcd - 1) / kNumXcd * kNumXcd;
    if (b < kNumXcd) b = kNumXcd;
    return (int)b;
}

#define SPHV_DISPATCH(KERNEL, a, direct, fp32, masked, s)                                                   \
    do {                                                                                                   \
        dim3 grid((unsigned)(a).nblocks), block(kWave);                                                    \
        if (direct) {                                                                                      \
            if (fp32) {                                                                                    \
                if (masked) hipLaunchKernelGGL((KERNEL<true, true, true>), grid, block, 0, s, a);          \
                else hipLaunchKernelGGL((KERNEL<true, true, false>), grid, block, 0, s, a);                \
            } else {                                                                                       \
                if (masked) hipLaunchKernelGGL((KERNEL<true, false, true>), grid, block, 0, s, a);         \
                else hipLaunchKernelGGL((KERNEL<true, false, false>), grid, block, 0, s, a);               \
            }                                                                                              \
        } else {                                                                                           \
            if (fp32) {                                                                                    \
                if (masked) hipLaunchKernelGGL((KERNEL<false, true, true>), grid, block, 0, s, a);         \
                else hipLaunchKernelGGL((KERNEL<false, true, false>), grid, block, 0, s, a);               \
            } else {                                                                                       \
                if (masked) hipLaunchKernelGGL((KERNEL<false, false, true>), grid, block, 0, s, a);        \
                else hipLaunchKernelGGL((KERNEL<false, false, false>), grid, block, 0, s, a);              \
            }                                                                                              \
        }                                                                                                  \
    } while (0)

hipError_t launch_density(const PairArgs& a, int direct, int fp32, int masked, hipStream_t s)
{
    SPHV_DISPATCH(k_density, a, direct, fp32, masked, s);
    return hipGetLastError();
}

hipError_t launch_force(const PairArgs& a, int direct, int fp32, int masked, hipStream_t s)
{
    SPHV_DISPATCH(k_force, a, direct, fp32, masked, s);
    return hipGetLastError();
}

hipError_t launch_force_reduce(const FieldRef* in6, const Access& rec, const FieldRef* out5, const Access& outacc,
                               int out_direct, DevState* st, double cfl, int64_t n, double* partials,
                               hipStream_t s)
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
    if (out_direct)
        hipLaunchKernelGGL(k_reduce_part<true>, dim3((unsigned)nb), dim3(kRedThreads), 0, s, r);
    else
        hipLaunchKernelGGL(k_reduce_part<false>, dim3((unsigned)nb), dim3(kRedThreads), 0, s, r);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, s, r, nb);
    return hipGetLastError();
}

}  // namespace sphv
