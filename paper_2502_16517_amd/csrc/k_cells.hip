// Cell binning, stable counting sort into cells, per-cell reach and the work
// items of the pair loops (paper Sec. 2.1: particles are sorted into cells so
// that only neighbouring cells interact; Sec. 5.2: the particles of one cell
// form one chunk, indexed by CSR-like offsets).
//
// Pipeline of cells_build (all on one stream, no host synchronisation):
//   clear       counts, hmax, meta := 0
//   bin         key_i, counts[key]++, hmax[key] = max 2 h headroom, flags
//   scan        cell_start = exclusive scan of counts, cursor = cell_start
//   place       perm_tmp[cursor[key_i]++] = i       (cell-grouped, any order)
//   segsort     perm[cell] = ascending record indices of the cell: the stable
//               order (ties by index), key_sorted, density reach
//   row groups  per row of cells: runs of sparse cells sharing one work item
//   scan, items offsets of each cell's items, then the items (cell, first,
//               count <= 64, cells) and n_items in the same second pass
// and of the force window, at the start of sph_force, from the converged h:
//   own reach per cell, its cover (three separable mask passes), exact window.
#include "k_common.h"

namespace sphv {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;   // 1024 elements per block

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

// Zeroes up to three ranges in one launch (a fill kernel, so that captured
// graphs hold no memset nodes).
struct Clear3 {
    uint32_t* p[3];
    int64_t n[3];
};

__global__ void k_clear3(Clear3 c)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int r = 0; r < 3; ++r)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < c.n[r]; i += stride) c.p[r][i] = 0u;
}

hipError_t clear3(uint32_t* p0, int64_t n0, uint32_t* p1, int64_t n1, uint32_t* p2, int64_t n2, hipStream_t s)
{
    Clear3 c{{p0, p1, p2}, {n0, n1, n2}};
    const int64_t m = std::max(n0, std::max(n1, n2));
    const unsigned b = (unsigned)std::max<int64_t>(1, std::min<int64_t>((m + 255) / 256, 2048));
    hipLaunchKernelGGL(k_clear3, dim3(b), dim3(256), 0, s, c);
    return hipGetLastError();
}

__global__ void k_state_init(DevState* st, int full)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (full) {
        uint32_t* w = (uint32_t*)st;
        for (size_t k = 0; k < sizeof(DevState) / 4; ++k) w[k] = 0u;
        return;
    }
    st->pairs_density = 0ull;
    st->pairs_force = 0ull;
    st->pair_evals_density = 0ull;
    st->max_iters = 0;
}

// Cell key and support bits of one particle; flags non-finite input and
// particles outside an open box.
__device__ __forceinline__ void bin_one(const double c[3], double h, const Geom& g, DevState* st, int& kk,
                                        uint32_t& hbits, int& sub)
{
    bool finite = isfinite(c[0]) && isfinite(c[1]) && isfinite(c[2]);
    int k[3];
    int s[3];
    bool outside = false;
    for (int d = 0; d < 3; ++d) {
        // k_d = clamp(floor((x_d - lo_d) * inv_cell_d), 0, n_d - 1), each step rounded
        double tr = __dmul_rn(__dsub_rn(c[d], g.lo[d]), g.inv_cell[d]);
        if (!isfinite(tr)) tr = 0.0;
        double t = floor(tr);
        if (t < 0.0) { t = 0.0; outside = true; }
        if (t > (double)(g.n[d] - 1)) { t = (double)(g.n[d] - 1); outside = true; }
        k[d] = (int)t;
        // sub-cell inside the cell: floor((t_raw - k) 2^kSubBits), clamped
        double q = floor(__dmul_rn(__dsub_rn(tr, t), (double)(1 << kSubBits)));
        q = q < 0.0 ? 0.0 : (q > (double)((1 << kSubBits) - 1) ? (double)((1 << kSubBits) - 1) : q);
        s[d] = (int)q;
    }
    kk = finite ? cell_key(k[0], k[1], k[2], g) : 0;
    // Morton index: bit b of s_x, s_y, s_z at bits 3b, 3b + 1, 3b + 2
    sub = 0;
    for (int b = 0; b < kSubBits; ++b)
        for (int d = 0; d < 3; ++d) sub |= ((s[d] >> b) & 1) << (3 * b + d);
    if (!finite) sub = 0;
    // support radius with headroom; positive floats order like their bits
    float H = __double2float_ru(2.0 * h * g.headroom);
    if (!(isfinite(h) && h > 0.0)) {
        set_flag(st, SPHV_F_NONFINITE_INPUT);
        H = 0.0f;
    }
    hbits = __float_as_uint(H);
    if (!finite) set_flag(st, SPHV_F_NONFINITE_INPUT);
    // open axes: outside the grid; periodic axes: outside [lo, lo + len), the
    // range kick_drift wraps into (an unwrapped coordinate is binned into an
    // edge cell whose window would miss some of its pairs)
    bool out_of_box = false;
    for (int d = 0; d < 3; ++d) {
        if (g.periodic[d]) out_of_box |= !(c[d] >= g.lo[d] && c[d] < __dadd_rn(g.lo[d], g.len[d]));
        else out_of_box |= outside;
    }
    if (finite && out_of_box) set_flag(st, SPHV_F_OUT_OF_BOX);
}

__global__ void k_bin(const FieldRef fx, const FieldRef fy, const FieldRef fz, const FieldRef fh,
                      uint64_t stride, const uint64_t* ptrs, Geom g, int64_t n, int32_t* key, int32_t* sub,
                      int32_t* counts, uint32_t* hmax_bits, DevState* st)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t rb = ptrs ? ptrs[i] : (uint64_t)i * stride;
    auto at = [&](const FieldRef& f) { return (const double*)((uintptr_t)f.base + f.off + rb); };
    double c[3];
    c[0] = *at(fx);
    c[1] = *at(fy);
    c[2] = *at(fz);
    const double h = *at(fh);
    int kk, sb;
    uint32_t hb;
    bin_one(c, h, g, st, kk, hb, sb);
    key[i] = kk;
    sub[i] = sb;
    atomicAdd(&counts[kk], 1);
    atomicMax(&hmax_bits[kk], hb);
}

// k_bin on records staged through LDS; consecutive particles of one cell (a
// lattice row, say) add to their cell's counters once per run of lanes.
__global__ __launch_bounds__(kStageThreads) void k_bin_staged(const FieldRef fx, const FieldRef fy, const FieldRef fz,
                                                              const FieldRef fh, StagePlan sp, uint64_t stride,
                                                              Geom g, int64_t n, int32_t* key, int32_t* sub,
                                                              int32_t* counts, uint32_t* hmax_bits, DevState* st)
{
    extern __shared__ uint4 tile[];
    const int64_t r0 = (int64_t)blockIdx.x * kStageThreads;
    stage_in(tile, fx.base, stride, nullptr, r0, n, sp);
    const int64_t i = r0 + threadIdx.x;
    const bool valid = i < n;
    int kk = 0;
    uint32_t hb = 0;
    if (valid) {
        const LocTile l{(char*)&tile[threadIdx.x * sp.nch] - (uint64_t)sp.c0 * 16};
        const double c[3] = {*(const double*)l.at(fx), *(const double*)l.at(fy), *(const double*)l.at(fz)};
        int sb;
        bin_one(c, *(const double*)l.at(fh), g, st, kk, hb, sb);
        key[i] = kk;
        sub[i] = sb;
    }
    const int head = run_head(kk, valid);
    hb = run_max_upto(hb, head);
    if (run_tail(kk, valid) && valid) {
        atomicAdd(&counts[kk], (int)(threadIdx.x & (kWave - 1)) - head + 1);
        atomicMax(&hmax_bits[kk], hb);
    }
}

// ---- exclusive scan of int32 (three passes)

__device__ int block_scan_excl(int v, int* lds, int& total)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int add = t >= off ? lds[t - off] : 0;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    total = lds[kScanThreads - 1];
    int excl = lds[t] - v;
    __syncthreads();
    return excl;
}

// exclusive scan of the block totals part[0..nb) in place; part[nb] = grand total
__device__ void scan_parts(int32_t* part, int64_t nb, int* lds)
{
    int carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        int64_t b = b0 + threadIdx.x;
        int v = b < nb ? part[b] : 0;
        int total;
        int ex = block_scan_excl(v, lds, total);
        if (b < nb) part[b] = carry + ex;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) part[nb] = carry;
}

// Block totals; the block that finishes last (ticket nb - 1 on a counter that
// cells_build zeroes) then scans them, so no separate launch is needed.
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t* in, int64_t m, int32_t* part,
                                                              int32_t* ticket)
{
    __shared__ int lds[kScanThreads];
    __shared__ int last;
    int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < m) s += in[base + k];
    int total;
    block_scan_excl(s, lds, total);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = total;
        __threadfence();                  // the total is visible before the ticket is taken
        last = atomicAdd(ticket, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();                      // every other block's total is visible from here
    scan_parts(part, gridDim.x, lds);
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t* in, int64_t m, const int32_t* part,
                                                             int32_t* out, int32_t* out2)
{
    __shared__ int lds[kScanThreads];
    int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < m ? in[base + k] : 0;
        s += v[k];
    }
    int total;
    int ex = block_scan_excl(s, lds, total) + part[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < m) {
            out[base + k] = ex;
            if (out2) out2[base + k] = ex;
        }
        ex += v[k];
    }
    int64_t nb = (m + kScanTile - 1) / kScanTile;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[m] = part[nb];
}

// ticket: a zeroed counter of its own for each scan between two zeroings
hipError_t scan_excl(const int32_t* in, int64_t m, int32_t* part, int32_t* out, int32_t* out2, int32_t* ticket,
                     hipStream_t s)
{
    int64_t nb = (m + kScanTile - 1) / kScanTile;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, m, part, ticket);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, m, part, out, out2);
    return hipGetLastError();
}

// Each particle takes a slot of its cell; a run of lanes with one cell takes
// its slots with one atomic (the order inside a cell is fixed by k_segsort).
__global__ void k_place(const int32_t* key, int64_t n, int32_t* cursor, int32_t* perm_tmp)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    const int k = valid ? key[i] : 0;
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int head = run_head(k, valid);
    // the run's last lane (lane 63 always ends a run)
    const int tail = (int)__builtin_ctzll(__ballot(run_tail(k, valid)) & (~0ull << lane));
    int base = 0;
    if (valid && lane == tail) base = atomicAdd(&cursor[k], tail - head + 1);
    base = __shfl(base, tail, kWave);
    if (valid) perm_tmp[base + lane - head] = (int32_t)i;
}

constexpr int kSortThreads = 128;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kSortLds = 2048;       // per-wave LDS capacity (64-bit keys), a power of two

// One wave per pair of cells (grid-stride): order each cell's record indices
// ascending, which, since the indices are distinct, is the stable order of the
// sort; inside a cell of more than kDense particles the order is by sub-cell
// code first (the second level of the cells), then by index.  Two cells of at
// most 32 particles are sorted side by side, one per half-wave; otherwise the
// cells are sorted one after the other.
__global__ __launch_bounds__(kSortThreads) void k_segsort(const int32_t* cell_start, const int32_t* perm_tmp,
                                                          const int32_t* sub, int32_t* perm, int32_t* key_sorted,
                                                          const uint32_t* hmax_bits, int32_t* reach_d,
                                                          Geom g, int64_t nc)
{
    __shared__ uint64_t lds[kSortWaves][kSortLds];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
    uint64_t* buf = lds[w];
    int64_t wave_id = (int64_t)blockIdx.x * kSortWaves + w;
    int64_t nwaves = (int64_t)gridDim.x * kSortWaves;
    auto reach_of = [&](int64_t c, int cnt) {
        int R = 0;
        if (cnt > 0) {
            float H = __uint_as_float(hmax_bits[c]);
            R = (int)ceil((double)H / g.cmin);
            if (R < 1) R = 1;
        }
        reach_d[c] = R;
    };
    auto sort_cell = [&](int64_t c, int b, int cnt) {
        if (cnt <= kWave) {
            int v = lane < cnt ? perm_tmp[b + lane] : 0x7fffffff;
            int rank = 0;
            for (int k = 0; k < cnt; ++k) {
                int u = __shfl(v, k, kWave);
                rank += u < v;
            }
            if (lane < cnt) {
                perm[b + rank] = v;
                key_sorted[b + lane] = (int32_t)c;
            }
        } else if (cnt <= kSortLds) {
            // a dense cell: bitonic sort of the keys (sub-cell code, index) in
            // LDS, padded to a power of two with keys above every real one
            int pw = kWave;
            while (pw < cnt) pw <<= 1;
            for (int k = lane; k < pw; k += kWave) {
                uint64_t key = ~0ull;
                if (k < cnt) {
                    const int v = perm_tmp[b + k];
                    key = ((uint64_t)(uint32_t)sub[v] << 32) | (uint32_t)v;
                }
                buf[k] = key;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_s_waitcnt(0);
            for (int kk = 2; kk <= pw; kk <<= 1) {
                for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                    for (int i = lane; i < pw; i += kWave) {
                        const int l = i ^ jj;
                        if (l > i) {
                            const uint64_t x = buf[i], y = buf[l];
                            const bool up = (i & kk) == 0;
                            if ((x > y) == up) {
                                buf[i] = y;
                                buf[l] = x;
                            }
                        }
                    }
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_s_waitcnt(0);
                }
            }
            for (int k = lane; k < cnt; k += kWave) {
                perm[b + k] = (int32_t)(uint32_t)(buf[k] & 0xffffffffull);
                key_sorted[b + k] = (int32_t)c;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_s_waitcnt(0);
        } else {
            for (int k = lane; k < cnt; k += kWave) {
                const int v = perm_tmp[b + k];
                const int sv = sub[v];
                int rank = 0;
                for (int t = 0; t < cnt; ++t) {
                    const int u = perm_tmp[b + t];
                    const int su = sub[u];
                    rank += (su < sv || (su == sv && u < v)) ? 1 : 0;
                }
                perm[b + rank] = v;
                key_sorted[b + k] = (int32_t)c;
            }
        }
        if (lane == 0) reach_of(c, cnt);
    };
    for (int64_t pr = wave_id; 2 * pr < nc; pr += nwaves) {
        const int64_t c0 = 2 * pr;
        const bool two = c0 + 1 < nc;
        const int b0 = cell_start[c0], b1 = cell_start[c0 + 1];
        const int e1 = two ? cell_start[c0 + 2] : b1;
        const int cnt0 = b1 - b0, cnt1 = e1 - b1;
        if (two && cnt0 <= kWave / 2 && cnt1 <= kWave / 2) {
            const int half = lane >> 5, hl = lane & 31;
            const int b = half ? b1 : b0, cnt = half ? cnt1 : cnt0;
            const int v = hl < cnt ? perm_tmp[b + hl] : 0x7fffffff;
            const int kmax = cnt0 > cnt1 ? cnt0 : cnt1;
            int rank = 0;
            for (int k = 0; k < kmax; ++k) {
                const int u = __shfl(v, (half << 5) + k, kWave);
                rank += (k < cnt && u < v) ? 1 : 0;
            }
            if (hl < cnt) {
                perm[b + rank] = v;
                key_sorted[b + hl] = (int32_t)(c0 + half);
            }
            if (hl == 0) reach_of(c0 + half, cnt);
        } else {
            sort_cell(c0, b0, cnt0);
            if (two) sort_cell(c0 + 1, b1, cnt1);
        }
    }
}

// Work items, one wave per row of cells along x.  A cell with more than
// kSparse particles is its own item (split at 64).  Runs of consecutive sparse
// cells of one row (empty cells included) whose density reach is at most
// kGroupReach and equal, and whose neighbourhood of +-kGroupReach cells in y,
// z and beyond the run in x holds only sparse cells, form one item of at most
// kGroupLen cells and kGroupMax particles; its window is the run widened by
// the reach, and on a periodic x axis it must not wrap onto itself (2 R + cells
// <= n_x).  Items are (first cell, first sorted position, particles, cells).
// Pass 1 counts the items of every row, pass 2 writes them at the row's offset.
constexpr int kSparse = 8;
constexpr int kGroupMax = 24;
constexpr int kGroupLen = 6;
constexpr int kGroupReach = 2;
constexpr int kRowMax = 1024;   // rows up to this length are staged in LDS and grouped

// One wave per row: lanes stage the row's counts and reaches and, per column x,
// whether every cell within +-kGroupReach of it (in x, y and z) is sparse;
// lane 0 then walks the row.  For every cell c it leaves gx[c], the cells
// covered by the items that start at c (0 inside a run), and nit[c], the number
// of those items; k_scan_items writes them at the exclusive scan of nit.
__global__ __launch_bounds__(kWave) void k_row_groups(const int32_t* cell_start, const int32_t* counts,
                                                      const int32_t* reach_d, Geom g, int32_t* nit, int32_t* gxo)
{
    __shared__ int scnt[kRowMax], srch[kRowMax], scol[kRowMax];
    __shared__ uint8_t sok[kRowMax];
    const int lane = threadIdx.x;
    const int64_t row = blockIdx.x;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int64_t base = row * nx;
    const int ky = (int)(row % ny), kz = (int)(row / ny);
    const bool staged = nx <= kRowMax;
    if (staged) {
        for (int x = lane; x < nx; x += kWave) {
            scnt[x] = counts[base + x];
            srch[x] = reach_d[base + x];
            // densest cell of column x over the rows within +-kGroupReach in y
            // and z: all 25 loads issued before any is used
            int rows[2 * kGroupReach + 1][2 * kGroupReach + 1];
#pragma unroll
            for (int dz = -kGroupReach; dz <= kGroupReach; ++dz) {
#pragma unroll
                for (int dy = -kGroupReach; dy <= kGroupReach; ++dy) {
                    int z = kz + dz, y = ky + dy;
                    bool in = true;
                    if (z < 0 || z >= nz) {
                        in = in && g.periodic[2];
                        z = z < 0 ? z + nz : z - nz;
                    }
                    if (y < 0 || y >= ny) {
                        in = in && g.periodic[1];
                        y = y < 0 ? y + ny : y - ny;
                    }
                    // a wrapped index of a short periodic axis may still be out of
                    // range (n < 2 kGroupReach + 1): such a row is skipped
                    in = in && z >= 0 && z < nz && y >= 0 && y < ny;
                    rows[dz + kGroupReach][dy + kGroupReach] = in ? counts[((int64_t)z * ny + y) * nx + x] : 0;
                }
            }
            int m = 0;
#pragma unroll
            for (int a = 0; a < 2 * kGroupReach + 1; ++a)
#pragma unroll
                for (int b = 0; b < 2 * kGroupReach + 1; ++b) m = rows[a][b] > m ? rows[a][b] : m;
            scol[x] = m;
        }
        __syncthreads();
        // column x may join a run: its whole +-kGroupReach neighbourhood is sparse
        for (int x = lane; x < nx; x += kWave) {
            bool ok = true;
            for (int d = -kGroupReach; d <= kGroupReach; ++d) {
                int xx = x + d;
                if (xx < 0 || xx >= nx) {
                    if (!g.periodic[0]) continue;
                    xx = xx < 0 ? xx + nx : xx - nx;
                }
                ok = ok && scol[xx] <= kSparse;
            }
            sok[x] = ok ? 1 : 0;
        }
    }
    __syncthreads();
    const bool px_ok = !g.periodic[0] || 2 * kGroupReach + 1 <= nx;
    if (staged && nx <= kWave) {
        // rows of at most 64 cells: lane x holds column x, and the whole wave
        // walks the row with lane reads (the walk is scalar, no LDS round trips)
        const int cnt = lane < nx ? scnt[lane] : 0;
        const int rch = lane < nx ? srch[lane] : 0;
        const int okl = lane < nx ? sok[lane] : 0;
        int my_gx = 0, my_nit = 0;
        int x = 0;
        while (x < nx) {
            const int c0 = __builtin_amdgcn_readlane(cnt, x);
            const int r0 = __builtin_amdgcn_readlane(rch, x);
            const int ok0 = __builtin_amdgcn_readlane(okl, x);
            if (!(px_ok && ok0 && (c0 == 0 || r0 <= kGroupReach))) {
                if (lane == x) {
                    my_gx = 1;
                    my_nit = (c0 + kWave - 1) / kWave;
                }
                ++x;
                continue;
            }
            int R = c0 > 0 ? r0 : 0, tot = c0, gx = 1;
            while (x + gx < nx && gx < kGroupLen && __builtin_amdgcn_readlane(okl, x + gx)) {
                const int c2 = __builtin_amdgcn_readlane(cnt, x + gx);
                if (tot + c2 > kGroupMax) break;
                const int r2 = c2 > 0 ? __builtin_amdgcn_readlane(rch, x + gx) : 0;
                if (r2 > kGroupReach || (c2 > 0 && R > 0 && r2 != R)) break;
                if (g.periodic[0] && 2 * kGroupReach + gx + 1 > nx) break;
                tot += c2;
                R = R > r2 ? R : r2;
                ++gx;
            }
            if (lane == x) {
                my_gx = gx;
                my_nit = tot > 0 ? 1 : 0;
            }
            x += gx;
        }
        if (lane < nx) {
            gxo[base + lane] = my_gx;
            nit[base + lane] = my_nit;
        }
        return;
    }
    if (lane != 0) return;
    int x = 0;
    while (x < nx) {
        const int c0 = staged ? scnt[x] : cell_start[base + x + 1] - cell_start[base + x];
        const bool groupable = staged && px_ok && sok[x] && (c0 == 0 || srch[x] <= kGroupReach);
        if (!groupable) {
            gxo[base + x] = 1;
            nit[base + x] = (c0 + kWave - 1) / kWave;
            ++x;
            continue;
        }
        int R = c0 > 0 ? srch[x] : 0, tot = c0, gx = 1;
        while (x + gx < nx && gx < kGroupLen && sok[x + gx]) {
            const int c2 = scnt[x + gx];
            if (tot + c2 > kGroupMax) break;
            const int r2 = c2 > 0 ? srch[x + gx] : 0;
            if (r2 > kGroupReach || (c2 > 0 && R > 0 && r2 != R)) break;
            if (g.periodic[0] && 2 * kGroupReach + gx + 1 > nx) break;
            tot += c2;
            R = R > r2 ? R : r2;
            ++gx;
        }
        gxo[base + x] = gx;
        nit[base + x] = tot > 0 ? 1 : 0;
        for (int k = 1; k < gx; ++k) {
            gxo[base + x + k] = 0;
            nit[base + x + k] = 0;
        }
        x += gx;
    }
}

// The second pass of the item scan and the item writes in one launch: each thread
// scans its kScanItems cells' item counts (nit) as k_scan_apply does and
// writes those cells' items at the offsets it just found.
__global__ __launch_bounds__(kScanThreads) void k_scan_items(const int32_t* nit, int64_t nc, const int32_t* part,
                                                             const int32_t* cell_start, const int32_t* gxo,
                                                             int64_t max_items, int4* items, int32_t* meta,
                                                             DevState* st)
{
    __shared__ int lds[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int sum = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < nc ? nit[base + k] : 0;
        sum += v[k];
    }
    int total;
    int o = block_scan_excl(sum, lds, total) + part[blockIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int all = part[gridDim.x];
        if (all > max_items) {
            set_flag(st, SPHV_F_QUEUE_OVERFLOW);
            all = (int)max_items;
        }
        meta[META_NITEMS] = all;
    }
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t c = base + k;
        if (c >= nc || v[k] == 0) {
            o += v[k];
            continue;
        }
        const int gx = gxo[c];
        const int b = cell_start[c];
        if (gx > 1) {
            if (o < max_items) items[o] = make_int4((int)c, b, cell_start[c + gx] - b, gx);
            ++o;
            continue;
        }
        const int e = cell_start[c + 1];
        for (int f = b; f < e; f += kWave) {
            if (o < max_items) items[o] = make_int4((int)c, f, min(kWave, e - f), 1);
            ++o;
        }
    }
}

// The cover of the force reach, G(A) = max{ R(B) : d(A,B) <= R(B) } with R
// the cells' own force reach and d the Chebyshev distance in cells: the
// largest own reach among the cells whose reach covers A.  Every force partner
// j of a particle of A lies in such a cell B (r < 2 h_j <= R(B) cmin and
// r >= (d - 1) cmin give d <= R(B)), so G(A) cmin bounds 2 h_j of all of them,
// and G(A) is at least the exact window.  Bit d of a cell's mask says that a
// cell within distance d has R >= d ("thermometer" bits 1..R of each own
// reach); the Chebyshev ball being a cube, the dilation is separable, one pass
// per axis, each OR-ing the masks at offset o into bits >= |o|.  The highest
// bit after the third pass is G.  Above kCoverBits (a global reach of more
// than 63 cells) every cell gets R_global, a looser bound.
constexpr int kCoverBits = 63;

__device__ __forceinline__ uint64_t reach_bits(int R)
{
    return R <= 0 ? 0ull : (R >= kCoverBits ? ~1ull : (1ull << (R + 1)) - 2ull);
}

// PASS 0 dilates the own reaches along x, 1 the masks along y, 2 along z into G
template <int PASS>
__global__ void k_cover_axis(const int32_t* own, const uint64_t* in, uint64_t* out, int32_t* bound, Geom g,
                             const int32_t* meta, int rslot, int64_t nc, DevState* st)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int Rg = meta[rslot];
    if (Rg > kCoverBits) {
        if constexpr (PASS == 2) bound[c] = Rg;
        return;
    }
    int R = Rg;
    const int n = g.n[PASS];
    if (g.periodic[PASS] && 2 * R + 1 > n) {
        if (c == 0) set_flag(st, SPHV_F_GRID_TOO_SMALL);
        R = (n - 1) / 2;
    }
    int k[3];
    cell_coords((int)c, g, k[0], k[1], k[2]);
    uint64_t m = 0;
    for (int d = -R; d <= R; ++d) {
        int kk = k[PASS] + d;
        if (g.periodic[PASS]) {
            kk = kk < 0 ? kk + n : (kk >= n ? kk - n : kk);
        } else if (kk < 0 || kk >= n) {
            continue;
        }
        int q[3] = {k[0], k[1], k[2]};
        q[PASS] = kk;
        const int key = cell_key(q[0], q[1], q[2], g);
        const uint64_t v = PASS == 0 ? reach_bits(own[key]) : in[key];
        const int ad = d < 0 ? -d : d;
        m |= v & (~0ull << ad);
    }
    if constexpr (PASS == 2) bound[c] = m ? 63 - __clzll((long long)m) : 0;
    else out[c] = m;
}

// Own force reach of every cell from its largest converged h: R = ceil(2 h / min
// cell) (0 for an empty cell), widened by 1e-12 so rounding never shrinks it.
// k_force_hbits folds 2 h of every particle into its cell (float bits rounded
// up, as k_bin does); k_force_own turns them into R and a block maximum of R
// into meta[rslot] (one atomic per block of 1024 cells).
template <bool VIEW>
__global__ void k_force_hbits(const int32_t* perm, const int32_t* key_sorted, FieldRef h, uint64_t stride,
                              const uint64_t* ptrs, Access vacc, int64_t n, uint32_t* hbits)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < n;
    int k = 0;
    uint32_t b = 0;
    if (valid) {
        double v;
        if constexpr (VIEW)
            v = ld_f64(h, locate<false>(vacc, p));
        else
            v = *(const double*)((uintptr_t)h.base + h.off +
                                 (ptrs ? ptrs[perm[p]] : (uint64_t)perm[p] * stride));
        b = __float_as_uint(__double2float_ru(2.0 * v));
        k = key_sorted[p];
    }
    // sorted positions: a cell's particles are consecutive lanes, one atomic per run
    b = run_max_upto(b, run_head(k, valid));
    if (valid && run_tail(k, valid)) atomicMax(&hbits[k], b);
}

constexpr int kOwnThreads = 1024;

__global__ __launch_bounds__(kOwnThreads) void k_force_own(const int32_t* cell_start, const uint32_t* hbits,
                                                          double cmin, int32_t* own, int32_t* meta, int rslot,
                                                          int64_t nc)
{
    __shared__ int s[kOwnThreads / kWave];
    const int64_t c = (int64_t)blockIdx.x * kOwnThreads + threadIdx.x;
    int R = 0;
    if (c < nc) {
        if (cell_start[c + 1] > cell_start[c]) {
            R = (int)ceil((double)__uint_as_float(hbits[c]) * (1.0 + 1e-12) / cmin);
            if (R < 1) R = 1;
        }
        own[c] = R;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(R, off, kWave);
        R = o > R ? o : R;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) s[threadIdx.x / kWave] = R;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = s[0];
        for (int k = 1; k < kOwnThreads / kWave; ++k) m = s[k] > m ? s[k] : m;
        if (m > 0) atomicMax(&meta[rslot], m);
    }
}

// Exact force window: cell A must see every cell B whose own reach covers it,
// R_f(A) = max(R(A), max{ d(A,B) : d(A,B) <= R(B) }) with d the Chebyshev
// distance in cells.  The cover G(A) (k_cover_axis) bounds it from above
// and stands in when R_global is large or a periodic axis is short; otherwise
// shells are scanned from the outermost (at most the bound) inward.
constexpr int kExactReach = 4;

__global__ void k_reach_exact(const int32_t* own_r, const int32_t* cover, int32_t* out, Geom g, const int32_t* meta,
                              int rslot, int64_t nc)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int R = meta[rslot];
    bool exact = R <= kExactReach;
    for (int d = 0; d < 3; ++d)
        if (g.periodic[d] && 2 * R + 1 > g.n[d]) exact = false;
    if (!exact) {
        out[c] = cover[c];
        return;
    }
    int k[3];
    cell_coords((int)c, g, k[0], k[1], k[2]);
    const int own = own_r[c];
    int best = own;
    const int top = cover[c] < R ? cover[c] : R;
    for (int d = top; d > own && best == own; --d) {
        for (int dz = -d; dz <= d && best == own; ++dz) {
            int z = k[2] + dz;
            if (z < 0 || z >= g.n[2]) {
                if (!g.periodic[2]) continue;
                z = z < 0 ? z + g.n[2] : z - g.n[2];
            }
            for (int dy = -d; dy <= d && best == own; ++dy) {
                int y = k[1] + dy;
                if (y < 0 || y >= g.n[1]) {
                    if (!g.periodic[1]) continue;
                    y = y < 0 ? y + g.n[1] : y - g.n[1];
                }
                const bool face = dz == -d || dz == d || dy == -d || dy == d;
                const int step = face ? 1 : 2 * d;
                for (int dx = -d; dx <= d; dx += step) {
                    int x = k[0] + dx;
                    if (x < 0 || x >= g.n[0]) {
                        if (!g.periodic[0]) continue;
                        x = x < 0 ? x + g.n[0] : x - g.n[0];
                    }
                    if (own_r[cell_key(x, y, z, g)] >= d) {
                        best = d;
                        break;
                    }
                }
            }
        }
    }
    out[c] = best;
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

}  // namespace

hipError_t launch_fill_u32(void* p, uint32_t v, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    unsigned b = (unsigned)std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(b), dim3(256), 0, s, (uint32_t*)p, v, count);
    return hipGetLastError();
}

hipError_t launch_state_init(DevState* st, int full, hipStream_t s)
{
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, full);
    return hipGetLastError();
}

hipError_t launch_cells_build(const CellsDev& c, const FieldRef* f, const Access& rec, const Geom& g, DevState* st,
                              hipStream_t s)
{
    hipError_t e;
    if ((e = clear3((uint32_t*)c.counts, c.nc, c.hmax_bits, 2 * c.nc, (uint32_t*)c.meta, META_SIZE, s)) != hipSuccess)
        return e;
    if (c.n > 0) {
        StagePlan sp;
        if (!rec.index && !rec.ptrs && plan_stage(f, 4, 0u, rec.stride, &sp))
            hipLaunchKernelGGL(k_bin_staged, dim3(nblk(c.n, kStageThreads)), dim3(kStageThreads),
                               kStageThreads * sp.nch * 16, s, f[0], f[1], f[2], f[3], sp, rec.stride, g, c.n, c.key,
                               c.sub, c.counts, c.hmax_bits, st);
        else
            hipLaunchKernelGGL(k_bin, dim3(nblk(c.n, 256)), dim3(256), 0, s, f[0], f[1], f[2], f[3], rec.stride,
                               rec.ptrs, g, c.n, c.key, c.sub, c.counts, c.hmax_bits, st);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = scan_excl(c.counts, c.nc, c.scan_part, c.cell_start, c.cursor, c.meta + META_SCAN, s)) != hipSuccess)
        return e;
    if (c.n > 0) {
        hipLaunchKernelGGL(k_place, dim3(nblk(c.n, 256)), dim3(256), 0, s, c.key, c.n, c.cursor, c.perm_tmp);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    unsigned sb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(((c.nc + 1) / 2 + kSortWaves - 1) / kSortWaves, 16384));
    hipLaunchKernelGGL(k_segsort, dim3(sb), dim3(kSortThreads), 0, s, c.cell_start, c.perm_tmp, c.sub, c.perm,
                       c.key_sorted, c.hmax_bits, c.reach_d, g, c.nc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t nrows = (int64_t)g.n[1] * g.n[2];
    hipLaunchKernelGGL(k_row_groups, dim3((unsigned)nrows), dim3(kWave), 0, s, c.cell_start, c.counts, c.reach_d, g,
                       c.tmp_a, c.tmp_b);
    {
        // item counts: block totals (the last block scans them), then offsets and items in one pass
        int64_t nb = (c.nc + kScanTile - 1) / kScanTile;
        if (nb == 0) nb = 1;
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, c.tmp_a, c.nc, c.scan_part,
                           c.meta + META_SCAN + 1);
        hipLaunchKernelGGL(k_scan_items, dim3((unsigned)nb), dim3(kScanThreads), 0, s, c.tmp_a, c.nc, c.scan_part,
                           c.cell_start, c.tmp_b, c.max_items, c.items, c.meta, st);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_force_reach(const CellsDev& c, const FieldRef& h, uint64_t stride, const Access* view_acc,
                              const Geom& g, DevState* st, hipStream_t s, const uint64_t* rec_ptrs)
{
    // hmax_f and the largest own reach start at zero with cells_build and only
    // grow: a later force call on larger h widens the windows, never narrows them
    hipError_t e;
    if (c.n > 0) {
        if (view_acc)
            hipLaunchKernelGGL(k_force_hbits<true>, dim3(nblk(c.n, 256)), dim3(256), 0, s, c.perm, c.key_sorted, h,
                               stride, rec_ptrs, *view_acc, c.n, c.hmax_f);
        else
            hipLaunchKernelGGL(k_force_hbits<false>, dim3(nblk(c.n, 256)), dim3(256), 0, s, c.perm, c.key_sorted, h,
                               stride, rec_ptrs, Access{}, c.n, c.hmax_f);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_force_own, dim3(nblk(c.nc, kOwnThreads)), dim3(kOwnThreads), 0, s, c.cell_start, c.hmax_f,
                       g.cmin, c.tmp_a, c.meta, (int)META_RGLOBAL_F, c.nc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the cover G of the own reaches (tmp_a -> cover -> cover + nc -> reach_s), then the exact window
    const unsigned nbc = nblk(c.nc, 256);
    hipLaunchKernelGGL(k_cover_axis<0>, dim3(nbc), dim3(256), 0, s, c.tmp_a, nullptr, c.cover, nullptr, g, c.meta,
                       (int)META_RGLOBAL_F, c.nc, st);
    hipLaunchKernelGGL(k_cover_axis<1>, dim3(nbc), dim3(256), 0, s, nullptr, c.cover, c.cover + c.nc, nullptr, g,
                       c.meta, (int)META_RGLOBAL_F, c.nc, st);
    hipLaunchKernelGGL(k_cover_axis<2>, dim3(nbc), dim3(256), 0, s, nullptr, c.cover + c.nc, nullptr, c.reach_s, g,
                       c.meta, (int)META_RGLOBAL_F, c.nc, st);
    hipLaunchKernelGGL(k_reach_exact, dim3(nblk(c.nc, 256)), dim3(256), 0, s, c.tmp_a, c.reach_s, c.reach_f, g, c.meta,
                       (int)META_RGLOBAL_F, c.nc);
    return hipGetLastError();
}

}  // namespace sphv
