// wsgrid device kernels (gfx950).  See wsgrid.hip for the launch sequence.
#pragma once
#include "common.hpp"
#include "fft.hpp"

namespace wsg {

// ---------------------------------------------------------------- utilities --

template <typename T>
__global__ void k_fill(T* __restrict__ p, size_t n, T v) {
    size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    size_t stride = size_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// ------------------------------------------------------ visibility binning --
//
// Hermitian fold (Sec. 5.4), normalised coordinates u' = (l_max/x0) u,
// v' = (m_max/y0) v, w' = n_scale w (Sec. 5.2), and for each axis the first
// support index F - W + 1 with F = floor(xi + W/2) and the offset
// nu = xi + W/2 - F - 1/2 (Sec. 3.3).  Products and sums are rounded one by one
// (no fused multiply-add) so that the support decision matches a plain
// evaluation of the same formulas.
struct VisCoords {
    int ru, rv, rt;
    double nu_u, nu_v, nu_w;
    double w;          // folded w
    bool folded;
};

__device__ __forceinline__ bool axis_support(double xi, int W, double& nu, long long& first) {
    double hw = 0.5 * W;
    double t = __dadd_rn(xi, hw);
    double F = floor(t);
    nu = __dadd_rn(__dadd_rn(t, -F), -0.5);
    first = (long long)F - W + 1;
    return true;
}

__device__ __forceinline__ bool vis_coords(const double* __restrict__ uvw, long long k,
                                           const DevParams& P, VisCoords& c) {
    double u = uvw[3 * k], v = uvw[3 * k + 1], w = uvw[3 * k + 2];
    if (!isfinite(u) || !isfinite(v) || !isfinite(w)) return false;
    c.folded = w < 0.0;
    if (c.folded) {
        u = -u;
        v = -v;
        w = -w;
    }
    if (w > P.wmax) return false;
    double up = __dmul_rn(P.umul, u), vp = __dmul_rn(P.umul, v), wp = __dmul_rn(P.nscale, w);
    if (fabs(up) > 1e15 || fabs(vp) > 1e15) return false;
    long long fu, fv, ft;
    axis_support(up, P.W, c.nu_u, fu);
    axis_support(vp, P.W, c.nu_v, fv);
    axis_support(wp, P.W, c.nu_w, ft);
    long long Np = P.Np;
    c.ru = int(((fu % Np) + Np) % Np);
    c.rv = int(((fv % Np) + Np) % Np);
    long long it = ft - P.t_lo;
    if (it < 0 || it > P.n_layers - P.W) return false;
    c.rt = int(it);
    c.w = w;
    return true;
}

__device__ __forceinline__ int bin_of(const VisCoords& c, const DevParams& P) {
    return (c.rt / kTileT * P.nbs + c.rv / kTileS) * P.nbr + c.ru / kTileR;
}

__global__ void k_bin_count(const double* __restrict__ uvw, long long M, DevParams P,
                            uint32_t* __restrict__ count, uint32_t* __restrict__ skipped) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    VisCoords c;
    if (!vis_coords(uvw, k, P, c)) {
        atomicAdd(skipped, 1u);
        return;
    }
    atomicAdd(&count[bin_of(c, P)], 1u);
}

// Exclusive scan of n uint32 counts: per-block scan (1024 items per block of
// 256 threads), scan of the block sums in one block, then add.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* sh, uint32_t& total) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) sh[wv] = inc;
    __syncthreads();
    uint32_t woff = 0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < wv; ++i) woff += sh[i];
    total = 0;
    for (int i = 0; i < nw; ++i) total += sh[i];
    __syncthreads();
    return woff + inc - x;
}

__global__ void k_scan_local(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int n,
                             uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t sh[16];
    const int base = blockIdx.x * 1024 + threadIdx.x * 4;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t total;
    uint32_t off = block_exclusive_scan(s, sh, total);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (base + i < n) out[base + i] = off;
        off += v[i];
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// single block of 1024 threads, nb <= 4096
__global__ void k_scan_sums(uint32_t* __restrict__ block_sums, int nb, uint32_t* __restrict__ grand) {
    __shared__ uint32_t sh[16];
    const int base = threadIdx.x * 4;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[i] = (base + i < nb) ? block_sums[base + i] : 0u;
        s += v[i];
    }
    uint32_t total;
    uint32_t off = block_exclusive_scan(s, sh, total);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (base + i < nb) block_sums[base + i] = off;
        off += v[i];
    }
    if (threadIdx.x == 0) *grand = total;
}

__global__ void k_scan_add(uint32_t* __restrict__ out, int n, const uint32_t* __restrict__ block_sums) {
    const int base = blockIdx.x * 1024 + threadIdx.x * 4;
    const uint32_t add = block_sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (base + i < n) out[base + i] += add;
}

// grid: v = V exp(+i 2 pi w (n0 - 1)) with n0 - 1 = -z0 n_scale (eq. n_params),
// V conjugated for a folded visibility.  degrid: v = exp(-i 2 pi w (n0 - 1)).
template <typename R, bool GRID>
__global__ void k_bin_scatter(const double* __restrict__ uvw, const cpx<R>* __restrict__ vis, long long M,
                              DevParams P, const uint32_t* __restrict__ start, uint32_t* __restrict__ cursor,
                              Rec<R>* __restrict__ rec) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    VisCoords c;
    if (!vis_coords(uvw, k, P, c)) return;
    const int b = bin_of(c, P);
    const uint32_t pos = start[b] + atomicAdd(&cursor[b], 1u);
    Rec<R> r;
    r.ruv = uint32_t(c.ru) | (uint32_t(c.rv) << 16);
    r.rt = uint32_t(c.rt);
    r.nu[0] = R(c.nu_u);
    r.nu[1] = R(c.nu_v);
    r.nu[2] = R(c.nu_w);
    double turns = c.w * (-P.z0 * P.nscale);     // w (n0 - 1)
    double s, co;
    phase_turns(GRID ? turns : -turns, &s, &co);
    if (GRID) {
        cpx<R> V = vis[k];
        double vx = double(V.x), vy = c.folded ? -double(V.y) : double(V.y);
        r.v[0] = R(vx * co - vy * s);
        r.v[1] = R(vx * s + vy * co);
        r.idx = 0;
    } else {
        r.v[0] = R(co);
        r.v[1] = R(s);
        r.idx = uint32_t(k) | (c.folded ? 0x80000000u : 0u);
    }
    rec[pos] = r;
}

// Second-level sort: inside each bin, order the records by their first support
// index within the tile (a 12-bit key: layer, u, v offsets), so that records
// with the same support box are adjacent (they form long runs on Earth-rotation
// tracks).  One block per bin: LDS histogram of the 4096 keys, exclusive scan,
// scatter to `out` in key order (order within one key is arbitrary).
template <typename R>
__global__ void __launch_bounds__(256) k_bin_local_sort(const Rec<R>* __restrict__ in, Rec<R>* __restrict__ out,
                                                        const uint32_t* __restrict__ start, DevParams P) {
    __shared__ uint32_t hist[kTileT * kTileR * kTileS];
    __shared__ uint32_t sh[16];
    const int bin = blockIdx.x;
    const uint32_t b0 = start[bin], b1 = start[bin + 1];
    if (b1 - b0 <= 1) {
        if (b1 > b0 && threadIdx.x == 0) out[b0] = in[b0];
        return;
    }
    const int br = bin % P.nbr, bs = (bin / P.nbr) % P.nbs, bt = bin / (P.nbr * P.nbs);
    const int tid = threadIdx.x;
    constexpr int NK = kTileT * kTileR * kTileS;
    for (int i = tid; i < NK; i += 256) hist[i] = 0u;
    __syncthreads();
    auto key_of = [&](const Rec<R>& r) {
        const int ru = int(r.ruv & 0xffffu) - br * kTileR, rv = int(r.ruv >> 16) - bs * kTileS;
        const int rt = int(r.rt) - bt * kTileT;
        return (rt * kTileR + ru) * kTileS + rv;
    };
    for (uint32_t i = b0 + tid; i < b1; i += 256) atomicAdd(&hist[key_of(in[i])], 1u);
    __syncthreads();
    // exclusive scan: 16 consecutive keys per thread
    uint32_t v[NK / 256], sum = 0;
#pragma unroll
    for (int k = 0; k < NK / 256; ++k) {
        v[k] = hist[tid * (NK / 256) + k];
        sum += v[k];
    }
    uint32_t total;
    uint32_t off = block_exclusive_scan(sum, sh, total);
#pragma unroll
    for (int k = 0; k < NK / 256; ++k) {
        hist[tid * (NK / 256) + k] = off;
        off += v[k];
    }
    __syncthreads();
    for (uint32_t i = b0 + tid; i < b1; i += 256) {
        const Rec<R> r = in[i];
        out[b0 + atomicAdd(&hist[key_of(r)], 1u)] = r;
    }
}

// ------------------------------------------------ 3-D scatter / gather tiles --
//
// One 256-thread block owns one tile of kTileT layers x kTileR u-cells x
// kTileS v-cells of the stack (layout [t][r][s], s fastest), held in LDS.  The
// visibilities whose support can reach the tile are those binned (by first
// support index) in this tile or the previous one along each axis (8 bins);
// each bin is sorted by first support index, so records with the same support
// box are adjacent.  Records are staged in rounds of kBatch: each thread loads
// one, tests it against the tile, and the touching ones are compacted in order
// into LDS with their kernel weights.  The staged list is cut into 4
// contiguous chunks, one per wave; a wave walks its chunk with its lanes over
// the W x W (u, v) support pairs and W layer registers per pair:
//   scatter: contributions of a run of equal supports accumulate in registers
//            and go into the LDS tile (atomic adds) once per run;
//   gather:  the run's cells are read from the LDS tile once and contracted
//            with each record's weights; the wave sum (DPP) is the record's
//            part from this tile.
// Each tile is read or written to HBM once.

// Kernel polynomial degree in nu per precision (the host fits both).
template <typename R>
struct KernelDegree {
    static constexpr int value = sizeof(R) == 8 ? 16 : 10;
};

template <typename R, int W>
struct TileCfg {
    static constexpr int kDeg = KernelDegree<R>::value;
    static constexpr int kBatch = 128;
    static constexpr int kPairs = W * W;
    static constexpr int kPI = (kPairs + 63) / 64;     // support pairs per lane
    static constexpr int kCells = kTileT * kTileR * kTileS;
};

template <typename R, int W>
struct TileStage {
    // words: C(s_a - nu_w) for a < W, then the value (2), then the packed
    // offsets (dr + 128) | (ds + 128) << 8 | (dt + 128) << 16
    R words[TileCfg<R, W>::kBatch][W + 3];
    R wuv[TileCfg<R, W>::kBatch][2 * W];     // C(s_a - nu_u), then C(s_a - nu_v)
    uint32_t idx[TileCfg<R, W>::kBatch];
    R out[TileCfg<R, W>::kBatch][2];         // gather: the record's sum over this tile
    int wcount[4];
    int n;
};

__device__ __forceinline__ float bits_to_word(int v, float) { return __int_as_float(v); }
__device__ __forceinline__ double bits_to_word(int v, double) { return __hiloint2double(0, v); }

// value of `v` in lane l, as a wave-uniform (scalar) value
__device__ __forceinline__ float lane_val(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_val(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ int lane_bits(float v, int l) { return __builtin_amdgcn_readlane(__float_as_int(v), l); }
__device__ __forceinline__ int lane_bits(double v, int l) { return __builtin_amdgcn_readlane(__double2loint(v), l); }

// Signed offset of a support start from the tile origin along a periodic axis.
__device__ __forceinline__ int wrap_offset(int first, int origin, int Np) {
    int d = first - origin;
    if (d >= Np / 2) d -= Np;
    if (d < -Np / 2) d += Np;
    return d;
}

// Stage records [base, min(base + kBatch, end)) that touch the tile.  Must be
// called by the whole block; ends with the staged list visible to all threads.
template <typename R, int W>
__device__ __forceinline__ void stage_round(const Rec<R>* __restrict__ rec, uint32_t base, uint32_t end, int r0,
                                            int s0, int t0, int nt_valid, const DevParams& P,
                                            const R* __restrict__ coef, TileStage<R, W>& st) {
    using Cfg = TileCfg<R, W>;
    constexpr int D = Cfg::kDeg;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint32_t i = base + uint32_t(tid);
    bool touch = false;
    Rec<R> r;
    int dr = 0, ds = 0, dt = 0;
    if (tid < Cfg::kBatch && i < end) {
        r = rec[i];
        const int ru = int(r.ruv & 0xffffu), rv = int(r.ruv >> 16), rt = int(r.rt);
        dr = wrap_offset(ru, r0, P.Np);
        ds = wrap_offset(rv, s0, P.Np);
        dt = rt - t0;
        touch = dr + W > 0 && dr < kTileR && ds + W > 0 && ds < kTileS && dt + W > 0 && dt < nt_valid;
    }
    // order-preserving compaction: wave prefix by ballot, block prefix over 4 waves
    const unsigned long long m = __ballot(touch);
    const int wpos = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) st.wcount[wv] = __popcll(m);
    __syncthreads();
    int off = 0;
    for (int w = 0; w < wv; ++w) off += st.wcount[w];
    if (tid == 0) st.n = st.wcount[0] + st.wcount[1] + st.wcount[2] + st.wcount[3];
    if (touch) {
        const int slot = off + wpos;
        // the same least-misfit function on every axis: each coefficient read
        // (an LDS broadcast) feeds the three Horner chains
#pragma unroll
        for (int a = 0; a < W; ++a) {
            const R* c = coef + a * (D + 1);
            R pu = c[D], pv = c[D], pt = c[D];
#pragma unroll
            for (int k = D - 1; k >= 0; --k) {
                const R ck = c[k];
                pu = pu * r.nu[0] + ck;
                pv = pv * r.nu[1] + ck;
                pt = pt * r.nu[2] + ck;
            }
            st.wuv[slot][a] = pu;
            st.wuv[slot][W + a] = pv;
            st.words[slot][a] = pt;
        }
        st.words[slot][W] = r.v[0];
        st.words[slot][W + 1] = r.v[1];
        st.words[slot][W + 2] = bits_to_word((dr + 128) | ((ds + 128) << 8) | ((dt + 128) << 16), R(0));
        st.idx[slot] = r.idx;
    }
    __syncthreads();
}

// The 8 bins whose visibilities can reach tile (bt, bs, br), in storage order.
struct BinWalk {
    int n_t, n_s, n_r;
    __device__ BinWalk(const DevParams& P, int bt) : n_t(bt > 0 ? 2 : 1), n_s(P.nbs > 1 ? 2 : 1), n_r(P.nbr > 1 ? 2 : 1) {}
    __device__ int bin(const DevParams& P, int bt, int bs, int br, int it, int is, int ir) const {
        return ((bt - it) * P.nbs + (bs - is + P.nbs) % P.nbs) * P.nbr + (br - ir + P.nbr) % P.nbr;
    }
};

template <typename R, int W>
__global__ void __launch_bounds__(256) k_grid_tiles(const Rec<R>* __restrict__ rec,
                                                    const uint32_t* __restrict__ start, DevParams P,
                                                    const R* __restrict__ coef_g, cpx<R>* __restrict__ stack) {
    using Cfg = TileCfg<R, W>;
    constexpr int PI = Cfg::kPI;
    __shared__ R tre[Cfg::kCells];
    __shared__ R tim[Cfg::kCells];
    __shared__ TileStage<R, W> st;
    __shared__ R coef[W * (Cfg::kDeg + 1)];

    const int nblocks = P.nbt * P.nbs * P.nbr;
    const int tile = xcd_interleave<4>(blockIdx.x, nblocks);
    const int br = tile % P.nbr, bs = (tile / P.nbr) % P.nbs, bt = tile / (P.nbr * P.nbs);
    const int r0 = br * kTileR, s0 = bs * kTileS, t0 = bt * kTileT;
    const int nt_valid = min(kTileT, P.n_layers - t0);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wl = min(lane, W + 2);
    int par[PI], pas[PI];
#pragma unroll
    for (int i = 0; i < PI; ++i) {
        const int p = min(lane + 64 * i, Cfg::kPairs - 1);
        par[i] = p / W;
        pas[i] = p % W;
    }

    for (int i = tid; i < Cfg::kCells; i += 256) tre[i] = tim[i] = R(0);
    for (int i = tid; i < W * (Cfg::kDeg + 1); i += 256) coef[i] = coef_g[i];
    __syncthreads();

    // add a run's registers into the LDS tile
    auto flush = [&](int d, const R (&ax)[PI][W], const R (&ay)[PI][W]) {
        const int dr = (d & 255) - 128, ds = ((d >> 8) & 255) - 128, dt = ((d >> 16) & 255) - 128;
#pragma unroll
        for (int i = 0; i < PI; ++i) {
            const int rr = dr + par[i], ss = ds + pas[i];
            if (lane + 64 * i < Cfg::kPairs && rr >= 0 && rr < kTileR && ss >= 0 && ss < kTileS) {
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    const int tt = dt + a;
                    if (tt >= 0 && tt < nt_valid) {
                        const int cell = (tt * kTileR + rr) * kTileS + ss;
                        atomicAdd(&tre[cell], ax[i][a]);
                        atomicAdd(&tim[cell], ay[i][a]);
                    }
                }
            }
        }
    };

    const BinWalk walk(P, bt);
    for (int it = 0; it < walk.n_t; ++it)
        for (int is = 0; is < walk.n_s; ++is)
            for (int ir = 0; ir < walk.n_r; ++ir) {
                const int bin = walk.bin(P, bt, bs, br, it, is, ir);
                const uint32_t b0 = start[bin], b1 = start[bin + 1];
                for (uint32_t base = b0; base < b1; base += Cfg::kBatch) {
                    stage_round<R, W>(rec, base, b1, r0, s0, t0, nt_valid, P, coef, st);
                    const int n = st.n;
                    const int j0 = (n * wv) >> 2, j1 = (n * (wv + 1)) >> 2;
                    R ax[PI][W], ay[PI][W];
#pragma unroll
                    for (int i = 0; i < PI; ++i)
#pragma unroll
                        for (int a = 0; a < W; ++a) ax[i][a] = ay[i][a] = R(0);
                    int prev = -1;
                    for (int j = j0; j < j1; ++j) {
                        const R word = st.words[j][wl];                    // one word per lane
                        const int d = lane_bits(word, W + 2);
                        if (d != prev) {                                   // a new support box
                            if (prev != -1) flush(prev, ax, ay);
#pragma unroll
                            for (int i = 0; i < PI; ++i)
#pragma unroll
                                for (int a = 0; a < W; ++a) ax[i][a] = ay[i][a] = R(0);
                            prev = d;
                        }
                        const R vx = lane_val(word, W), vy = lane_val(word, W + 1);
                        R wt[W];
#pragma unroll
                        for (int a = 0; a < W; ++a) wt[a] = lane_val(word, a);
#pragma unroll
                        for (int i = 0; i < PI; ++i) {
                            const R f = st.wuv[j][par[i]] * st.wuv[j][W + pas[i]];
                            const R fx = vx * f, fy = vy * f;
#pragma unroll
                            for (int a = 0; a < W; ++a) {
                                ax[i][a] += fx * wt[a];
                                ay[i][a] += fy * wt[a];
                            }
                        }
                    }
                    if (prev != -1) flush(prev, ax, ay);
                    __syncthreads();
                }
            }
    // write the tile: rows of kTileS cells
    for (int i = tid; i < nt_valid * kTileR * kTileS; i += 256) {
        const int ss = i % kTileS, rr = (i / kTileS) % kTileR, tt = i / (kTileR * kTileS);
        stack[((size_t)(t0 + tt) * P.Np + (r0 + rr)) * P.Np + (s0 + ss)] = cpx<R>{tre[i], tim[i]};
    }
}

template <typename R, int W>
__global__ void __launch_bounds__(256) k_degrid_tiles(const Rec<R>* __restrict__ rec,
                                                      const uint32_t* __restrict__ start, DevParams P,
                                                      const R* __restrict__ coef_g,
                                                      const cpx<R>* __restrict__ stack, R* __restrict__ vis) {
    using Cfg = TileCfg<R, W>;
    constexpr int PI = Cfg::kPI;
    __shared__ R tre[Cfg::kCells];
    __shared__ R tim[Cfg::kCells];
    __shared__ TileStage<R, W> st;
    __shared__ R coef[W * (Cfg::kDeg + 1)];
    __shared__ uint32_t any;

    const int nblocks = P.nbt * P.nbs * P.nbr;
    const int tile = xcd_interleave<4>(blockIdx.x, nblocks);
    const int br = tile % P.nbr, bs = (tile / P.nbr) % P.nbs, bt = tile / (P.nbr * P.nbs);
    const int r0 = br * kTileR, s0 = bs * kTileS, t0 = bt * kTileT;
    const int nt_valid = min(kTileT, P.n_layers - t0);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wl = min(lane, W + 2);
    const BinWalk walk(P, bt);

    // a tile no visibility can reach is not read at all
    if (tid == 0) {
        uint32_t tot = 0;
        for (int it = 0; it < walk.n_t; ++it)
            for (int is = 0; is < walk.n_s; ++is)
                for (int ir = 0; ir < walk.n_r; ++ir) {
                    const int bin = walk.bin(P, bt, bs, br, it, is, ir);
                    tot += start[bin + 1] - start[bin];
                }
        any = tot;
    }
    for (int i = tid; i < W * (Cfg::kDeg + 1); i += 256) coef[i] = coef_g[i];
    __syncthreads();
    if (any == 0) return;
    for (int i = tid; i < nt_valid * kTileR * kTileS; i += 256) {
        const int ss = i % kTileS, rr = (i / kTileS) % kTileR, tt = i / (kTileR * kTileS);
        const cpx<R> q = stack[((size_t)(t0 + tt) * P.Np + (r0 + rr)) * P.Np + (s0 + ss)];
        tre[i] = q.x;
        tim[i] = q.y;
    }
    int par[PI], pas[PI];
#pragma unroll
    for (int i = 0; i < PI; ++i) {
        const int p = min(lane + 64 * i, Cfg::kPairs - 1);
        par[i] = p / W;
        pas[i] = p % W;
    }
    __syncthreads();

    for (int it = 0; it < walk.n_t; ++it)
        for (int is = 0; is < walk.n_s; ++is)
            for (int ir = 0; ir < walk.n_r; ++ir) {
                const int bin = walk.bin(P, bt, bs, br, it, is, ir);
                const uint32_t b0 = start[bin], b1 = start[bin + 1];
                for (uint32_t base = b0; base < b1; base += Cfg::kBatch) {
                    stage_round<R, W>(rec, base, b1, r0, s0, t0, nt_valid, P, coef, st);
                    const int n = st.n;
                    const int j0 = (n * wv) >> 2, j1 = (n * (wv + 1)) >> 2;
                    R qx[PI][W], qy[PI][W];
                    int prev = -1;
                    for (int j = j0; j < j1; ++j) {
                        const R word = st.words[j][wl];                    // one word per lane
                        const int d = lane_bits(word, W + 2);
                        if (d != prev) {                                   // a new support box: read its cells
                            const int dr = (d & 255) - 128, ds = ((d >> 8) & 255) - 128;
                            const int dt = ((d >> 16) & 255) - 128;
#pragma unroll
                            for (int i = 0; i < PI; ++i) {
                                const int rr = dr + par[i], ss = ds + pas[i];
                                const bool ok = lane + 64 * i < Cfg::kPairs && rr >= 0 && rr < kTileR && ss >= 0 &&
                                                ss < kTileS;
#pragma unroll
                                for (int a = 0; a < W; ++a) {
                                    const int tt = dt + a;
                                    const bool in = ok && tt >= 0 && tt < nt_valid;
                                    const int cell = in ? (tt * kTileR + rr) * kTileS + ss : 0;
                                    qx[i][a] = in ? tre[cell] : R(0);
                                    qy[i][a] = in ? tim[cell] : R(0);
                                }
                            }
                            prev = d;
                        }
                        R wt[W];
#pragma unroll
                        for (int a = 0; a < W; ++a) wt[a] = lane_val(word, a);
                        R px = R(0), py = R(0);
#pragma unroll
                        for (int i = 0; i < PI; ++i) {
                            R sx0 = R(0), sy0 = R(0), sx1 = R(0), sy1 = R(0);
#pragma unroll
                            for (int a = 0; a < W; ++a) {
                                if (a & 1) {
                                    sx1 += qx[i][a] * wt[a];
                                    sy1 += qy[i][a] * wt[a];
                                } else {
                                    sx0 += qx[i][a] * wt[a];
                                    sy0 += qy[i][a] * wt[a];
                                }
                            }
                            const R f = st.wuv[j][par[i]] * st.wuv[j][W + pas[i]];
                            px += (sx0 + sx1) * f;
                            py += (sy0 + sy1) * f;
                        }
                        px = wave_sum_lane63(px);
                        py = wave_sum_lane63(py);
                        if (lane == 63) {
                            st.out[j][0] = px;
                            st.out[j][1] = py;
                        }
                    }
                    __syncthreads();
                    // one global update per record and tile: phase exp(-i 2 pi w (n0 - 1)),
                    // conjugate for a folded visibility
                    if (tid < n) {
                        const R sx = st.out[tid][0], sy = st.out[tid][1];
                        const R cx = st.words[tid][W], cy = st.words[tid][W + 1];
                        R ox = sx * cx - sy * cy, oy = sx * cy + sy * cx;
                        const uint32_t idx = st.idx[tid];
                        if (idx & 0x80000000u) oy = -oy;
                        const size_t k = idx & 0x7fffffffu;
                        atomicAdd(&vis[2 * k], ox);
                        atomicAdd(&vis[2 * k + 1], oy);
                    }
                    __syncthreads();
                }
            }
}

// --------------------------------------------------------------- FFT passes --
//
// Stack layout [t][r][s] (s fastest); intermediate layout [t][q][r] (r fastest),
// q the image row.  Image rows j <-> q and columns i <-> p.  The FFT output bin
// f of a line maps to image index (f + N/2) mod N' and is kept when below N
// (Algorithm 5 step 3c); the degrid input places image index p at bin
// (p - N/2) mod N' (zero padding, Algorithm 6 step 3b).

template <typename R, int LOGN>
struct FftCfg {
    static constexpr int N = 1 << LOGN;
    static constexpr int T = N / 16;
    static constexpr int kLineBytes = LinePad<N>::size * int(sizeof(cpx<R>));
    // lines per block for the transposed passes: enough for >= 64-byte runs, within LDS
    static constexpr int kNLt0 = (160 * 1024 - 4096) / kLineBytes;
    static constexpr int kNLt1 = kNLt0 < 1 ? 1 : kNLt0;
    static constexpr int kNLt2 = kNLt1 >= 16 ? 16 : kNLt1 >= 8 ? 8 : kNLt1 >= 4 ? 4 : kNLt1 >= 2 ? 2 : 1;
    static constexpr int kNLt = (kNLt2 * T > 1024) ? 1024 / T : kNLt2;   // a power of two
    // lines per block for the row passes: at least 256 threads
    static constexpr int kNLr = (T >= 256) ? 1 : 256 / T;
};

// grid pass A: IFFT along s of stack rows [t][r][:], keep image rows q, write
// the intermediate transposed [t][q][r].
template <typename R, int LOGN>
__global__ void __launch_bounds__((FftCfg<R, LOGN>::kNLt * FftCfg<R, LOGN>::T))
    k_grid_fft_a(const cpx<R>* __restrict__ stack, cpx<R>* __restrict__ inter, const cpx<R>* __restrict__ tw,
                 int N, int n_layers) {
    using C = FftCfg<R, LOGN>;
    constexpr int Np = C::N, T = C::T, NL = C::kNLt, LP = LinePad<Np>::size;
    __shared__ cpx<R> buf[NL * LP];
    const int blocks_per_plane = Np / NL;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int t = lb / blocks_per_plane, r0 = (lb % blocks_per_plane) * NL;
    const int line = threadIdx.x / T, j = threadIdx.x % T;
    cpx<R>* lbuf = buf + line * LP;
    const cpx<R>* src = stack + ((size_t)t * Np + (r0 + line)) * Np;
    cpx<R> v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = src[j + T * k];
    fft_line<R, LOGN, +1>(v, lbuf, tw, j);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) lbuf[lpad(j + T * k)] = v[k];
    __syncthreads();
    cpx<R>* dst = inter + (size_t)t * N * Np + r0;
    const int half = N / 2;
    for (int idx = threadIdx.x; idx < N * NL; idx += NL * T) {
        const int q = idx / NL, l = idx % NL;
        const int f = (q - half) & (Np - 1);
        dst[(size_t)q * Np + l] = buf[l * LP + lpad(f)];
    }
}

// grid pass B: IFFT along r of intermediate rows [t][q][:] for every layer t,
// w-screen exp(+i 2 pi t z) and accumulation of the real part in registers
// (Algorithm 5 steps 3b-4), then the 3-D correction (step 5): dirty[q][p].
template <typename R, int LOGN>
__global__ void __launch_bounds__((FftCfg<R, LOGN>::kNLr * FftCfg<R, LOGN>::T))
    k_grid_fft_b(const cpx<R>* __restrict__ inter, const cpx<R>* __restrict__ tw, const R* __restrict__ corr,
                 R* __restrict__ dirty, DevParams P) {
    using C = FftCfg<R, LOGN>;
    constexpr int Np = C::N, T = C::T, NL = C::kNLr, LP = LinePad<Np>::size;
    __shared__ cpx<R> buf[NL * LP];
    const int N = P.N, half = N / 2;
    const int line = threadIdx.x / T, j = threadIdx.x % T;
    const int q = xcd_remap(blockIdx.x, gridDim.x) * NL + line;
    const bool row_ok = q < N;
    const int qq = row_ok ? q : 0;
    cpx<R>* lbuf = buf + line * LP;
    double z[16];
    R acc[16];
    int pix[16];
    const double m = double(qq - half) * P.dl;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int f = j + T * k;
        const int p = (f + half) & (Np - 1);
        pix[k] = (row_ok && p < N) ? p : -1;
        const double l = double(min(p, N - 1) - half) * P.dl;   // bins outside the image are not used
        const double r2 = l * l + m * m;
        const double nm1 = -r2 / (1.0 + sqrt(1.0 - r2));     // n - 1
        z[k] = nm1 / P.nscale + P.z0;                         // (n - n0) / n_scale
        acc[k] = R(0);
    }
    for (int t = 0; t < P.n_layers; ++t) {
        const cpx<R>* src = inter + ((size_t)t * N + qq) * Np;
        cpx<R> v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = src[j + T * k];
        fft_line<R, LOGN, +1>(v, lbuf, tw, j);
        const double tl = double(t + P.t_lo);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (pix[k] >= 0) {
                R s, c;
                phase_turns(tl * z[k], &s, &c);
                acc[k] += v[k].x * c - v[k].y * s;
            }
        }
    }
    if (!row_ok) return;
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (pix[k] >= 0) dirty[(size_t)q * N + pix[k]] = acc[k] * corr[(size_t)q * N + pix[k]];
}

// degrid pass B': for each image row q and layer t: f h_x h_y h_z exp(-i 2 pi t z)
// zero-padded along p, FFT along p -> intermediate [t][q][r] (Algorithm 6 steps 2-3).
template <typename R, int LOGN>
__global__ void __launch_bounds__((FftCfg<R, LOGN>::kNLr * FftCfg<R, LOGN>::T))
    k_degrid_fft_b(const R* __restrict__ image, const R* __restrict__ corr, const cpx<R>* __restrict__ tw,
                   cpx<R>* __restrict__ inter, DevParams P) {
    using C = FftCfg<R, LOGN>;
    constexpr int Np = C::N, T = C::T, NL = C::kNLr, LP = LinePad<Np>::size;
    __shared__ cpx<R> buf[NL * LP];
    const int N = P.N, half = N / 2;
    const int line = threadIdx.x / T, j = threadIdx.x % T;
    const int q = xcd_remap(blockIdx.x, gridDim.x) * NL + line;
    const bool row_ok = q < N;
    const int qq = row_ok ? q : 0;
    cpx<R>* lbuf = buf + line * LP;
    double z[16];
    R g[16];
    const double m = double(qq - half) * P.dl;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int f = j + T * k;
        const int p = (f + half) & (Np - 1);
        const bool ok = row_ok && p < N;
        g[k] = ok ? image[(size_t)qq * N + p] * corr[(size_t)qq * N + p] : R(0);
        const double l = double(min(p, N - 1) - half) * P.dl;   // keeps z finite on padding bins
        const double r2 = l * l + m * m;
        const double nm1 = -r2 / (1.0 + sqrt(1.0 - r2));
        z[k] = nm1 / P.nscale + P.z0;
    }
    for (int t = 0; t < P.n_layers; ++t) {
        const double tl = double(t + P.t_lo);
        cpx<R> v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            R s, c;
            phase_turns(-tl * z[k], &s, &c);
            v[k] = cpx<R>{g[k] * c, g[k] * s};
        }
        fft_line<R, LOGN, -1>(v, lbuf, tw, j);
        if (row_ok) {
            cpx<R>* dst = inter + ((size_t)t * N + q) * Np;
#pragma unroll
            for (int k = 0; k < 16; ++k) dst[j + T * k] = v[k];
        }
    }
}

// degrid pass A': for each layer t and block of columns r: read intermediate
// column [t][:][r] (transposed), zero-pad along q, FFT along q -> stack row [t][r][s].
template <typename R, int LOGN>
__global__ void __launch_bounds__((FftCfg<R, LOGN>::kNLt * FftCfg<R, LOGN>::T))
    k_degrid_fft_a(const cpx<R>* __restrict__ inter, const cpx<R>* __restrict__ tw, cpx<R>* __restrict__ stack,
                   int N, int n_layers) {
    using C = FftCfg<R, LOGN>;
    constexpr int Np = C::N, T = C::T, NL = C::kNLt, LP = LinePad<Np>::size;
    __shared__ cpx<R> buf[NL * LP];
    const int blocks_per_plane = Np / NL;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int t = lb / blocks_per_plane, r0 = (lb % blocks_per_plane) * NL;
    const int line = threadIdx.x / T, j = threadIdx.x % T;
    cpx<R>* lbuf = buf + line * LP;
    const int half = N / 2;
    // zero the padding bins, then the transposed load of the N image rows
    for (int idx = threadIdx.x; idx < (Np - N) * NL; idx += NL * T) {
        const int l = idx % NL, e = idx / NL;                 // e-th bin outside the image
        const int f = (N - half + e) & (Np - 1);              // bins N/2 .. Np - N/2 - 1
        buf[l * LP + lpad(f)] = cpx<R>{R(0), R(0)};
    }
    const cpx<R>* src = inter + (size_t)t * N * Np + r0;
    for (int idx = threadIdx.x; idx < N * NL; idx += NL * T) {
        const int q = idx / NL, l = idx % NL;
        const int f = (q - half) & (Np - 1);
        buf[l * LP + lpad(f)] = src[(size_t)q * Np + l];
    }
    __syncthreads();
    cpx<R> v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = lbuf[lpad(j + T * k)];
    fft_line<R, LOGN, -1>(v, lbuf, tw, j);
    cpx<R>* dst = stack + ((size_t)t * Np + (r0 + line)) * Np;
#pragma unroll
    for (int k = 0; k < 16; ++k) dst[j + T * k] = v[k];
}

// --------------------------------------------------------------- plan tables --
//
// Correction map corr[j][i] = h(x_i) h(y_j) h(z_ji) (Algorithm 5 step 5): h at the
// pixel columns comes from the host, h(z) is evaluated here from the pointwise
// optimality formula h(z) = int Re g dnu / int |g|^2 dnu over Gauss-Legendre
// nodes nu_j, g(z, nu) = sum_a c_a(nu) exp(i 2 pi (s_a - nu) z).
__global__ void k_corr_map(const double* __restrict__ hx, const double* __restrict__ cnodes,
                           const double* __restrict__ nun, const double* __restrict__ wn, int n_nu, DevParams P,
                           double* __restrict__ corr64, float* __restrict__ corr32) {
    const int N = P.N, half = N / 2;
    const int i = blockIdx.x * blockDim.x + threadIdx.x, jrow = blockIdx.y;
    if (i >= N) return;
    const double l = double(i - half) * P.dl, m = double(jrow - half) * P.dl;
    const double r2 = l * l + m * m;
    const double z = (-r2 / (1.0 + sqrt(1.0 - r2))) / P.nscale + P.z0;
    const int W = P.W;
    double step_s, step_c;
    sincospi(2.0 * z, &step_s, &step_c);                         // exp(i 2 pi z)
    double num = 0.0, den = 0.0;
    for (int jn = 0; jn < n_nu; ++jn) {
        double es, ec;
        sincospi(2.0 * (-0.5 * (W - 1) - nun[jn]) * z, &es, &ec);  // a = 0 term
        double gr = 0.0, gi = 0.0;
        for (int a = 0; a < W; ++a) {
            const double c = cnodes[jn * W + a];
            gr += c * ec;
            gi += c * es;
            const double nc = ec * step_c - es * step_s, ns = ec * step_s + es * step_c;
            ec = nc;
            es = ns;
        }
        num += wn[jn] * gr;
        den += wn[jn] * (gr * gr + gi * gi);
    }
    const double v = hx[i] * hx[jrow] * (num / den);
    corr64[(size_t)jrow * N + i] = v;
    corr32[(size_t)jrow * N + i] = float(v);
}

}  // namespace wsg
