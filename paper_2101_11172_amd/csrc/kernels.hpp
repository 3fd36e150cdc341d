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

// ------------------------------------------------ 3-D scatter / gather tiles --
//
// One block owns one tile of kTileT layers x kTileR u-cells x kTileS v-cells of
// the stack (layout [t][r][s], s fastest) and takes every contribution that
// lands in it (owner computes: no global atomics, every tile written once).
// The visibilities whose support can reach the tile are those binned (by first
// support index) in this tile or in the previous tile along each axis.
// Each wave takes a batch of up to 64 records: lane i evaluates record i's
// 3W kernel weights (Horner in nu, per-segment polynomial) into the wave's LDS
// scratch, then the wave walks the records that touch the tile, with its lanes
// over the (a_r, a_s) support pairs and a loop over the layers a_t.

template <typename R, int W>
struct TileCfg {
    static constexpr int kWaves = 4;
    static constexpr int kBatch = (sizeof(R) == 8 && W > 8) ? 32 : 64;
    static constexpr int kPairs = W * W;
    static constexpr int kPairIters = (kPairs + 63) / 64;
    static constexpr int kCells = kTileT * kTileR * kTileS;
};

// Signed offset of a support start from the tile origin along a periodic axis.
__device__ __forceinline__ int wrap_offset(int first, int origin, int Np) {
    int d = first - origin;
    if (d >= Np / 2) d -= Np;
    if (d < -Np / 2) d += Np;
    return d;
}

template <typename R, int W>
struct WaveScratch {
    R w[TileCfg<R, W>::kBatch][3 * W];
    R val[TileCfg<R, W>::kBatch][2];
    int box[TileCfg<R, W>::kBatch][4];     // d_r, d_s, d_t packed bounds, idx
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R>
__device__ __forceinline__ R horner(const R* __restrict__ c, int degree, R nu) {
    R v = c[degree];
    for (int k = degree - 1; k >= 0; --k) v = v * nu + c[k];
    return v;
}

// Load the records of bin range [b0, b1) that touch the tile; returns the
// ballot of lanes holding a touching record.  Bounds per axis are packed as
// lo | hi << 8 | (d + 128) << 16 in weight-index space.
template <typename R, int W>
__device__ __forceinline__ unsigned long long stage_batch(const Rec<R>* __restrict__ rec, uint32_t i,
                                                          uint32_t end, int r0, int s0, int t0, int nt_valid,
                                                          const DevParams& P, const R* __restrict__ coef,
                                                          WaveScratch<R, W>& ws, int lane, bool gather) {
    bool touch = false;
    if (i < end) {
        Rec<R> r = rec[i];
        const int ru = int(r.ruv & 0xffffu), rv = int(r.ruv >> 16), rt = int(r.rt);
        const int dr = wrap_offset(ru, r0, P.Np), ds = wrap_offset(rv, s0, P.Np), dt = rt - t0;
        const int lor = max(0, -dr), hir = min(W - 1, kTileR - 1 - dr);
        const int los = max(0, -ds), his = min(W - 1, kTileS - 1 - ds);
        const int lot = max(0, -dt), hit = min(W - 1, nt_valid - 1 - dt);
        touch = lor <= hir && los <= his && lot <= hit;
        if (touch) {
            const int D = P.degree;
#pragma unroll
            for (int a = 0; a < W; ++a) {
                ws.w[lane][a] = horner(coef + a * (D + 1), D, r.nu[0]);
                ws.w[lane][W + a] = horner(coef + a * (D + 1), D, r.nu[1]);
                ws.w[lane][2 * W + a] = horner(coef + a * (D + 1), D, r.nu[2]);
            }
            ws.val[lane][0] = r.v[0];
            ws.val[lane][1] = r.v[1];
            ws.box[lane][0] = lor | (hir << 8) | ((dr + 128) << 16);
            ws.box[lane][1] = los | (his << 8) | ((ds + 128) << 16);
            ws.box[lane][2] = lot | (hit << 8) | ((dt + 128) << 16);
            ws.box[lane][3] = int(r.idx);
        }
    }
    (void)gather;
    return __ballot(touch);
}

template <typename R, int W>
__global__ void __launch_bounds__(256) k_grid_tiles(const Rec<R>* __restrict__ rec,
                                                    const uint32_t* __restrict__ start, DevParams P,
                                                    const R* __restrict__ coef_g, cpx<R>* __restrict__ stack) {
    using Cfg = TileCfg<R, W>;
    __shared__ R tre[Cfg::kCells];
    __shared__ R tim[Cfg::kCells];
    __shared__ WaveScratch<R, W> scratch[Cfg::kWaves];
    __shared__ R coef[W * 24];

    const int nblocks = P.nbt * P.nbs * P.nbr;
    const int tile = xcd_remap(blockIdx.x, nblocks);
    const int br = tile % P.nbr, bs = (tile / P.nbr) % P.nbs, bt = tile / (P.nbr * P.nbs);
    const int r0 = br * kTileR, s0 = bs * kTileS, t0 = bt * kTileT;
    const int nt_valid = min(kTileT, P.n_layers - t0);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    for (int i = tid; i < Cfg::kCells; i += 256) {
        tre[i] = R(0);
        tim[i] = R(0);
    }
    for (int i = tid; i < W * (P.degree + 1); i += 256) coef[i] = coef_g[i];
    __syncthreads();

    WaveScratch<R, W>& ws = scratch[wv];
    const int nbr_prev = (P.nbr > 1) ? 2 : 1, nbs_prev = (P.nbs > 1) ? 2 : 1, nbt_prev = (bt > 0) ? 2 : 1;
    for (int it = 0; it < nbt_prev; ++it)
        for (int is = 0; is < nbs_prev; ++is)
            for (int ir = 0; ir < nbr_prev; ++ir) {
                const int cbt = bt - it;
                const int cbs = (bs - is + P.nbs) % P.nbs;
                const int cbr = (br - ir + P.nbr) % P.nbr;
                const int bin = (cbt * P.nbs + cbs) * P.nbr + cbr;
                const uint32_t b0 = start[bin], b1 = start[bin + 1];
                for (uint32_t base = b0 + uint32_t(wv) * Cfg::kBatch; base < b1;
                     base += uint32_t(Cfg::kWaves) * Cfg::kBatch) {
                    // every lane takes part in the ballot; lanes past the batch hold no record
                    const uint32_t ri = lane < Cfg::kBatch ? base + uint32_t(lane) : b1;
                    unsigned long long mask =
                        stage_batch<R, W>(rec, ri, b1, r0, s0, t0, nt_valid, P, coef, ws, lane, false);
                    wave_sync();
                    while (mask) {
                        const int q = __ffsll(mask) - 1;
                        mask &= mask - 1;
                        const int br_ = ws.box[q][0], bs_ = ws.box[q][1], bt_ = ws.box[q][2];
                        const int lor = br_ & 255, hir = (br_ >> 8) & 255, dr = (br_ >> 16) - 128;
                        const int los = bs_ & 255, his = (bs_ >> 8) & 255, ds = (bs_ >> 16) - 128;
                        const int lot = bt_ & 255, hit = (bt_ >> 8) & 255, dt = (bt_ >> 16) - 128;
                        const R vx = ws.val[q][0], vy = ws.val[q][1];
#pragma unroll
                        for (int pi = 0; pi < Cfg::kPairIters; ++pi) {
                            const int pr = lane + 64 * pi;
                            const int ar = pr / W, as = pr - (pr / W) * W;
                            if (pr < Cfg::kPairs && ar >= lor && ar <= hir && as >= los && as <= his) {
                                const R wrs = ws.w[q][ar] * ws.w[q][W + as];
                                const R px = vx * wrs, py = vy * wrs;
                                const int cell_rs = (dr + ar) * kTileS + (ds + as);
                                for (int at = lot; at <= hit; ++at) {
                                    const R wt = ws.w[q][2 * W + at];
                                    const int cell = (dt + at) * (kTileR * kTileS) + cell_rs;
                                    atomicAdd(&tre[cell], px * wt);
                                    atomicAdd(&tim[cell], py * wt);
                                }
                            }
                        }
                    }
                    wave_sync();
                }
            }
    __syncthreads();
    // write the tile: rows of kTileS cells
    for (int i = tid; i < nt_valid * kTileR * kTileS; i += 256) {
        const int ss = i % kTileS, rr = (i / kTileS) % kTileR, tt = i / (kTileR * kTileS);
        const size_t g = ((size_t)(t0 + tt) * P.Np + (r0 + rr)) * P.Np + (s0 + ss);
        stack[g] = cpx<R>{tre[i], tim[i]};
    }
}

template <typename R, int W>
__global__ void __launch_bounds__(256) k_degrid_tiles(const Rec<R>* __restrict__ rec,
                                                      const uint32_t* __restrict__ start, DevParams P,
                                                      const R* __restrict__ coef_g,
                                                      const cpx<R>* __restrict__ stack, R* __restrict__ vis) {
    using Cfg = TileCfg<R, W>;
    __shared__ R tre[Cfg::kCells];
    __shared__ R tim[Cfg::kCells];
    __shared__ WaveScratch<R, W> scratch[Cfg::kWaves];
    __shared__ R coef[W * 24];

    const int nblocks = P.nbt * P.nbs * P.nbr;
    const int tile = xcd_remap(blockIdx.x, nblocks);
    const int br = tile % P.nbr, bs = (tile / P.nbr) % P.nbs, bt = tile / (P.nbr * P.nbs);
    const int r0 = br * kTileR, s0 = bs * kTileS, t0 = bt * kTileT;
    const int nt_valid = min(kTileT, P.n_layers - t0);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    for (int i = tid; i < nt_valid * kTileR * kTileS; i += 256) {
        const int ss = i % kTileS, rr = (i / kTileS) % kTileR, tt = i / (kTileR * kTileS);
        const cpx<R> q = stack[((size_t)(t0 + tt) * P.Np + (r0 + rr)) * P.Np + (s0 + ss)];
        tre[i] = q.x;
        tim[i] = q.y;
    }
    for (int i = tid; i < W * (P.degree + 1); i += 256) coef[i] = coef_g[i];
    __syncthreads();

    WaveScratch<R, W>& ws = scratch[wv];
    const int nbr_prev = (P.nbr > 1) ? 2 : 1, nbs_prev = (P.nbs > 1) ? 2 : 1, nbt_prev = (bt > 0) ? 2 : 1;
    for (int it = 0; it < nbt_prev; ++it)
        for (int is = 0; is < nbs_prev; ++is)
            for (int ir = 0; ir < nbr_prev; ++ir) {
                const int cbt = bt - it;
                const int cbs = (bs - is + P.nbs) % P.nbs;
                const int cbr = (br - ir + P.nbr) % P.nbr;
                const int bin = (cbt * P.nbs + cbs) * P.nbr + cbr;
                const uint32_t b0 = start[bin], b1 = start[bin + 1];
                for (uint32_t base = b0 + uint32_t(wv) * Cfg::kBatch; base < b1;
                     base += uint32_t(Cfg::kWaves) * Cfg::kBatch) {
                    // every lane takes part in the ballot; lanes past the batch hold no record
                    const uint32_t ri = lane < Cfg::kBatch ? base + uint32_t(lane) : b1;
                    unsigned long long mask =
                        stage_batch<R, W>(rec, ri, b1, r0, s0, t0, nt_valid, P, coef, ws, lane, true);
                    wave_sync();
                    while (mask) {
                        const int q = __ffsll(mask) - 1;
                        mask &= mask - 1;
                        const int br_ = ws.box[q][0], bs_ = ws.box[q][1], bt_ = ws.box[q][2];
                        const int lor = br_ & 255, hir = (br_ >> 8) & 255, dr = (br_ >> 16) - 128;
                        const int los = bs_ & 255, his = (bs_ >> 8) & 255, ds = (bs_ >> 16) - 128;
                        const int lot = bt_ & 255, hit = (bt_ >> 8) & 255, dt = (bt_ >> 16) - 128;
                        R ax = R(0), ay = R(0);
#pragma unroll
                        for (int pi = 0; pi < Cfg::kPairIters; ++pi) {
                            const int pr = lane + 64 * pi;
                            const int ar = pr / W, as = pr - (pr / W) * W;
                            if (pr < Cfg::kPairs && ar >= lor && ar <= hir && as >= los && as <= his) {
                                const int cell_rs = (dr + ar) * kTileS + (ds + as);
                                R sx = R(0), sy = R(0);
                                for (int at = lot; at <= hit; ++at) {
                                    const R wt = ws.w[q][2 * W + at];
                                    const int cell = (dt + at) * (kTileR * kTileS) + cell_rs;
                                    sx += tre[cell] * wt;
                                    sy += tim[cell] * wt;
                                }
                                const R wrs = ws.w[q][ar] * ws.w[q][W + as];
                                ax += sx * wrs;
                                ay += sy * wrs;
                            }
                        }
#pragma unroll
                        for (int o = 32; o > 0; o >>= 1) {
                            ax += __shfl_xor(ax, o, 64);
                            ay += __shfl_xor(ay, o, 64);
                        }
                        if (lane == 0) {
                            const R px = ws.val[q][0], py = ws.val[q][1];
                            R ox = ax * px - ay * py, oy = ax * py + ay * px;
                            const uint32_t idx = uint32_t(ws.box[q][3]);
                            if (idx & 0x80000000u) oy = -oy;
                            const size_t k = idx & 0x7fffffffu;
                            atomicAdd(&vis[2 * k], ox);
                            atomicAdd(&vis[2 * k + 1], oy);
                        }
                    }
                    wave_sync();
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
