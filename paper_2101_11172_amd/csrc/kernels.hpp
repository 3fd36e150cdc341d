// wsgrid device kernels (gfx950).  See wsgrid.hip for the launch sequence.
// The header is included by several compilation units: kernels that are not
// templates are static (one copy per unit that launches them).
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

// Streaming copy for the bandwidth probe: each block walks kProbeUnroll
// consecutive 16-byte vectors per thread per round (all loads issued before
// the stores, non-temporal both ways), rounds strided by the whole grid.  Of
// the shapes measured (128-1024 threads, 4-16 vectors, 512-16384 blocks,
// temporal or not) this one streamed fastest.
constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 8;
typedef unsigned int probe_vec __attribute__((ext_vector_type(4)));
static __global__ void __launch_bounds__(kProbeThreads) k_copy_probe(const probe_vec* __restrict__ src,
                                                                   probe_vec* __restrict__ dst, size_t n) {
    const size_t step = size_t(gridDim.x) * kProbeThreads * kProbeUnroll;
    for (size_t base = size_t(blockIdx.x) * kProbeThreads * kProbeUnroll + threadIdx.x; base < n; base += step) {
        probe_vec v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const size_t i = base + size_t(u) * kProbeThreads;
            if (i < n) v[u] = __builtin_nontemporal_load(src + i);
        }
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const size_t i = base + size_t(u) * kProbeThreads;
            if (i < n) __builtin_nontemporal_store(v[u], dst + i);
        }
    }
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

// The non-negative residue of the integer-valued f (|f| < 2^53) modulo n, in
// FP64: the quotient's floor may be one off after rounding, which the two
// corrections undo; q n and f - q n are exact.
__device__ __forceinline__ int residue(double f, int n) {
    const double dn = double(n);
    const double q = floor(__ddiv_rn(f, dn));
    double r = __dadd_rn(f, -__dmul_rn(q, dn));
    if (r < 0.0) r += dn;
    if (r >= dn) r -= dn;
    return int(r);
}

// ch: the visibility's channel (virtual layer offset ch nbt kTileT)
__device__ __forceinline__ bool vis_coords_of(double u, double v, double w, int ch, const DevParams& P,
                                              VisCoords& c) {
    if (!isfinite(u) || !isfinite(v) || !isfinite(w)) return false;
    c.folded = w < 0.0;
    if (c.folded) {
        u = -u;
        v = -v;
        w = -w;
    }
    if (w > P.wmax) return false;
    double up = __dmul_rn(P.umul, u), vp = __dmul_rn(P.umul, v), wp = __dadd_rn(__dmul_rn(P.nscale, w), P.wshift);
    if (fabs(up) > 1e15 || fabs(vp) > 1e15) return false;
    long long fu, fv, ft;
    axis_support(up, P.W, c.nu_u, fu);
    axis_support(vp, P.W, c.nu_v, fv);
    axis_support(wp, P.Wz, c.nu_w, ft);
    // the non-negative residues modulo N' (|first| < 2^51 after the check above)
    c.ru = residue(double(fu), P.Np);
    c.rv = residue(double(fv), P.Np);
    long long it = ft - P.t_lo;
    if (P.tclamp && it == P.n_layers) it = P.n_layers - 1;      // w = wmax: the last bin is closed
    if (it < 0 || it > P.n_layers - P.Wz) return false;
    c.rt = int(it) + ch * P.nbt * kTileT;
    c.w = w;
    return true;
}

__device__ __forceinline__ bool vis_coords(const double* __restrict__ uvw, long long k, int ch,
                                           const DevParams& P, VisCoords& c) {
    return vis_coords_of(uvw[3 * k], uvw[3 * k + 1], uvw[3 * k + 2], ch, P, c);
}

__device__ __forceinline__ int bin_of(const VisCoords& c, const DevParams& P) {
    return (c.rt / kTileT * P.nbs + c.rv / kTileS) * P.nbr + c.ru / kTileR;
}

// Bin counts and cursors are updated with device-scope atomics, whose cost is
// per operation.  A block therefore takes a chunk of kAggChunk consecutive
// visibilities (a run of time steps of every baseline, whose tracks stay in few
// bins) and aggregates them per bin in an LDS table (open addressing, bounded
// probing) before one global update per distinct bin; a visibility whose bin
// finds no table slot updates the global counter directly.
constexpr int kAggThreads = 1024;
constexpr int kAggPer = 8;
constexpr int kAggChunk = kAggThreads * kAggPer;
constexpr int kAggSlots = 4096;
constexpr int kAggProbes = 32;

struct AggTable {
    int key[kAggSlots];
    uint32_t cnt[kAggSlots];
    uint32_t base[kAggSlots];
    uint32_t skipped;
};

// Binning blocks of a batched call: block b belongs to channel c when
// cblk[c] <= b < cblk[c + 1]; channel c's visibilities are [coff[c], coff[c + 1])
// of the concatenated arrays, kAggChunk of them per block (one channel per
// block, so the lookup is wave-uniform).
struct ChunkRange {
    long long k0, k1;
    int ch;
};
__device__ __forceinline__ ChunkRange chunk_of_block(const long long* __restrict__ coff,
                                                     const int* __restrict__ cblk, int nch) {
    const int b = blockIdx.x;
    int c = 0;
    while (c + 1 < nch && cblk[c + 1] <= b) ++c;
    ChunkRange r;
    r.ch = c;
    r.k0 = coff[c] + (long long)(b - cblk[c]) * kAggChunk;
    r.k1 = min(coff[c + 1], r.k0 + kAggChunk);
    return r;
}

__device__ __forceinline__ void agg_init(AggTable& T) {
    for (int i = threadIdx.x; i < kAggSlots; i += blockDim.x) {
        T.key[i] = -1;
        T.cnt[i] = 0u;
    }
    if (threadIdx.x == 0) T.skipped = 0u;
}

// slot of key (inserted if absent), or -1 when the probe sequence is full
__device__ __forceinline__ int agg_slot(AggTable& T, int key) {
    int h = int((uint32_t(key) * 2654435761u) >> (32 - 12)) & (kAggSlots - 1);
    for (int p = 0; p < kAggProbes; ++p) {
        const int k = T.key[h];
        if (k == key) return h;
        if (k == -1) {
            const int old = atomicCAS(&T.key[h], -1, key);
            if (old == -1 || old == key) return h;
        }
        h = (h + 1) & (kAggSlots - 1);
    }
    return -1;
}

static __global__ void __launch_bounds__(kAggThreads) k_bin_count(const double* __restrict__ uvw,
                                                           const long long* __restrict__ coff,
                                                           const int* __restrict__ cblk, DevParams P,
                                                           uint32_t* __restrict__ count,
                                                           uint32_t* __restrict__ skipped) {
    __shared__ AggTable T;
    agg_init(T);
    __syncthreads();
    const ChunkRange cr = chunk_of_block(coff, cblk, P.nch);
    uint32_t my_skipped = 0;
    // the thread's coordinates, all loads in flight at once
    double xu[kAggPer], xv[kAggPer], xw[kAggPer];
#pragma unroll
    for (int i = 0; i < kAggPer; ++i) {
        const long long k = cr.k0 + (long long)i * kAggThreads + threadIdx.x;
        const bool in = k < cr.k1;
        xu[i] = in ? uvw[3 * k] : 0.0;
        xv[i] = in ? uvw[3 * k + 1] : 0.0;
        xw[i] = in ? uvw[3 * k + 2] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kAggPer; ++i) {
        const long long k = cr.k0 + (long long)i * kAggThreads + threadIdx.x;
        if (k >= cr.k1) break;
        VisCoords c;
        if (!vis_coords_of(xu[i], xv[i], xw[i], cr.ch, P, c)) {
            ++my_skipped;
            continue;
        }
        const int b = bin_of(c, P);
        const int sl = agg_slot(T, b);
        if (sl >= 0)
            atomicAdd(&T.cnt[sl], 1u);
        else
            atomicAdd(&count[b], 1u);
    }
    if (my_skipped) atomicAdd(&T.skipped, my_skipped);
    __syncthreads();
    for (int i = threadIdx.x; i < kAggSlots; i += kAggThreads)
        if (T.key[i] >= 0) atomicAdd(&count[T.key[i]], T.cnt[i]);
    if (threadIdx.x == 0 && T.skipped) atomicAdd(skipped, T.skipped);
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

static __global__ void k_scan_local(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int n,
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

// single block of 1024 threads; each thread scans ceil(nb / 1024) consecutive sums
static __global__ void k_scan_sums(uint32_t* __restrict__ block_sums, int nb, uint32_t* __restrict__ grand) {
    __shared__ uint32_t sh[16];
    const int per = (nb + 1023) / 1024;
    const int base = threadIdx.x * per;
    uint32_t s = 0;
    for (int i = 0; i < per; ++i)
        if (base + i < nb) s += block_sums[base + i];
    uint32_t total;
    uint32_t off = block_exclusive_scan(s, sh, total);
    for (int i = 0; i < per; ++i) {
        if (base + i < nb) {
            const uint32_t v = block_sums[base + i];
            block_sums[base + i] = off;
            off += v;
        }
    }
    if (threadIdx.x == 0) *grand = total;
}

static __global__ void k_scan_add(uint32_t* __restrict__ out, int n, const uint32_t* __restrict__ block_sums) {
    const int base = blockIdx.x * 1024 + threadIdx.x * 4;
    const uint32_t add = block_sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (base + i < n) out[base + i] += add;
}

// grid: v = V exp(+i 2 pi w (n0 - 1)) with n0 - 1 = -zshift n_scale (eq. n_params:
// zshift = z0; zero without z offset, eq. n_params_no_offset),
// V conjugated for a folded visibility.  degrid: v = exp(-i 2 pi w (n0 - 1)).
template <typename R, bool GRID>
__global__ void __launch_bounds__(kAggThreads) k_bin_scatter(const double* __restrict__ uvw,
                                                             const cpx<R>* __restrict__ vis,
                                                             const long long* __restrict__ coff,
                                                             const int* __restrict__ cblk, DevParams P,
                                                             const uint32_t* __restrict__ start,
                                                             uint32_t* __restrict__ cursor, Rec<R>* __restrict__ rec) {
    __shared__ AggTable T;
    agg_init(T);
    __syncthreads();
    const ChunkRange cr = chunk_of_block(coff, cblk, P.nch);
    const long long k0 = cr.k0;
    // the thread's coordinates, loaded once for both passes, all in flight at once
    double xu[kAggPer], xv[kAggPer], xw[kAggPer];
#pragma unroll
    for (int i = 0; i < kAggPer; ++i) {
        const long long k = k0 + (long long)i * kAggThreads + threadIdx.x;
        const bool in = k < cr.k1;
        xu[i] = in ? uvw[3 * k] : 0.0;
        xv[i] = in ? uvw[3 * k + 1] : 0.0;
        xw[i] = in ? uvw[3 * k + 2] : 0.0;
    }
    // pass 1: rank of each visibility among this block's visibilities of its bin
    uint32_t tag[kAggPer];             // slot << 16 | rank; 0xffffffff: direct update
#pragma unroll
    for (int i = 0; i < kAggPer; ++i) {
        tag[i] = 0xffffffffu;
        const long long k = k0 + (long long)i * kAggThreads + threadIdx.x;
        VisCoords c;
        if (k < cr.k1 && vis_coords_of(xu[i], xv[i], xw[i], cr.ch, P, c)) {
            const int sl = agg_slot(T, bin_of(c, P));
            if (sl >= 0) tag[i] = (uint32_t(sl) << 16) | atomicAdd(&T.cnt[sl], 1u);
        }
    }
    __syncthreads();
    // one reservation per distinct bin of the block
    for (int i = threadIdx.x; i < kAggSlots; i += kAggThreads)
        if (T.key[i] >= 0) T.base[i] = atomicAdd(&cursor[T.key[i]], T.cnt[i]);
    __syncthreads();
    // pass 2: write the records
#pragma unroll
    for (int i = 0; i < kAggPer; ++i) {
        const long long k = k0 + (long long)i * kAggThreads + threadIdx.x;
        VisCoords c;
        if (!(k < cr.k1 && vis_coords_of(xu[i], xv[i], xw[i], cr.ch, P, c))) continue;
        const int b = bin_of(c, P);
        const uint32_t off = tag[i] != 0xffffffffu ? T.base[tag[i] >> 16] + (tag[i] & 0xffffu)
                                                   : atomicAdd(&cursor[b], 1u);
        Rec<R> r;
        r.ruv = uint32_t(c.ru) | (uint32_t(c.rv) << 16);
        r.rt = uint32_t(c.rt);
        r.nu[0] = R(c.nu_u);
        r.nu[1] = R(c.nu_v);
        r.nu[2] = R(c.nu_w);
        double turns = c.w * (-P.zshift * P.nscale);     // w (n0 - 1)
        double sn, co;
        phase_turns(GRID ? turns : -turns, &sn, &co);
        if (GRID) {
            cpx<R> V = vis[k];
            double vx = double(V.x), vy = c.folded ? -double(V.y) : double(V.y);
            r.v[0] = R(vx * co - vy * sn);
            r.v[1] = R(vx * sn + vy * co);
            r.idx = 0;
        } else {
            r.v[0] = R(co);
            r.v[1] = R(sn);
            r.idx = uint32_t(k) | (c.folded ? 0x80000000u : 0u);
        }
        rec[start[b] + off] = r;
    }
}

// Second-level sort and touch classes.  With B = 17 - W, a record whose first
// support index inside its tile is >= B along an axis also reaches the next
// tile along that axis (W <= 16: never the one after).  Its touch class is the
// 3-bit set c = (layer >= B) | (u >= B) << 1 | (v >= B) << 2.  A tile reads,
// from the bin one tile back along the axes of a set m, exactly the records
// whose class contains m.  Classes are stored in Gray-code order (position q
// holds class q ^ (q >> 1)): the records a tile needs from one bin are then at
// most two contiguous ranges, ten over the eight bins.  Inside a class, records
// are ordered by (layer, u, v) of their first support index, so that records
// with the same support box are adjacent (long runs along Earth-rotation
// tracks).
// With separate widths, the layer axis uses Bt = 17 - W_z and the u, v axes
// Buv = 17 - W.
__device__ __forceinline__ int class_part(int hi, int B) { return hi ? kTileT - B : B; }
__device__ __forceinline__ int class_position(int c) { return c ^ (c >> 1) ^ (c >> 2); }   // inverse Gray code
__device__ __forceinline__ int class_of(int lt, int lr, int ls, int Bt, int Buv) {
    return int(lt >= Bt) | (int(lr >= Buv) << 1) | (int(ls >= Buv) << 2);
}
// rank of the first key of class position q (q = 0..8) among the 4096 keys
__device__ __forceinline__ int class_base(int q, int Bt, int Buv) {
    int b = 0;
    for (int k = 0; k < q; ++k) {
        const int c = k ^ (k >> 1);
        b += class_part(c & 1, Bt) * class_part(c & 2, Buv) * class_part(c & 4, Buv);
    }
    return b;
}

// One block per bin: LDS histogram over the 4096 in-tile positions enumerated
// in (class position, layer, u, v) order, exclusive scan, scatter to `out`
// (order among equal keys is arbitrary).  cls[8 bin + q] receives the start of
// class position q in `out`.
template <typename R>
__global__ void __launch_bounds__(256) k_bin_local_sort(const Rec<R>* __restrict__ in, Rec<R>* __restrict__ out,
                                                        const uint32_t* __restrict__ start,
                                                        uint32_t* __restrict__ cls, DevParams P) {
    constexpr int NK = kTileT * kTileR * kTileS;
    __shared__ uint32_t hist[NK];
    __shared__ uint32_t sh[16];
    __shared__ int cbase[9];
    const int bin = blockIdx.x;
    const uint32_t b0 = start[bin], b1 = start[bin + 1];
    if (b1 == b0) return;
    const int br = bin % P.nbr, bs = (bin / P.nbr) % P.nbs, bt = bin / (P.nbr * P.nbs);
    const int tid = threadIdx.x;
    const int Buv = 17 - P.W, Bt = 17 - P.Wz;
    if (tid < 9) cbase[tid] = class_base(tid, Bt, Buv);
    for (int i = tid; i < NK; i += 256) hist[i] = 0u;
    __syncthreads();
    auto key_of = [&](const Rec<R>& r) {
        const int lr = int(r.ruv & 0xffffu) - br * kTileR, ls = int(r.ruv >> 16) - bs * kTileS;
        const int lt = int(r.rt) - bt * kTileT;
        const int c = class_of(lt, lr, ls, Bt, Buv);
        const int it = (c & 1) ? lt - Bt : lt, ir = (c & 2) ? lr - Buv : lr, is = (c & 4) ? ls - Buv : ls;
        return cbase[class_position(c)] + (it * class_part(c & 2, Buv) + ir) * class_part(c & 4, Buv) + is;
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
    if (tid < 8) cls[8 * size_t(bin) + tid] = b0 + (cbase[tid] < NK ? hist[cbase[tid]] : total);
    __syncthreads();
    for (uint32_t i = b0 + tid; i < b1; i += 256) {
        const Rec<R> r = in[i];
        out[b0 + atomicAdd(&hist[key_of(r)], 1u)] = r;
    }
}

// Tile occupancy: a tile is marked when some visibility reaches it: its own bin
// is non-empty, or the bin one tile back along the axes of a set m holds
// visibilities whose touch class contains m (from the class starts of the
// per-bin sort).  Only marked tiles of the stack are written (grid) or filled
// (degrid); the FFT passes treat unmarked tiles as zero (grid) or skip them
// (degrid).  A row of tiles (t tile, u tile) is marked in `rows` when one of
// its tiles is (`rows` zero on entry; racing stores all write 1).
static __global__ void k_tile_occupancy(const uint32_t* __restrict__ start, const uint32_t* __restrict__ cls, DevParams P,
                                 uint8_t* __restrict__ occ, uint8_t* __restrict__ rows, uint32_t* __restrict__ flag) {
    const int tile = blockIdx.x * blockDim.x + threadIdx.x;
    const int nt = P.nch * P.nbt * P.nbs * P.nbr;
    if (tile >= nt) return;
    const int br = tile % P.nbr, bs = (tile / P.nbr) % P.nbs, bt = tile / (P.nbr * P.nbs);
    bool any = false;
    for (int nb = 0; nb < 8 && !any; ++nb) {
        const int it = (nb >> 2) & 1, is = (nb >> 1) & 1, ir = nb & 1;
        if (bt % P.nbt - it < 0) continue;      // not across a channel start
        const int bin = ((bt - it) * P.nbs + (bs - is + P.nbs) % P.nbs) * P.nbr + (br - ir + P.nbr) % P.nbr;
        const uint32_t b0 = start[bin], b1 = start[bin + 1];
        if (b1 == b0) continue;
        const int m = it | (ir << 1) | (is << 2);
        for (int q = 0; q < 8; ++q) {
            const int c = q ^ (q >> 1);
            if ((c & m) != m) continue;
            const uint32_t lo = cls[8 * size_t(bin) + q], hi = q < 7 ? cls[8 * size_t(bin) + q + 1] : b1;
            if (hi > lo) {
                any = true;
                break;
            }
        }
    }
    occ[tile] = any ? 1 : 0;
    flag[tile] = any ? 1u : 0u;
    if (any) rows[bt * P.nbr + br] = 1;
}

// The occupied tiles in tile order: list[pos[t]] = t for every marked tile t,
// pos the exclusive scan of the flags (pos[n] = number of marked tiles).
static __global__ void k_tile_list(const uint8_t* __restrict__ occ, const uint32_t* __restrict__ pos, int n,
                            uint32_t* __restrict__ list) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && occ[t]) list[pos[t]] = uint32_t(t);
}

// ------------------------------------------------ 3-D scatter / gather tiles --
//
// One 256-thread block owns one tile of kTileT layers x kTileR u-cells x
// kTileS v-cells of the stack (layout [t][r][s], s fastest), held in LDS.  The
// records that reach the tile (from its own bin and the seven bins one tile
// back, selected by touch class) form a virtual list of at most 64 ranges of
// the record array.  The list is cut into four contiguous quarters, one per
// wave; the waves work independently between the tile's set-up and its
// write-out, and each holds its next records in registers while it works on
// the current ones.  Each tile is read or written to HBM once.

// Kernel polynomial degree in nu per precision (the host fits both).
template <typename R>
struct KernelDegree {
    static constexpr int value = sizeof(R) == 8 ? 16 : 8;
};

// The records that reach one tile: ranges [lo[g], lo[g] + off[g+1] - off[g])
// of the record array, concatenated into a virtual list [0, off[n]).
struct TileSegs {
    uint32_t lo[64];
    uint32_t off[65];
    uint8_t nbr[64];      // neighbour set of the range's bin: it | ir << 1 | is << 2
    int n;
};

// Built by wave 0 (a block barrier must follow).  Lane l handles class position
// q = l & 7 of the bin one tile back along t, v, u by the bits of l >> 3.
__device__ __forceinline__ void tile_segments(const uint32_t* __restrict__ start, const uint32_t* __restrict__ cls,
                                              const DevParams& P, int bt, int bs, int br, TileSegs& sg) {
    const int lane = threadIdx.x & 63;
    const int nb = lane >> 3, q = lane & 7;
    const int it = (nb >> 2) & 1, is = (nb >> 1) & 1, ir = nb & 1;
    uint32_t lo = 0, hi = 0;
    bool need = false;
    if (bt % P.nbt - it >= 0) {      // not across a channel start
        const int bin = ((bt - it) * P.nbs + (bs - is + P.nbs) % P.nbs) * P.nbr + (br - ir + P.nbr) % P.nbr;
        const uint32_t b0 = start[bin], b1 = start[bin + 1];
        if (b1 > b0) {
            lo = cls[8 * size_t(bin) + q];
            hi = q < 7 ? cls[8 * size_t(bin) + q + 1] : b1;
            const int c = q ^ (q >> 1);
            const int m = it | (ir << 1) | (is << 2);
            need = (c & m) == m;
        }
    }
    const uint32_t len = need ? hi - lo : 0u;
    const unsigned long long nm = __ballot(need);
    const bool first = need && !(q > 0 && ((nm >> (lane - 1)) & 1ull));
    const unsigned long long fm = __ballot(first);
    uint32_t inc = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (first) {
        const int g = __popcll(fm & ((1ull << lane) - 1ull));
        sg.lo[g] = lo;
        sg.off[g] = inc - len;
        sg.nbr[g] = uint8_t(it | (ir << 1) | (is << 2));
    }
    if (lane == 63) {
        const int n = __popcll(fm);
        sg.n = n;
        sg.off[n] = inc;
    }
}

// Record array index of virtual position v; g is the caller's current range,
// moved forward to the one holding v (a lane's positions only grow, so the
// search is incremental).
__device__ __forceinline__ uint32_t seg_advance(const TileSegs& sg, int n, uint32_t v, int& g) {
    while (g + 1 < n && sg.off[g + 1] <= v) ++g;
    return sg.lo[g] + (v - sg.off[g]);
}

// Signed offset of a support start from the tile origin along a periodic axis.
__device__ __forceinline__ int wrap_offset(int first, int origin, int Np) {
    int d = first - origin;
    if (d >= Np / 2) d -= Np;
    if (d < -Np / 2) d += Np;
    return d;
}

// x mod W in [0, W) for x > -16 W
template <int W>
__device__ __forceinline__ int mod_w(int x) {
    return (x + 16 * W) % W;
}

// The launch has one block per tile of the current layer pass (tile layers
// pl0 / kTileT onwards), and the blocks take the pass's occupied tiles from the
// ordered list (groups of 4 neighbours per XCD); the result is the global tile
// index, or -1 for a block beyond the occupied tiles (it exits at once).
__device__ __forceinline__ int tile_of_block(const DevParams& P, const uint32_t* __restrict__ tlist,
                                             const uint32_t* __restrict__ tpos) {
    const int per_layer = P.nbs * P.nbr;
    const int nbt_pass = (P.pln + kTileT - 1) / kTileT;
    const int a = (P.pl0 / kTileT) * per_layer, e = a + nbt_pass * per_layer;
    const int first = int(tpos[a]), cnt = int(tpos[e]) - first;
    if (int(blockIdx.x) >= cnt) return -1;
    return int(tlist[first + xcd_interleave<4>(blockIdx.x, cnt)]);
}

// Kernel weights of one record on the three axes by Horner's rule: u and v
// from coef (width W), the layer axis from coefz (width WZ).  SAME: the w-axis
// design is the u, v one (WZ == W), so each coefficient read feeds three chains.
template <typename R, int W, int WZ, bool SAME>
__device__ __forceinline__ void record_weights(const Rec<R>& r, const R* __restrict__ coef, const R* __restrict__ coefz,
                                               R (&wu)[W], R (&wv)[W], R (&wt)[WZ]) {
    constexpr int D = KernelDegree<R>::value;
    static_assert(!SAME || WZ == W, "one design on all axes needs equal widths");
#pragma unroll
    for (int a = 0; a < W; ++a) {
        const R* c = coef + a * (D + 1);
        const R* cz = (SAME ? coef : coefz) + (a < WZ ? a : 0) * (D + 1);
        R hu = c[D], hv = c[D], ht = cz[D];
#pragma unroll
        for (int k = D - 1; k >= 0; --k) {
            const R ck = c[k];
            hu = hu * r.nu[0] + ck;
            hv = hv * r.nu[1] + ck;
            ht = ht * r.nu[2] + (SAME ? ck : cz[k]);
        }
        wu[a] = hu;
        wv[a] = hv;
        if (a < WZ) wt[a] = ht;
    }
}

// Orders this wave's LDS accesses around a hand-over between its lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float bits_to_word(int v, float) { return __int_as_float(v); }
__device__ __forceinline__ double bits_to_word(int v, double) { return __hiloint2double(0, v); }
__device__ __forceinline__ int word_bits(float v) { return __float_as_int(v); }
__device__ __forceinline__ int word_bits(double v) { return __double2loint(v); }

// Scatter: residue classes (Romein 2012, extended to three axes).  Lane (x, y)
// owns, among the W x W x WZ support cells of a record, the WZ cells whose u
// and v indices are congruent to x and y modulo W, one per layer residue a: for
// support start (dr, ds, dt) the u-cell dr + ((x - dr) mod W), the v-cell
// ds + ((y - ds) mod W) and the layer dt + ((a - dt) mod WZ).  Each round a wave
// stages 16 or 32 records into its slots (four or two lanes per record): the u
// weights times the value and the v weights rotated by the support start (so lane x reads position x
// whatever the record), and the layer weights rotated by dt with the packed
// support start, read by the whole wave as broadcasts.  Sums stay in registers
// while the owned cell stays the same; when the support moves, the lanes (or
// layer residues) whose owned cell changed add their sums to the LDS tile
// (atomics: the four waves share it) and restart from zero.  Records are sorted
// by support start inside each touch class, so supports mostly coincide or
// move by one cell.
template <typename R, int W, int WZ>
struct ScatterCfg {
    // records per wave round: 16 (four lanes stage each) for W <= 7, where the
    // block then fits in 40 KB of LDS (FP32: four blocks per CU) or 80 KB
    // (FP64: two), else 32 (two lanes each; at W = 7 that measured 8 % slower)
    static constexpr int kWaveBatch = W <= 7 ? 16 : 32;
    static constexpr int kLanesPerRecord = 64 / kWaveBatch;
    // waves per block, each on its own part of the tile's record list (eight
    // waves at three blocks per CU measured 13 % slower than four at four)
    static constexpr int kWaves = 4;
    static constexpr int kThreads = 64 * kWaves;
    static constexpr int kSlots = kWaves * kWaveBatch;
    static constexpr int kPairs = W * W;
    static constexpr int kPI = (kPairs + 63) / 64;                // (x, y) residue pairs per lane
    static constexpr int kCells = kTileT * kTileR * kTileS;
    static constexpr int kWords = (WZ * sizeof(R) + 15) / 16 * 16 / sizeof(R);   // 16-byte rows
};

template <typename R, int W, int WZ>
struct __align__(16) ScatterStage {
    // layer weights rotated (position (a + dt) mod WZ holds C_z(s_a - nu_w))
    R words[ScatterCfg<R, W, WZ>::kSlots][ScatterCfg<R, W, WZ>::kWords];
    // value times u weights (real, imaginary), rotated by dr; v weights rotated by ds
    R wuv[ScatterCfg<R, W, WZ>::kSlots][3 * W];
};

// PREP: the records are those of a shared binning (degridding records: the
// phase e^{-i 2 pi w (n0 - 1)} and the visibility index with the fold flag);
// each record's value is then the visibility it names, conjugated when folded,
// times the conjugate phase (formed in FP64), and the lane keeps two records
// in flight so that the value's load (which needs the record's index) is
// issued a round before its staging.
template <typename R, int W, int WZ, bool SAME, bool PREP>
__global__ void __launch_bounds__((ScatterCfg<R, W, WZ>::kThreads)) k_grid_tiles(const Rec<R>* __restrict__ rec,
                                                    const uint32_t* __restrict__ start,
                                                    const uint32_t* __restrict__ cls,
                                                    const uint32_t* __restrict__ tlist,
                                                    const uint32_t* __restrict__ tpos, DevParams P,
                                                    const R* __restrict__ coef_g, const R* __restrict__ coefz_g,
                                                    const cpx<R>* __restrict__ vis, cpx<R>* __restrict__ stack) {
    using Cfg = ScatterCfg<R, W, WZ>;
    constexpr int PI = Cfg::kPI, WB = Cfg::kWaveBatch, D = KernelDegree<R>::value;
    __shared__ R tre[Cfg::kCells];
    __shared__ R tim[Cfg::kCells];
    __shared__ ScatterStage<R, W, WZ> st;
    __shared__ TileSegs sg;

    const int tile = tile_of_block(P, tlist, tpos);
    if (tile < 0) return;     // unoccupied tiles are left unwritten and read as zero
    const int br = tile % P.nbr, bs = (tile / P.nbr) % P.nbs, bt = tile / (P.nbr * P.nbs);
    const int r0 = br * kTileR, s0 = bs * kTileS, t0 = bt * kTileT;
    const int nt_valid = min(kTileT, P.n_layers - t0 % (P.nbt * kTileT));   // layers of its channel
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);

    constexpr int NT = Cfg::kThreads, NW = Cfg::kWaves;
    if (tid < 64) tile_segments(start, cls, P, bt, bs, br, sg);
    for (int i = tid; i < Cfg::kCells; i += NT) tre[i] = tim[i] = R(0);
    __syncthreads();
    const int nseg = sg.n;
    const uint32_t total = sg.off[nseg];
    // this wave's part of the list
    const uint32_t part = (total + NW - 1) / NW;
    const uint32_t q0 = min(total, part * uint32_t(wv)), q1 = min(total, q0 + part);

    if (q1 > q0) {
        // the lane's residue pairs, owned cells and register sums
        int px[PI], py[PI], cr[PI], cs[PI];
        bool pv[PI];
#pragma unroll
        for (int i = 0; i < PI; ++i) {
            const int p = lane + 64 * i;
            pv[i] = p < Cfg::kPairs;
            const int pc = min(p, Cfg::kPairs - 1);
            px[i] = pc / W;
            py[i] = pc % W;
            cr[i] = cs[i] = -1000;
        }
        int ct[WZ];                                  // owned layer per residue (wave-uniform)
        R ax[PI][WZ], ay[PI][WZ];
#pragma unroll
        for (int a = 0; a < WZ; ++a) ct[a] = -1000;
#pragma unroll
        for (int i = 0; i < PI; ++i)
#pragma unroll
            for (int a = 0; a < WZ; ++a) ax[i][a] = ay[i][a] = R(0);
        // add sum (i, a) to its owned cell if that cell is in the tile
        auto add_cell = [&](int i, int a) {
            const int t = ct[a];
            if (pv[i] && unsigned(cr[i]) < unsigned(kTileR) && unsigned(cs[i]) < unsigned(kTileS) &&
                unsigned(t) < unsigned(nt_valid)) {
                const int cell = (t * kTileR + cr[i]) * kTileS + cs[i];
                atomicAdd(&tre[cell], ax[i][a]);
                atomicAdd(&tim[cell], ay[i][a]);
            }
            ax[i][a] = ay[i][a] = R(0);
        };
        int prev = -1, prev_dt = -1000;
        // the support starts at packed d: flush the sums of owned cells that change
        auto move_to = [&](int d) {
            prev = d;
            const int dr = (d & 255) - 128, ds = ((d >> 8) & 255) - 128, dt = ((d >> 16) & 255) - 128;
            const int mr = mod_w<W>(-dr), ms = mod_w<W>(-ds);
#pragma unroll
            for (int i = 0; i < PI; ++i) {
                int xr = px[i] + mr, ys = py[i] + ms;
                xr -= xr >= W ? W : 0;
                ys -= ys >= W ? W : 0;
                const int nr = dr + xr, ns = ds + ys;
                if (nr != cr[i] || ns != cs[i]) {
#pragma unroll
                    for (int a = 0; a < WZ; ++a) add_cell(i, a);
                    cr[i] = nr;
                    cs[i] = ns;
                }
            }
            if (dt != prev_dt) {
                prev_dt = dt;
                const int mt = mod_w<WZ>(-dt);
#pragma unroll
                for (int a = 0; a < WZ; ++a) {
                    int k = a + mt;
                    k -= k >= WZ ? WZ : 0;
                    const int nt = dt + k;
                    if (nt != ct[a]) {
#pragma unroll
                        for (int i = 0; i < PI; ++i) add_cell(i, a);
                        ct[a] = nt;
                    }
                }
            }
        };

        const int slot0 = wv * WB;
        // staging: the lanes rl + WB h (h = 0 .. LPR - 1) take record rl, lane h
        // the kernel segments [h A0, (h + 1) A0), so the Horner work is spread
        // over the whole wave; the coefficients come from global memory (the
        // whole wave reads the same few, so the vector cache serves them)
        constexpr int LPR = Cfg::kLanesPerRecord;
        static_assert(WB * LPR == 64, "the wave stages WB records with LPR lanes each");
        constexpr int A0 = (W + LPR - 1) / LPR;
        static_assert(WZ <= W, "the w-axis function is at most as wide as the u, v one");
        const int rl = lane & (WB - 1), half = lane / WB;
        // The lane's coefficients, loaded once into registers when they fit in
        // 40 of them (else read from global memory at each staging).
        constexpr bool kRegCoef = A0 * (D + 1) * (SAME ? 1 : 2) * int(sizeof(R)) <= 160;
        R creg[kRegCoef ? A0 : 1][D + 1], czreg[(kRegCoef && !SAME) ? A0 : 1][D + 1];
        if constexpr (kRegCoef) {
#pragma unroll
            for (int i = 0; i < A0; ++i) {
                const int a = i + half * A0;
#pragma unroll
                for (int k = 0; k <= D; ++k) {
                    creg[i][k] = coef_g[min(a, W - 1) * (D + 1) + k];
                    if constexpr (!SAME) czreg[i][k] = coefz_g[min(a, WZ - 1) * (D + 1) + k];
                }
            }
        }
        // the lane's next record: virtual position vn in range g (ranges only
        // move forward as vn grows by WB per round)
        uint32_t vn = q0 + uint32_t(rl);
        int g = 0;
        Rec<R> nxt{}, nxt2{};
        cpx<R> nval{R(0), R(0)};
        if (vn < q1) nxt = rec[seg_advance(sg, nseg, vn, g)];
        if constexpr (PREP) {
            if (vn < q1) nval = vis[nxt.idx & 0x7fffffffu];
            if (vn + WB < q1) nxt2 = rec[seg_advance(sg, nseg, vn + WB, g)];
        }
        for (uint32_t base = q0; base < q1; base += WB) {
            const int n = __builtin_amdgcn_readfirstlane(int(min(uint32_t(WB), q1 - base)));
            // support start of this lane's record, relative to the tile, packed
            const int dr = wrap_offset(int(nxt.ruv & 0xffffu), r0, P.Np);
            const int ds = wrap_offset(int(nxt.ruv >> 16), s0, P.Np);
            const int dt = int(nxt.rt) - t0;
            const int d = (dr + 128) | ((ds + 128) << 8) | ((dt + 128) << 16);
            if (rl < n) {
                // stage: rotated weights, value folded into the u weights
                const int pr = mod_w<W>(dr), ps = mod_w<W>(ds), pt = mod_w<WZ>(dt);
                const int slot = slot0 + rl;
                R v0 = nxt.v[0], v1 = nxt.v[1];
                if constexpr (PREP) {
                    const double vx = double(nval.x), vy = (nxt.idx & 0x80000000u) ? -double(nval.y) : double(nval.y);
                    const double co = double(nxt.v[0]), sn = -double(nxt.v[1]);
                    v0 = R(vx * co - vy * sn);
                    v1 = R(vx * sn + vy * co);
                }
#pragma unroll
                for (int i = 0; i < A0; ++i) {
                    const int a = i + half * A0;
                    const R* c = coef_g + min(a, W - 1) * (D + 1);
                    const R* cz = (SAME ? coef_g : coefz_g) + min(a, WZ - 1) * (D + 1);
                    auto cu = [&](int k) { if constexpr (kRegCoef) return creg[i][k]; else return c[k]; };
                    auto cw = [&](int k) {
                        if constexpr (SAME) return cu(k);
                        else if constexpr (kRegCoef) return czreg[i][k];
                        else return cz[k];
                    };
                    R hu = cu(D), hv = cu(D), ht = cw(D);
#pragma unroll
                    for (int k = D - 1; k >= 0; --k) {
                        const R ck = cu(k);
                        hu = hu * nxt.nu[0] + ck;
                        hv = hv * nxt.nu[1] + ck;
                        ht = ht * nxt.nu[2] + cw(k);
                    }
                    if (a < W) {
                        int ku = pr + a, kv = ps + a;
                        ku -= ku >= W ? W : 0;
                        kv -= kv >= W ? W : 0;
                        st.wuv[slot][ku] = v0 * hu;
                        st.wuv[slot][W + ku] = v1 * hu;
                        st.wuv[slot][2 * W + kv] = hv;
                    }
                    if (a < WZ) {
                        int kt = pt + a;
                        kt -= kt >= WZ ? WZ : 0;
                        st.words[slot][kt] = ht;
                    }
                }
            }
            // slots whose support start differs from the previous slot's (slot 0:
            // from the wave's current one): a scalar bit mask, so that the
            // per-record check below costs no vector instruction
            const int d_before = __shfl_up(d, 1, 64);
            const bool moved = half == 0 && rl < n && (rl == 0 ? d != prev : d != d_before);
            const uint64_t move_mask = __ballot(moved);
            wave_sync();
            vn += WB;
            if constexpr (PREP) {
                nxt = nxt2;
                if (vn < q1) nval = vis[nxt.idx & 0x7fffffffu];
                if (vn + WB < q1) nxt2 = rec[seg_advance(sg, nseg, vn + WB, g)];
            } else {
                if (vn < q1) nxt = rec[seg_advance(sg, nseg, vn, g)];
            }

            // groups of four slots with fixed offsets (one address update per
            // group); each slot's stage values are read while the previous
            // slot's products are formed
            struct Slot {
                R wt[WZ], fx[PI], fy[PI], fv[PI];
            };
            auto read_slot = [&](int slot, Slot& q) {
#pragma unroll
                for (int a = 0; a < WZ; ++a) q.wt[a] = st.words[slot][a];      // broadcast
#pragma unroll
                for (int i = 0; i < PI; ++i) {
                    q.fx[i] = st.wuv[slot][px[i]];
                    q.fy[i] = st.wuv[slot][W + px[i]];
                    q.fv[i] = st.wuv[slot][2 * W + py[i]];
                }
            };
            Slot q[2];            // slot j in q[j & 1]: two register sets, no copies
            read_slot(slot0, q[0]);
            for (int j0 = 0; j0 < n; j0 += 4) {
                const uint32_t m4 = uint32_t(move_mask >> j0) & 15u;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int j = j0 + jj;
                    if (j >= n) break;
                    if (j + 1 < n) read_slot(slot0 + j + 1, q[(jj + 1) & 1]);
                    if (m4 & (1u << jj)) move_to(__builtin_amdgcn_readlane(d, j));
                    const Slot& c = q[jj & 1];
#pragma unroll
                    for (int i = 0; i < PI; ++i) {
                        const R gx = c.fx[i] * c.fv[i], gy = c.fy[i] * c.fv[i];
#pragma unroll
                        for (int a = 0; a < WZ; ++a) {
                            ax[i][a] += gx * c.wt[a];
                            ay[i][a] += gy * c.wt[a];
                        }
                    }
                }
            }
            wave_sync();
        }
#pragma unroll
        for (int i = 0; i < PI; ++i)
#pragma unroll
            for (int a = 0; a < WZ; ++a) add_cell(i, a);
    }
    __syncthreads();
    // write the tile: rows of kTileS cells
    for (int i = tid; i < nt_valid * kTileR * kTileS; i += NT) {
        const int ss = i % kTileS, rr = (i / kTileS) % kTileR, tt = i / (kTileR * kTileS);
        stack[((size_t)(t0 - P.pl0 + tt) * P.Np + (r0 + rr)) * P.Np + (s0 + ss)] = cpx<R>{tre[i], tim[i]};
    }
}

// Gather: lanes over records.  The tile sits in LDS as complex cells, rows
// kLR = 17 cells and layers kLT = 16 kLR + 1 cells apart (the padding cells are
// zero), with a zero guard of (kLR + 1)(W - 1) cells before and after, so that
// for any support start (dr, ds) in [-(W-1), 15] the cell address
// base + kLR x + y of every support offset is inside the array.  Each lane
// evaluates its own record's weights, sets those of out-of-tile indices to zero
// (the cells read there are finite neighbours or zeros), clamps the layer of
// each residue and sums the W^3 products; no cross-lane reduction is needed.
template <typename R, int W>
struct GatherCfg {
    static constexpr int kLR = kTileS + 1;              // row stride (cells): skews rows and
    static constexpr int kLT = kTileR * kLR + 1;        // layers over the LDS banks
    static constexpr int kGuard = (kLR + 1) * (W - 1);
    static constexpr int kCells = kTileT * kLT;
    static constexpr int kLen = kCells + 2 * kGuard;
};

// At least two waves per SIMD: left alone, the FP64 instances hold a layer's
// cell loads in flight in 320 registers (one wave per SIMD); at two waves they
// spill a little and run 1.5x faster (FP32 is at four waves either way).
template <typename R, int W, int WZ, bool SAME>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_degrid_tiles(const Rec<R>* __restrict__ rec,
                                                      const uint32_t* __restrict__ start,
                                                      const uint32_t* __restrict__ cls,
                                                      const uint32_t* __restrict__ tlist,
                                                      const uint32_t* __restrict__ tpos, DevParams P,
                                                      const R* __restrict__ coef_g,
                                                      const R* __restrict__ coefz_g,
                                                      const cpx<R>* __restrict__ stack, cpx<R>* __restrict__ part,
                                                      size_t part_stride) {
    using G = GatherCfg<R, W>;
    constexpr int D = KernelDegree<R>::value;
    constexpr int WB = 64;
    __shared__ cpx<R> g[G::kLen];
    __shared__ R coef[W * (D + 1)];
    __shared__ R coefz[SAME ? 1 : WZ * (D + 1)];
    __shared__ TileSegs sg;

    const int tile = tile_of_block(P, tlist, tpos);
    if (tile < 0) return;     // only occupied tiles are visited
    const int br = tile % P.nbr, bs = (tile / P.nbr) % P.nbs, bt = tile / (P.nbr * P.nbs);
    const int r0 = br * kTileR, s0 = bs * kTileS, t0 = bt * kTileT;
    const int nt_valid = min(kTileT, P.n_layers - t0 % (P.nbt * kTileT));   // layers of its channel
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);

    if (tid < 64) tile_segments(start, cls, P, bt, bs, br, sg);
    for (int i = tid; i < W * (D + 1); i += 256) coef[i] = coef_g[i];
    if (!SAME)
        for (int i = tid; i < WZ * (D + 1); i += 256) coefz[i] = coefz_g[i];
    __syncthreads();
    const int nseg = sg.n;
    const uint32_t total = sg.off[nseg];
    if (total == 0) return;     // a tile no visibility reaches is not read at all
    const uint32_t quarter = (total + 3) / 4;
    const uint32_t q0 = min(total, quarter * uint32_t(wv)), q1 = min(total, q0 + quarter);

    Rec<R> nxt;
    uint32_t nxt_p = 0, nxt_m = 0;
    int g_ = 0;
    if (q0 + uint32_t(lane) < q1) {
        nxt_p = seg_advance(sg, nseg, q0 + uint32_t(lane), g_);
        nxt_m = sg.nbr[g_];
        nxt = rec[nxt_p];
    }
    for (int i = tid; i < G::kLen; i += 256) {
        const int c = i - G::kGuard;
        cpx<R> q{R(0), R(0)};
        if (c >= 0 && c < G::kCells) {
            const int tt = c / G::kLT, rem = c % G::kLT, rr = rem / G::kLR, ss = rem % G::kLR;
            if (tt < nt_valid && rr < kTileR && ss < kTileS)
                q = stack[((size_t)(t0 - P.pl0 + tt) * P.Np + (r0 + rr)) * P.Np + (s0 + ss)];
        }
        g[i] = q;
    }
    __syncthreads();

    for (uint32_t base = q0; base < q1; base += WB) {
        const bool live = base + uint32_t(lane) < q1;
        const Rec<R> r = nxt;
        const uint32_t p = nxt_p, m = nxt_m;
        const uint32_t vn = base + WB + uint32_t(lane);
        if (vn < q1) {
            nxt_p = seg_advance(sg, nseg, vn, g_);
            nxt_m = sg.nbr[g_];
            nxt = rec[nxt_p];
        }
        if (!live) continue;

        const int dr = wrap_offset(int(r.ruv & 0xffffu), r0, P.Np);
        const int ds = wrap_offset(int(r.ruv >> 16), s0, P.Np);
        const int dt = int(r.rt) - t0;
        R wu[W], wv_[W], wt[WZ];
        record_weights<R, W, WZ, SAME>(r, coef, coefz, wu, wv_, wt);
#pragma unroll
        for (int a = 0; a < W; ++a) {
            wu[a] = unsigned(dr + a) < unsigned(kTileR) ? wu[a] : R(0);
            wv_[a] = unsigned(ds + a) < unsigned(kTileS) ? wv_[a] : R(0);
        }
#pragma unroll
        for (int a = 0; a < WZ; ++a) wt[a] = unsigned(dt + a) < unsigned(nt_valid) ? wt[a] : R(0);
        const cpx<R>* row = g + (G::kGuard + dr * G::kLR + ds);
        R sx = R(0), sy = R(0);
#pragma unroll
        for (int a = 0; a < WZ; ++a) {
            const int tt = min(max(dt + a, 0), kTileT - 1);
            const cpx<R>* pa = row + tt * G::kLT;
            R ax = R(0), ay = R(0);
#pragma unroll
            for (int x = 0; x < W; ++x) {
                R bx = R(0), by = R(0);
#pragma unroll
                for (int y = 0; y < W; ++y) {
                    const cpx<R> q = pa[x * G::kLR + y];
                    bx += q.x * wv_[y];
                    by += q.y * wv_[y];
                }
                ax += bx * wu[x];
                ay += by * wu[x];
            }
            sx += ax * wt[a];
            sy += ay * wt[a];
        }
        // this tile's part of record p, in the slot of the tile's offset from
        // the record's own bin (no two tiles share a slot)
        part[(size_t)m * part_stride + p] = cpx<R>{sx, sy};
    }
}

// Sum of each record's parts over the tiles it reaches (slot m is written by
// the tile one step forward along the axes of m, present when the record's
// touch class contains m), times the phase exp(-i 2 pi w (n0 - 1)), conjugated
// for a folded visibility, stored to its visibility.
template <typename R>
__global__ void k_degrid_finish(const Rec<R>* __restrict__ rec, const uint32_t* __restrict__ n_rec,
                                const cpx<R>* __restrict__ part, size_t part_stride, int W, int Wz,
                                cpx<R>* __restrict__ vis) {
    const size_t p = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= *n_rec) return;
    const Rec<R> r = rec[p];
    const int c = class_of(int(r.rt) & (kTileT - 1), int(r.ruv & 0xffffu) & (kTileR - 1),
                           int(r.ruv >> 16) & (kTileS - 1), 17 - Wz, 17 - W);
    R sx = R(0), sy = R(0);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        if ((c & m) == m) {
            const cpx<R> q = part[(size_t)m * part_stride + p];
            sx += q.x;
            sy += q.y;
        }
    }
    R ox = sx * r.v[0] - sy * r.v[1], oy = sx * r.v[1] + sy * r.v[0];
    if (r.idx & 0x80000000u) oy = -oy;
    vis[r.idx & 0x7fffffffu] = cpx<R>{ox, oy};
}

// --------------------------------------------------------------- FFT passes --
//
// Stack layout [t][r][s] (s fastest).  Every FFT pass reads and writes whole
// lines: grid writes [t][r][q] and reads [t][q][r], degrid writes [t][q][r] and
// reads [t][r][q], with k_transpose in between (q is the image row).  Image
// rows j <-> q and columns i <-> p.  The FFT output bin
// f of a line maps to image index (f + N/2) mod N' and is kept when below N
// (Algorithm 5 step 3c); the degrid input places image index p at bin
// (p - N/2) mod N' (zero padding, Algorithm 6 step 3b).

template <typename R, int NP>
struct FftCfg {
    static constexpr int N = NP;
    static constexpr int T = N / 16;
    // lines per block for the row passes: at least ~256 threads; lengths 3 2^a
    // (T = 3 2^b) take 384 threads in FP32, so that 2048 rows fill whole rounds
    // of blocks (one 192-thread line per block left a partly empty last round;
    // FP64 at 384 threads measured 28 % slower)
    static constexpr int kNLr =
        (T >= 256) ? 1 : (N % 3 == 0 && T < 384 && sizeof(R) == 4) ? 384 / T : 256 / T;
    // lines per block for the tile-row passes: a power of two dividing the 16
    // rows of a row of tiles
    static constexpr int kNLt = kNLr >= 16 ? 16 : kNLr >= 8 ? 8 : kNLr >= 4 ? 4 : kNLr >= 2 ? 2 : 1;
};

// (f + N/2) mod N' for a bin f < N' (image index of FFT bin f, or the bin of
// image index f)
template <int NP>
__device__ __forceinline__ int shift_half(int f, int half) {
    const int q = f + half;
    return q >= NP ? q - NP : q;
}

// grid pass A: IFFT along s of stack rows [t][r][:], keep image rows q, write
// the lines [t][r][q] (transposed afterwards by k_transpose).  One block per
// layer and row of tiles (kTileR stack rows, taken NL at a time); the next NL
// rows are loaded while the current ones are transformed.  Unmarked tiles are
// read as zero; a row of tiles with none marked is neither transformed nor
// written (its lines are zero).  Layer t of the pass is virtual layer
// t + t_base; in a batched call (chl = the channels' layer stride, else 0) a
// padding layer (virtual layer mod chl >= n_layers) is skipped.
template <typename R, int NP>
__global__ void __launch_bounds__((FftCfg<R, NP>::kNLt * FftCfg<R, NP>::T))
    k_grid_fft_a(const cpx<R>* __restrict__ stack, const uint8_t* __restrict__ occ, cpx<R>* __restrict__ inter,
                 const cpx<R>* __restrict__ tw, int N, int n_layers, int chl, int nbr, int t_base) {
    using C = FftCfg<R, NP>;
    constexpr int Np = C::N, T = C::T, NL = C::kNLt, LP = LinePad<Np>::size, NG = kTileR / NL;
    static_assert(kTileR % NL == 0, "a row of tiles is a whole number of line groups");
    __shared__ cpx<R> buf[NL * LP];
    const int rows = Np / kTileR;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int t = lb / rows, rt = lb % rows;
    if (chl > 0 && (t + t_base) % chl >= n_layers) return;     // padding layer of a channel (block-uniform)
    const int line = threadIdx.x / T, j = threadIdx.x % T;
    cpx<R>* lbuf = buf + line * LP;
    // tile (t / 16, s / 16, rt) holds s = j + T k
    const uint8_t* orow = occ + (size_t)((t + t_base) / kTileT) * (Np / kTileS) * nbr + rt;
    bool on[16], any = false;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        on[k] = orow[(size_t)((j + T * k) / kTileS) * nbr] != 0;
        any = any || on[k];
    }
    cpx<R>* dst0 = inter + ((size_t)t * Np + rt * kTileR) * N;
    if (!__syncthreads_or(any)) return;     // zero lines: the transpose reads them as zeros
    auto load = [&](int g, cpx<R> (&v)[16]) {
        const cpx<R>* src = stack + ((size_t)t * Np + (rt * kTileR + g * NL + line)) * Np;
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = on[k] ? src[j + T * k] : cpx<R>{R(0), R(0)};
    };
    const int half = N / 2;
    cpx<R> nx[16];
    load(0, nx);
    for (int g = 0; g < NG; ++g) {
        cpx<R> v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = nx[k];
        if (g + 1 < NG) load(g + 1, nx);
        fft_line<R, NP, +1>(v, lbuf, tw, j);
        // bin f = j + T k holds image row q = (f + N/2) mod N', kept when below N
        cpx<R>* dst = dst0 + (size_t)(g * NL + line) * N;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int q = shift_half<Np>(j + T * k, half);
            if (q < N) store_stream(dst + q, v[k]);
        }
    }
}

// Bit k set when frequency r = j + T k (the k-th value of thread j of a line)
// lies in a marked row of tiles of the tile layer whose marks start at `mark`.
template <int T>
__device__ __forceinline__ uint32_t live_mask(const uint8_t* __restrict__ mark, int j) {
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) m |= uint32_t(mark[(j + T * k) / kTileR] != 0) << k;
    return m;
}

// grid pass B: IFFT along r of intermediate rows [t][q][:] for every layer t,
// w-screen exp(+i 2 pi t z) and accumulation of the real part in registers
// (Algorithm 5 steps 3b-4), then the 3-D correction (step 5): dirty[q][p].
// One launch covers a segment of P.pln consecutive layers of one channel: the
// segment starts at layer seg0 of the pass's buffer and at layer tloc0 of the
// channel; `accumulate` adds to the map instead of writing it.
template <typename R, int NP>
__global__ void __launch_bounds__((FftCfg<R, NP>::kNLr * FftCfg<R, NP>::T))
    k_grid_fft_b(const cpx<R>* __restrict__ inter, const uint8_t* __restrict__ rows, const cpx<R>* __restrict__ tw,
                 const R* __restrict__ corr, R* __restrict__ dirty, DevParams P, int seg0, int tloc0, int accumulate) {
    using C = FftCfg<R, NP>;
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
        const int p = shift_half<Np>(f, half);
        pix[k] = (row_ok && p < N) ? p : -1;
        const double l = double(min(p, N - 1) - half) * P.dl;   // bins outside the image are not used
        const double r2 = l * l + m * m;
        const double nm1 = -r2 / (1.0 + sqrt(1.0 - r2));     // n - 1
        z[k] = nm1 / P.nscale + P.zshift;                     // (n - n0) / n_scale
        acc[k] = R(0);
    }
    // bit k: frequency r = j + T k lies in a row of tiles with an occupied tile
    // in the current tile layer (the others are zero and not stored)
    uint32_t live = 0;
    int live_layer = -1;
    for (int t = 0; t < P.pln; ++t) {
        const cpx<R>* src = inter + ((size_t)(seg0 + t) * N + qq) * Np;
        const int tile_layer = __builtin_amdgcn_readfirstlane((P.pl0 + seg0 + t) / kTileT);
        if (tile_layer != live_layer) {
            live_layer = tile_layer;
            live = live_mask<T>(rows + (size_t)tile_layer * P.nbr, j);
        }
        cpx<R> v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = (live >> k) & 1u ? src[j + T * k] : cpx<R>{R(0), R(0)};
        fft_line<R, NP, +1>(v, lbuf, tw, j);
        const double tl = double(tloc0 + t + P.t_lo) + P.tphase;
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
    // the channel's first layer segment writes the map, later ones add to it
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (pix[k] >= 0) {
            const size_t o = (size_t)q * N + pix[k];
            const R d = acc[k] * corr[o];
            dirty[o] = accumulate ? dirty[o] + d : d;
        }
}

// degrid pass B': for each image row q and layer t: f h_x h_y h_z exp(-i 2 pi t z)
// zero-padded along p, FFT along p -> intermediate [t][q][r] (Algorithm 6 steps 2-3).
// Segments of one channel's layers as for k_grid_fft_b.
template <typename R, int NP>
__global__ void __launch_bounds__((FftCfg<R, NP>::kNLr * FftCfg<R, NP>::T))
    k_degrid_fft_b(const R* __restrict__ image, const R* __restrict__ corr, const cpx<R>* __restrict__ tw,
                   const uint8_t* __restrict__ rows, cpx<R>* __restrict__ inter, DevParams P, int seg0, int tloc0) {
    using C = FftCfg<R, NP>;
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
        const int p = shift_half<Np>(f, half);
        const bool ok = row_ok && p < N;
        g[k] = ok ? image[(size_t)qq * N + p] * corr[(size_t)qq * N + p] : R(0);
        const double l = double(min(p, N - 1) - half) * P.dl;   // keeps z finite on padding bins
        const double r2 = l * l + m * m;
        const double nm1 = -r2 / (1.0 + sqrt(1.0 - r2));
        z[k] = nm1 / P.nscale + P.zshift;
    }
    uint32_t live = 0;
    int live_layer = -1;
    for (int t = 0; t < P.pln; ++t) {
        const double tl = double(tloc0 + t + P.t_lo) + P.tphase;
        cpx<R> v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            R s, c;
            phase_turns(-tl * z[k], &s, &c);
            v[k] = cpx<R>{g[k] * c, g[k] * s};
        }
        fft_line<R, NP, -1>(v, lbuf, tw, j);
        if (row_ok) {
            // only frequencies r of rows of tiles with an occupied tile are used later
            const int tile_layer = __builtin_amdgcn_readfirstlane((P.pl0 + seg0 + t) / kTileT);
            if (tile_layer != live_layer) {
                live_layer = tile_layer;
                live = live_mask<T>(rows + (size_t)tile_layer * P.nbr, j);
            }
            cpx<R>* dst = inter + ((size_t)(seg0 + t) * N + q) * Np;
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if ((live >> k) & 1u) store_stream(dst + j + T * k, v[k]);
        }
    }
}

// degrid pass A': for each layer t and frequency r: the intermediate line
// [t][r][:] placed at its bins and zero-padded along q, FFT along q -> stack
// row [t][r][s].  One block per layer and row of tiles (kTileR lines, taken NL
// at a time); the next NL lines are loaded while the current ones are
// transformed.  Only marked tiles are stored (the gather reads no other); a row
// of tiles with none marked is skipped.  Layers and padding layers as for
// k_grid_fft_a.
template <typename R, int NP>
__global__ void __launch_bounds__((FftCfg<R, NP>::kNLt * FftCfg<R, NP>::T))
    k_degrid_fft_a(const cpx<R>* __restrict__ inter, const uint8_t* __restrict__ occ, const cpx<R>* __restrict__ tw,
                   cpx<R>* __restrict__ stack, int N, int n_layers, int chl, int nbr, int t_base) {
    using C = FftCfg<R, NP>;
    constexpr int Np = C::N, T = C::T, NL = C::kNLt, LP = LinePad<Np>::size, NG = kTileR / NL;
    static_assert(kTileR % NL == 0, "a row of tiles is a whole number of line groups");
    __shared__ cpx<R> buf[NL * LP];
    const int rows = Np / kTileR;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int t = lb / rows, rt = lb % rows;
    if (chl > 0 && (t + t_base) % chl >= n_layers) return;     // padding layer of a channel (block-uniform)
    const int line = threadIdx.x / T, j = threadIdx.x % T;
    cpx<R>* lbuf = buf + line * LP;
    const uint8_t* orow = occ + (size_t)((t + t_base) / kTileT) * (Np / kTileS) * nbr + rt;
    bool on[16], any = false;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        on[k] = orow[(size_t)((j + T * k) / kTileS) * nbr] != 0;
        any = any || on[k];
    }
    if (!__syncthreads_or(any)) return;
    const int half = N / 2;
    // thread j of a line holds bins f = j + T k; bin f carries image row
    // q = (f + N/2) mod N' when that is below N, else zero padding
    auto load = [&](int g, cpx<R> (&v)[16]) {
        const cpx<R>* src = inter + ((size_t)t * Np + (rt * kTileR + g * NL + line)) * N;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int q = shift_half<Np>(j + T * k, half);
            v[k] = q < N ? src[q] : cpx<R>{R(0), R(0)};
        }
    };
    cpx<R> nx[16];
    load(0, nx);
    for (int g = 0; g < NG; ++g) {
        cpx<R> v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = nx[k];
        if (g + 1 < NG) load(g + 1, nx);
        fft_line<R, NP, -1>(v, lbuf, tw, j);
        cpx<R>* dst = stack + ((size_t)t * Np + (rt * kTileR + g * NL + line)) * Np;
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (on[k]) dst[j + T * k] = v[k];
    }
}

// out[t][b][a] = in[t][a][b] for a < A, b < B, through a 64 x 64 LDS tile:
// reads and writes are whole 64-element rows (512 B FP32) away from the edges.
// The stack frequency r (16 per row of tiles) is the row index a of the input
// when R_IN, else the row index b of the output.  Lines of r whose row of
// tiles (t / 16, r / 16) is not marked in `rows` are zero on input (R_IN: not
// read) or not needed on output (not written; a tile with none needed is
// skipped whole).
template <typename R, int THREADS, bool R_IN>
__global__ void __launch_bounds__(THREADS) k_transpose(const cpx<R>* __restrict__ in, cpx<R>* __restrict__ out,
                                                       int A, int B, const uint8_t* __restrict__ rows, int nbr,
                                                       int t_base, int chl, int n_layers) {
    __shared__ cpx<R> tile[64][65];
    __shared__ uint8_t live[4];
    const int ta_n = (A + 63) / 64, tb_n = (B + 63) / 64;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int t = lb / (ta_n * tb_n), rem = lb % (ta_n * tb_n);
    if (chl > 0 && (t + t_base) % chl >= n_layers) return;     // padding layer of a channel (block-uniform)
    const int a0 = (rem / tb_n) * 64, b0 = (rem % tb_n) * 64;
    const int r0 = R_IN ? a0 : b0;
    if (threadIdx.x < 4)
        live[threadIdx.x] = rows[((t + t_base) / kTileT) * nbr + min(r0 / kTileR + int(threadIdx.x), nbr - 1)];
    __syncthreads();
    if (!(live[0] | live[1] | live[2] | live[3])) return;
    // only the live frequencies r are moved: the others are zero in the grid
    // direction (the pass-B FFT reads them as zeros) and unused in the degrid
    // direction (pass A' skips their rows)
    const cpx<R>* src = in + (size_t)t * A * B;
    for (int i = threadIdx.x; i < 64 * 64; i += THREADS) {
        const int a = a0 + i / 64, b = b0 + i % 64;
        if (a < A && b < B && live[(R_IN ? i / 64 : i % 64) / kTileR]) tile[i / 64][i % 64] = src[(size_t)a * B + b];
    }
    __syncthreads();
    cpx<R>* dst = out + (size_t)t * A * B;
    for (int i = threadIdx.x; i < 64 * 64; i += THREADS) {
        const int b = b0 + i / 64, a = a0 + i % 64;
        if (a < A && b < B && live[(R_IN ? i % 64 : i / 64) / kTileR])
            store_stream(dst + (size_t)b * A + a, tile[i % 64][i / 64]);
    }
}

// --------------------------------------------------------------- plan tables --
//
// Correction map corr[j][i] = h(x_i) h(y_j) h_z(z_ji) (Algorithm 5 step 5): h at
// the pixel columns comes from the host, h_z is evaluated here from the
// pointwise optimality formula h(z) = int Re g dnu / int |g|^2 dnu over
// Gauss-Legendre nodes nu_j, g(z, nu) = sum_a c_a(nu) exp(i 2 pi (s_a - nu) z),
// with the w-axis design's c (width Wz); hz_one: no correction along z (the
// original W-stacking corrects in x and y only, Algorithm 3 step 5).
static __global__ void k_corr_map(const double* __restrict__ hx, const double* __restrict__ cnodes,
                           const double* __restrict__ nun, const double* __restrict__ wn, int n_nu, int Wz,
                           int hz_one, DevParams P, double* __restrict__ corr64, float* __restrict__ corr32) {
    const int N = P.N, half = N / 2;
    const int i = blockIdx.x * blockDim.x + threadIdx.x, jrow = blockIdx.y;
    if (i >= N) return;
    if (hz_one) {
        const double v = hx[i] * hx[jrow];
        corr64[(size_t)jrow * N + i] = v;
        corr32[(size_t)jrow * N + i] = float(v);
        return;
    }
    const double l = double(i - half) * P.dl, m = double(jrow - half) * P.dl;
    const double r2 = l * l + m * m;
    const double z = (-r2 / (1.0 + sqrt(1.0 - r2))) / P.nscale + P.zshift;
    const int W = Wz;
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
