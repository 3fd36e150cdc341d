// C-ABI of the wsgrid library: plans, workspace layout and the launch sequences
// of Algorithm 5 (grid) and Algorithm 6 (degrid) on one gfx950 device.
//
// bin = k_bin_count, scan, k_bin_scatter, k_bin_local_sort (by touch class and
//       support start), k_tile_occupancy
// grid_visibilities:   bin -> k_grid_tiles (3-D scatter into the occupied tiles
//                      of the stack [t][r][s]) -> k_grid_fft_a (IFFT along s,
//                      crop, lines [t][r][q]) -> k_transpose ([t][q][r]) ->
//                      k_grid_fft_b (IFFT along r, crop, w-screen, sum over
//                      layers, correction) -> dirty [N][N]
// degrid_visibilities: bin; k_degrid_fft_b (correction, w-screen, pad, FFT
//                      along p, lines [t][q][r]) -> k_transpose ([t][r][q]) ->
//                      k_degrid_fft_a (pad, FFT along q, occupied tiles) ->
//                      k_degrid_tiles (3-D gather, one part per tile reached) ->
//                      k_degrid_finish (sum of parts, phase, fold) -> vis [M]
// Everything after binning runs once per layer pass when the workspace holds
// fewer layers than the plan has (k_degrid_finish once, at the end).  Batched
// calls put the channels' layers end to end on one virtual layer axis: one
// launch per stage covers all channels, except the pass-B FFTs, which run per
// channel segment (each has its own map).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/wsgrid.h"
#include "design.hpp"
#include "kernels.hpp"
#include "launch.hpp"

using namespace wsg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define WSG_HIP(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(WSG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kMaxBins = 1 << 25;   // bins over all channels (the bin tables take ~50 bytes per bin)

// Workspace of grid_visibilities_noalloc: one file-scope device array, which
// each device that loads the library holds (its own copy) until the process
// ends.  Host code never passes its name to a kernel (on the host the name is
// a stand-in, not a device address): the address comes from
// hipGetSymbolAddress, once per device, and only that pointer is used.
constexpr size_t kScratchBytes = size_t(WSG_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on device `dev` (which must be current),
// looked up on the first request for that device.
int scratch_on(int dev, void** ptr) {
    if (dev < 0 || dev >= kMaxDevices) return fail(WSG_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(WSG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return WSG_OK;
}

// per-thread stage timing (wsg_stage_timing / wsg_stage_times)
struct StageEvent {
    int stage;
    hipEvent_t a, b;
};
thread_local bool g_timing = false;
thread_local std::vector<StageEvent> g_events;

}  // namespace

namespace wsg {

StageMark::StageMark(hipStream_t s_, int st) : s(s_), stage(st) {
    static_assert(WSG_NSTAGES == 10, "stage ids are listed in wsgrid.h");
    if (g_timing && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, s);
}

StageMark::~StageMark() {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) == hipSuccess && hipEventRecord(b, s) == hipSuccess)
        g_events.push_back({stage, a, b});
    else
        (void)hipEventDestroy(a);
}

}  // namespace wsg

struct wsg_plan {
    PlanParams pp;
    KernelDesign kd;        // u, v (and w when same_design)
    KernelDesign kdz;       // w axis: its own least-misfit design, or the top hat
    bool same_design = true;
    int device = -1;
    int nbr = 0, nbs = 0, nbt = 0;
    double* poly64 = nullptr;
    float* poly32 = nullptr;
    double* polyz64 = nullptr;     // w-axis coefficients (same_design: poly64 again)
    float* polyz32 = nullptr;
    double* corr64 = nullptr;
    float* corr32 = nullptr;
    cpx<double>* tw64 = nullptr;
    cpx<float>* tw32 = nullptr;
    // the most recent call's workspace and stream (grid_last_skipped)
    mutable std::mutex last_mu;
    mutable const void* last_ws = nullptr;
    mutable void* last_stream = nullptr;
    // the binning kept by grid_prepare: its workspace, size, precision and
    // per-channel visibility counts (prep_ws null: none)
    mutable const void* prep_ws = nullptr;
    mutable size_t prep_bytes = 0;
    mutable int prep_prec = -1;
    mutable std::vector<int64_t> prep_M;

    int nbins() const { return nbr * nbs * nbt; }
};

namespace {

struct Layout {
    size_t stack, inter, inter2, rec, rec2, part, count, start, cursor, bsums, cls, occ, rows, chan, tpos, tlist, skipped,
        total;
    int nch, nbins, nscan;
    int last_layer;    // end of the last channel's layers on the virtual layer axis
    int pass_layers;   // virtual layers held in the stack and FFT buffers at a time (a multiple of kTileT, or all)
};

constexpr int kMaxChannels = 64;

// Channel table of a batched call, copied to the workspace by one tiny kernel:
// visibility offsets and first binning block of each channel.
struct ChanArgs {
    long long off[kMaxChannels + 1];
    int blk[kMaxChannels + 1];
};

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
size_t al2m(size_t x) { return (x + (size_t(2) << 20) - 1) & ~((size_t(2) << 20) - 1); }

// Workspace for nch channels (M visibilities in all) taken in passes of
// `tiles_per_pass` tile layers (kTileT virtual layers each).
Layout layout_of(const wsg_plan* p, wsg_prec prec, int64_t M, int tiles_per_pass, int nch = 1) {
    Layout L{};
    const size_t cs = prec == WSG_F32 ? sizeof(cpx<float>) : sizeof(cpx<double>);
    const size_t rs = prec == WSG_F32 ? sizeof(Rec<float>) : sizeof(Rec<double>);
    L.nch = nch;
    L.last_layer = (nch - 1) * p->nbt * kTileT + p->pp.n_layers();
    L.pass_layers = std::min(L.last_layer, std::max(1, std::min(tiles_per_pass, nch * p->nbt)) * kTileT);
    const size_t Np = size_t(p->pp.Nprime), N = size_t(p->pp.N), nl = size_t(L.pass_layers);
    L.nbins = nch * p->nbins();
    L.nscan = (L.nbins + 1023) / 1024;
    // the skipped counter sits at offset 0 whatever M and the precision
    size_t off = 0;
    L.skipped = off; off += 256;
    L.count = off;   off += al256(size_t(L.nbins) * 4);
    L.start = off;   off += al256(size_t(L.nbins + 1) * 4);
    L.cursor = off;  off += al256(size_t(L.nbins) * 4);
    L.bsums = off;   off += al256(size_t(L.nscan) * 4);
    L.cls = off;     off += al256(size_t(L.nbins) * 8 * 4);
    L.occ = off;     off += al256(size_t(L.nbins));
    L.rows = off;    off += al256(size_t(nch) * p->nbt * p->nbr);
    L.tpos = off;    off += al256(size_t(L.nbins + 1) * 4);
    L.tlist = off;   off += al256(size_t(L.nbins) * 4);
    L.chan = off;    off += al256(sizeof(long long) * (kMaxChannels + 1)) + al256(sizeof(int) * (kMaxChannels + 1));
    // the large buffers start on 2 MiB boundaries (their power-of-two line
    // strides then meet the memory channels the same way whatever precedes them)
    off = al2m(off);
    L.stack = off;   off += al2m(nl * Np * Np * cs);
    L.inter = off;   off += al2m(nl * N * Np * cs);
    L.inter2 = off;  off += al2m(nl * N * Np * cs);   // the transposed intermediate
    L.rec = off;     off += al256(size_t(M) * rs);
    L.rec2 = off;    off += al256(size_t(M) * rs);
    L.part = off;    off += al256(size_t(8) * size_t(M) * cs);   // degrid: per-tile parts
    L.total = off;
    return L;
}

DevParams dev_params(const wsg_plan* p) {
    DevParams P{};
    P.N = p->pp.N;
    P.Np = p->pp.Nprime;
    P.W = p->pp.W;
    P.Wz = p->pp.Wz;
    P.tclamp = p->pp.method == kOriginal ? 1 : 0;
    P.wshift = p->pp.w_shift;
    P.tphase = p->pp.t_phase;
    P.n_layers = p->pp.n_layers();
    P.t_lo = p->pp.t_lo;
    P.nbr = p->nbr;
    P.nbs = p->nbs;
    P.nbt = p->nbt;
    P.nch = 1;
    P.pl0 = 0;
    P.pln = p->pp.n_layers();
    P.umul = p->pp.l_max / p->pp.x0;
    P.nscale = p->pp.n_scale;
    P.zshift = p->pp.z_shift;
    P.wmax = p->pp.wmax;
    P.dl = p->pp.L / p->pp.N;
    return P;
}

template <typename T>
void fill(T* ptr, size_t n, T v, hipStream_t s) {
    if (n == 0) return;
    size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill<T>, dim3(unsigned(blocks)), dim3(256), 0, s, ptr, n, v);
}

void scan(const uint32_t* count, uint32_t* start, uint32_t* bsums, int n, hipStream_t s) {
    const int nb = (n + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(256), 0, s, count, start, n, bsums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, bsums, nb, start + n);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(256), 0, s, start, n, (const uint32_t*)bsums);
}

__global__ void k_set_chan(ChanArgs ca, int nch, long long* __restrict__ coff, int* __restrict__ cblk) {
    const int i = threadIdx.x;
    if (i <= nch) {
        coff[i] = ca.off[i];
        cblk[i] = ca.blk[i];
    }
}

// a: the input array, b: the output array; with M = 0 the visibility-sized
// one of them may be null (nothing is read from or written to it).  Mc: the
// nch channels' visibility counts (host); *M receives their sum.
int check_call(const wsg_plan* plan, wsg_prec prec, int nch, const int64_t* Mc, int64_t* M, const double* uvw,
               const void* a, bool a_empty_ok, const void* b, bool b_empty_ok, void* ws, size_t ws_bytes,
               Layout* L, bool uvw_needed = true) {
    if (!plan) return fail(WSG_EINVAL, "null plan");
    if (prec != WSG_F32 && prec != WSG_F64) return fail(WSG_EINVAL, "prec must be WSG_F32 or WSG_F64");
    if (nch < 1 || nch > kMaxChannels) return fail(WSG_EINVAL, "channels must be in [1, 64]");
    if (!Mc) return fail(WSG_EINVAL, "null visibility counts");
    int64_t tot = 0;
    for (int c = 0; c < nch; ++c) {
        if (Mc[c] < 0 || Mc[c] > 0x7fffffffLL) return fail(WSG_EINVAL, "M must be in [0, 2^31)");
        tot += Mc[c];
    }
    if (tot > 0x7fffffffLL) return fail(WSG_EINVAL, "total M must be below 2^31");
    *M = tot;
    if ((long long)nch * plan->nbins() > kMaxBins) return fail(WSG_EINVAL, "too many tiles over the channels");
    if (uvw_needed && tot > 0 && !uvw) return fail(WSG_EINVAL, "null uvw pointer");
    if (!a && (tot > 0 || !a_empty_ok)) return fail(WSG_EINVAL, "null visibility/image pointer");
    if (!b && (tot > 0 || !b_empty_ok)) return fail(WSG_EINVAL, "null output pointer");
    if (!ws) return fail(WSG_EINVAL, "null workspace");
    // as many tile layers per pass as the workspace holds
    int tiles = nch * plan->nbt;
    *L = layout_of(plan, prec, tot, tiles, nch);
    while (tiles > 1 && ws_bytes < L->total) *L = layout_of(plan, prec, tot, --tiles, nch);
    if (ws_bytes < L->total)
        return fail(WSG_EWORKSPACE, "workspace too small: need at least " + std::to_string(L->total) + " bytes");
    int dev = -1;
    WSG_HIP(hipGetDevice(&dev));
    if (dev != plan->device) return fail(WSG_EINVAL, "plan was created on another device");
    return WSG_OK;
}

// Binning (Alg. 5 step 2, Alg. 6 steps 4-5 preprocessing; Sec. 5.4 fold):
// records binned by tile and sorted by touch class into `rec`, the class
// starts, the occupancy marks and the ordered tile list.  Grid records carry the
// phase-rotated visibility, degrid records the phase and the visibility index.
template <typename R>
void bin_stage(const wsg_plan* plan, bool grid, int stage, const int64_t* Mc, const double* uvw, const void* in,
               void* ws, const Layout& L, hipStream_t s) {
    DevParams P = dev_params(plan);
    P.nch = L.nch;
    char* w = static_cast<char*>(ws);
    auto* rec_bin = reinterpret_cast<Rec<R>*>(w + L.rec2);   // binned, unordered within a bin
    auto* rec = reinterpret_cast<Rec<R>*>(w + L.rec);        // binned and sorted within each bin
    auto* count = reinterpret_cast<uint32_t*>(w + L.count);
    auto* start = reinterpret_cast<uint32_t*>(w + L.start);
    auto* cursor = reinterpret_cast<uint32_t*>(w + L.cursor);
    auto* bsums = reinterpret_cast<uint32_t*>(w + L.bsums);
    auto* cls = reinterpret_cast<uint32_t*>(w + L.cls);
    auto* occ = reinterpret_cast<uint8_t*>(w + L.occ);
    auto* rows = reinterpret_cast<uint8_t*>(w + L.rows);
    auto* tpos = reinterpret_cast<uint32_t*>(w + L.tpos);
    auto* tlist = reinterpret_cast<uint32_t*>(w + L.tlist);
    auto* coff = reinterpret_cast<long long*>(w + L.chan);
    auto* cblk = reinterpret_cast<int*>(w + L.chan + al256(sizeof(long long) * (kMaxChannels + 1)));
    auto* skipped = reinterpret_cast<uint32_t*>(w + L.skipped);

    // channel table: visibility offsets and binning blocks (one channel per block)
    ChanArgs ca{};
    for (int c = 0; c < L.nch; ++c) {
        ca.off[c + 1] = ca.off[c] + Mc[c];
        ca.blk[c + 1] = ca.blk[c] + int((Mc[c] + kAggChunk - 1) / kAggChunk);
    }
    const unsigned vblocks = unsigned(ca.blk[L.nch]);
    {
        StageMark mark(s, stage);
        hipLaunchKernelGGL(k_set_chan, dim3(1), dim3(128), 0, s, ca, L.nch, coff, cblk);
        fill<uint32_t>(count, size_t(L.nbins), 0u, s);
        fill<uint32_t>(cursor, size_t(L.nbins), 0u, s);
        fill<uint32_t>(skipped, 1, 0u, s);
        if (vblocks > 0)
            hipLaunchKernelGGL(k_bin_count, dim3(vblocks), dim3(kAggThreads), 0, s, uvw, (const long long*)coff,
                               (const int*)cblk, P, count, skipped);
        scan(count, start, bsums, L.nbins, s);
        if (vblocks > 0) {
            if (grid)
                hipLaunchKernelGGL((k_bin_scatter<R, true>), dim3(vblocks), dim3(kAggThreads), 0, s, uvw,
                                   static_cast<const cpx<R>*>(in), (const long long*)coff, (const int*)cblk, P,
                                   (const uint32_t*)start, cursor, rec_bin);
            else
                hipLaunchKernelGGL((k_bin_scatter<R, false>), dim3(vblocks), dim3(kAggThreads), 0, s, uvw,
                                   (const cpx<R>*)nullptr, (const long long*)coff, (const int*)cblk, P,
                                   (const uint32_t*)start, cursor, rec_bin);
            hipLaunchKernelGGL(k_bin_local_sort<R>, dim3(L.nbins), dim3(256), 0, s, (const Rec<R>*)rec_bin, rec,
                               (const uint32_t*)start, cls, P);
        }
        fill<uint8_t>(rows, size_t(L.nch) * P.nbt * P.nbr, uint8_t(0), s);
        // occupancy marks, then the ordered list of occupied tiles (the bin
        // counts are no longer needed: they take the 32-bit marks for the scan)
        hipLaunchKernelGGL(k_tile_occupancy, dim3((L.nbins + 255) / 256), dim3(256), 0, s, (const uint32_t*)start,
                           (const uint32_t*)cls, P, occ, rows, count);
        scan(count, tpos, bsums, L.nbins, s);
        hipLaunchKernelGGL(k_tile_list, dim3((L.nbins + 255) / 256), dim3(256), 0, s, (const uint8_t*)occ,
                           (const uint32_t*)tpos, L.nbins, tlist);
    }
}

// Layer passes over the binned records `rec` (grid: scatter, transforms,
// w-screen and correction into `out`; degrid: transforms and gather from `in`,
// then the per-visibility finish into `out`).
template <typename R>
int pass_stage(const wsg_plan* plan, bool grid, const Rec<R>* rec, int64_t M, const void* in, void* out, void* ws,
               const Layout& L, hipStream_t s, const cpx<R>* prep_vis = nullptr) {
    DevParams P = dev_params(plan);
    P.nch = L.nch;
    char* w = static_cast<char*>(ws);
    auto* stack = reinterpret_cast<cpx<R>*>(w + L.stack);
    auto* inter = reinterpret_cast<cpx<R>*>(w + L.inter);
    auto* inter2 = reinterpret_cast<cpx<R>*>(w + L.inter2);
    auto* start = reinterpret_cast<uint32_t*>(w + L.start);
    auto* cls = reinterpret_cast<uint32_t*>(w + L.cls);
    auto* occ = reinterpret_cast<uint8_t*>(w + L.occ);
    auto* rows = reinterpret_cast<uint8_t*>(w + L.rows);
    auto* tpos = reinterpret_cast<uint32_t*>(w + L.tpos);
    auto* tlist = reinterpret_cast<uint32_t*>(w + L.tlist);
    const bool f64 = sizeof(R) == 8;
    const R* coef = f64 ? reinterpret_cast<const R*>(plan->poly64) : reinterpret_cast<const R*>(plan->poly32);
    const R* coefz = f64 ? reinterpret_cast<const R*>(plan->polyz64) : reinterpret_cast<const R*>(plan->polyz32);
    const R* corr = f64 ? reinterpret_cast<const R*>(plan->corr64) : reinterpret_cast<const R*>(plan->corr32);
    const cpx<R>* tw = f64 ? reinterpret_cast<const cpx<R>*>(plan->tw64) : reinterpret_cast<const cpx<R>*>(plan->tw32);
    // Layer passes over the virtual layer axis (channel c's layers start at
    // c nbt kTileT): the stack and FFT buffers hold L.pass_layers layers at a
    // time.  Grid: each pass scatters into its tiles and transforms them; a
    // channel's first layers write its map, later ones add to it.  Degrid: each
    // pass transforms its layers and gathers from its tiles; every (visibility,
    // tile) part belongs to exactly one pass, and k_degrid_finish sums them at
    // the end.  Virtual layers past a channel's n_layers are padding, skipped.
    const int per_layer = P.nbs * P.nbr;
    auto* part = reinterpret_cast<cpx<R>*>(w + L.part);
    for (int pl0 = 0; pl0 < L.last_layer; pl0 += L.pass_layers) {
        DevParams Q = P;
        Q.pl0 = pl0;
        Q.pln = std::min(L.pass_layers, L.last_layer - pl0);
        const int nblocks = ((Q.pln + kTileT - 1) / kTileT) * per_layer;
        if (grid) {
            {
                StageMark mark(s, 1);
                launch_tiles<R>(true, P.W, P.Wz, plan->same_design, nblocks, rec, start, cls, tlist, tpos, Q, coef,
                                coefz, prep_vis, stack, nullptr, 0, s);
            }
            launch_fft<R>(true, Q, occ, rows, stack, inter, inter2, tw, corr, nullptr,
                          static_cast<R*>(out), s);
        } else {
            launch_fft<R>(false, Q, occ, rows, stack, inter, inter2, tw, corr,
                          static_cast<const R*>(in), nullptr, s);
            if (M > 0) {
                StageMark mark(s, 7);
                launch_tiles<R>(false, P.W, P.Wz, plan->same_design, nblocks, rec, start, cls, tlist, tpos, Q, coef,
                                coefz, nullptr, stack, part, size_t(M), s);
            }
        }
    }
    if (!grid) {
        fill<R>(static_cast<R*>(out), size_t(2 * M), R(0), s);     // skipped visibilities stay zero
        StageMark mark(s, 7);
        if (M > 0)
            hipLaunchKernelGGL(k_degrid_finish<R>, dim3(unsigned((M + 255) / 256)), dim3(256), 0, s,
                               (const Rec<R>*)rec, (const uint32_t*)(start + L.nbins), (const cpx<R>*)part,
                               size_t(M), P.W, P.Wz, static_cast<cpx<R>*>(out));
    }
    WSG_HIP(hipGetLastError());
    return WSG_OK;
}

template <typename R>
int run(const wsg_plan* plan, bool grid, const int64_t* Mc, int64_t M, const double* uvw, const void* in, void* out,
        void* ws, const Layout& L, hipStream_t s) {
    bin_stage<R>(plan, grid, grid ? 0 : 4, Mc, uvw, grid ? in : nullptr, ws, L, s);
    return pass_stage<R>(plan, grid, reinterpret_cast<const Rec<R>*>(static_cast<char*>(ws) + L.rec), M, in, out,
                         ws, L, s);
}

// Directions on a shared binning (the degridding records): degrid as usual;
// grid with the scatter taking each record's value from the visibilities.
template <typename R>
int run_prepared(const wsg_plan* plan, bool grid, int64_t M, const void* in, void* out, void* ws, const Layout& L,
                 hipStream_t s) {
    char* w = static_cast<char*>(ws);
    const auto* rec = reinterpret_cast<const Rec<R>*>(w + L.rec);
    if (!grid) return pass_stage<R>(plan, false, rec, M, in, out, ws, L, s);
    return pass_stage<R>(plan, true, rec, M, in, out, ws, L, s, M > 0 ? static_cast<const cpx<R>*>(in) : nullptr);
}

template <typename T>
int upload(T** dst, const T* src, size_t n) {
    WSG_HIP(hipMalloc(reinterpret_cast<void**>(dst), n * sizeof(T)));
    WSG_HIP(hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice));
    return WSG_OK;
}

int build_tables(wsg_plan* p) {
    const PlanParams& pp = p->pp;
    const KernelDesign& kd = p->kd;
    const KernelDesign& kz = p->same_design ? p->kd : p->kdz;
    const int N = pp.N, Np = pp.Nprime;
    for (const KernelDesign* d : {&kd, &kz})
        if (d->degree != KernelDegree<double>::value || d->degree_lo != KernelDegree<float>::value)
            return fail(WSG_EINVAL, "kernel polynomial degree mismatch between design and device code");
    std::vector<double> poly64(kd.poly);
    std::vector<float> poly32(kd.poly_lo.begin(), kd.poly_lo.end());
    int rc;
    if ((rc = upload(&p->poly64, poly64.data(), poly64.size()))) return rc;
    if ((rc = upload(&p->poly32, poly32.data(), poly32.size()))) return rc;
    if (p->same_design) {
        p->polyz64 = p->poly64;
        p->polyz32 = p->poly32;
    } else {
        std::vector<double> pz64(kz.poly);
        std::vector<float> pz32(kz.poly_lo.begin(), kz.poly_lo.end());
        if ((rc = upload(&p->polyz64, pz64.data(), pz64.size()))) return rc;
        if ((rc = upload(&p->polyz32, pz32.data(), pz32.size()))) return rc;
    }
    std::vector<cpx<double>> tw64(Np);
    std::vector<cpx<float>> tw32(Np);
    const double two_pi = 6.283185307179586476925286766559;
    for (int k = 0; k < Np; ++k) {
        double a = two_pi * double(k) / double(Np);
        tw64[k] = {std::cos(a), std::sin(a)};
        tw32[k] = {float(tw64[k].x), float(tw64[k].y)};
    }
    if ((rc = upload(&p->tw64, tw64.data(), tw64.size()))) return rc;
    if ((rc = upload(&p->tw32, tw32.data(), tw32.size()))) return rc;

    std::vector<double> hx(N);
    for (int i = 0; i < N; ++i) hx[i] = kd.h_at(double(i - N / 2) / double(Np));
    double *d_hx = nullptr, *d_c = nullptr, *d_nu = nullptr, *d_wn = nullptr;
    if ((rc = upload(&d_hx, hx.data(), hx.size()))) return rc;
    // h_z from the w-axis design (the top hat of the original method: none)
    const bool hz_one = pp.method == kOriginal;
    const KernelDesign& kn = hz_one ? kd : kz;
    if ((rc = upload(&d_c, kn.c_nodes.data(), kn.c_nodes.size()))) return rc;
    if ((rc = upload(&d_nu, kn.nun.data(), kn.nun.size()))) return rc;
    if ((rc = upload(&d_wn, kn.wn.data(), kn.wn.size()))) return rc;
    WSG_HIP(hipMalloc(reinterpret_cast<void**>(&p->corr64), size_t(N) * N * sizeof(double)));
    WSG_HIP(hipMalloc(reinterpret_cast<void**>(&p->corr32), size_t(N) * N * sizeof(float)));
    DevParams P = dev_params(p);
    hipLaunchKernelGGL(k_corr_map, dim3((N + 255) / 256, N), dim3(256), 0, 0, (const double*)d_hx,
                       (const double*)d_c, (const double*)d_nu, (const double*)d_wn, int(kn.nun.size()), kn.W,
                       hz_one ? 1 : 0, P, p->corr64, p->corr32);
    WSG_HIP(hipGetLastError());
    WSG_HIP(hipDeviceSynchronize());
    WSG_HIP(hipFree(d_hx));
    WSG_HIP(hipFree(d_c));
    WSG_HIP(hipFree(d_nu));
    WSG_HIP(hipFree(d_wn));
    return WSG_OK;
}

// Every call records its workspace and stream; a call that is not a
// prepared one overwrites the binning grid_prepare left in that workspace.
void remember_call(const wsg_plan* p, const void* ws, void* stream, bool keeps_binning = false) {
    std::lock_guard<std::mutex> g(p->last_mu);
    p->last_ws = ws;
    p->last_stream = stream;
    if (!keeps_binning && p->prep_ws == ws) p->prep_ws = nullptr;
}

void free_tables(wsg_plan* p) {
    if (p->polyz64 != p->poly64 && p->polyz64) (void)hipFree(p->polyz64);
    if (p->polyz32 != p->poly32 && p->polyz32) (void)hipFree(p->polyz32);
    void* ptrs[] = {p->poly64, p->poly32, p->corr64, p->corr32, p->tw64, p->tw32};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
}

}  // namespace

extern "C" {

const char* grid_last_error(void) { return g_err.c_str(); }

void wsg_stage_timing(int enable) { g_timing = enable != 0; }

int wsg_stage_times(double* ms, int* launches, int n) {
    std::vector<double> acc(WSG_NSTAGES, 0.0);
    std::vector<int> cnt(WSG_NSTAGES, 0);
    int rc = WSG_OK;
    for (const StageEvent& e : g_events) {
        float t = 0.f;
        if (rc == WSG_OK) {
            hipError_t err = hipEventSynchronize(e.b);
            if (err == hipSuccess) err = hipEventElapsedTime(&t, e.a, e.b);
            if (err != hipSuccess) rc = fail(WSG_EHIP, std::string("stage timing: ") + hipGetErrorString(err));
        }
        if (e.stage >= 0 && e.stage < WSG_NSTAGES) {
            acc[e.stage] += t;
            cnt[e.stage] += 1;
        }
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    g_events.clear();
    if (rc != WSG_OK) return rc;
    for (int i = 0; i < n && i < WSG_NSTAGES; ++i) {
        if (ms) ms[i] = acc[i];
        if (launches) launches[i] = cnt[i];
    }
    return WSG_NSTAGES;
}

int wsg_plan_params(int N, double L, int W, double x0, double wmax, int z_offset, int* Nprime, int* t_lo,
                    int* t_hi, double* n0, double* n_scale) {
    PlanParams pp;
    std::string e = make_plan_params(N, L, W, x0, wmax, &pp, z_offset != 0);
    if (!e.empty()) return fail(WSG_EINVAL, e);
    if (Nprime) *Nprime = pp.Nprime;
    if (t_lo) *t_lo = pp.t_lo;
    if (t_hi) *t_hi = pp.t_hi;
    if (n0) *n0 = pp.n0;
    if (n_scale) *n_scale = pp.n_scale;
    return WSG_OK;
}

int wsg_design_eval(int W, double x0, int n_nu, const double* nu, double* c_out, int n_x, const double* x,
                    double* h_out, double* E_out) {
    try {
        if (n_nu < 0 || n_x < 0) return fail(WSG_EINVAL, "negative count");
        if ((n_nu > 0 && (!nu || !c_out)) || (n_x > 0 && (!x || !h_out))) return fail(WSG_EINVAL, "null pointer");
        KernelDesign kd = design_kernel(W, x0);
        for (int k = 0; k < n_nu; ++k) {
            if (!(nu[k] >= -0.5 && nu[k] <= 0.5)) return fail(WSG_EINVAL, "nu outside [-1/2, 1/2]");
            for (int a = 0; a < W; ++a) c_out[size_t(k) * W + a] = kd.c_poly(a, nu[k]);
        }
        for (int k = 0; k < n_x; ++k) {
            if (!(std::fabs(x[k]) <= 0.5)) return fail(WSG_EINVAL, "|x| > 1/2");
            h_out[k] = kd.h_at(x[k]);
        }
        if (E_out) *E_out = kd.E;
        return WSG_OK;
    } catch (const std::exception& e) {
        return fail(WSG_EINVAL, e.what());
    }
}

wsg_plan* grid_create(int N, double L, int W, double x0, double wmax) {
    return grid_create_axes(N, L, W, x0, W, x0, wmax, WSG_IMPROVED, 0);
}

wsg_plan* grid_create_variant(int N, double L, int W, double x0, double wmax, int z_offset) {
    return grid_create_axes(N, L, W, x0, W, x0, wmax, z_offset ? WSG_IMPROVED : WSG_IMPROVED_NO_OFFSET, 0);
}

wsg_plan* grid_create_axes(int N, double L, int W, double x0, int Wz, double z0, double wmax, wsg_method method,
                           int n_bins) {
    wsg_plan* p = nullptr;
    try {
        PlanParams pp;
        std::string e = make_plan_params_ext(N, L, W, x0, Wz, z0, wmax, int(method), n_bins, &pp);
        if (!e.empty()) {
            fail(WSG_EINVAL, e);
            return nullptr;
        }
        if (!fft_supported(pp.Nprime)) {
            fail(WSG_EINVAL, "N / (2 x0) must be 2^a or 3 2^a in [64, 8192]");
            return nullptr;
        }
        const bool same = method != WSG_ORIGINAL && Wz == W && z0 == x0;
        if (!tiles_supported(W, Wz, same)) {
            fail(WSG_EINVAL, "this pair of widths (W, W_z) is not compiled: W_z = W, or W = 7 with W_z <= 7, "
                             "or W_z = 1 with W in 3 .. 8");
            return nullptr;
        }
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess) {
            fail(WSG_EHIP, "no HIP device");
            return nullptr;
        }
        const int Np = pp.Nprime;
        p = new wsg_plan();
        p->pp = pp;
        p->device = dev;
        p->same_design = same;
        p->nbr = Np / kTileR;
        p->nbs = Np / kTileS;
        p->nbt = (pp.n_layers() + kTileT - 1) / kTileT;
        if ((long long)p->nbr * p->nbs * p->nbt > kMaxBins) {
            fail(WSG_EINVAL, "too many tiles: reduce N / (2 x0) or wmax");
            delete p;
            return nullptr;
        }
        p->kd = design_kernel(W, x0);
        if (!same) p->kdz = method == WSG_ORIGINAL ? top_hat_design() : design_kernel(Wz, z0);
        void* sp = nullptr;
        if (scratch_on(dev, &sp) != WSG_OK) {     // set-up: the no-alloc call's workspace on this device
            delete p;
            return nullptr;
        }
        if (build_tables(p) != WSG_OK) {
            free_tables(p);
            delete p;
            return nullptr;
        }
        return p;
    } catch (const std::exception& ex) {
        fail(WSG_ENOMEM, ex.what());
        if (p) {
            free_tables(p);
            delete p;
        }
        return nullptr;
    }
}

int grid_plan_axes(const wsg_plan* plan, int* W, double* x0, int* Wz, double* z0, int* method, int* n_bins,
                   double* E_z) {
    if (!plan) return fail(WSG_EINVAL, "null plan");
    const PlanParams& pp = plan->pp;
    if (W) *W = pp.W;
    if (x0) *x0 = pp.x0;
    if (Wz) *Wz = pp.Wz;
    if (z0) *z0 = pp.z0;
    if (method) *method = pp.method;
    if (n_bins) *n_bins = pp.n_bins;
    if (E_z) *E_z = plan->same_design ? plan->kd.E : plan->kdz.E;
    return WSG_OK;
}

int wsg_plan_params_axes(int N, double L, int W, double x0, int Wz, double z0, double wmax, wsg_method method,
                         int n_bins, int* Nprime, int* t_lo, int* t_hi, double* n0, double* n_scale) {
    PlanParams pp;
    std::string e = make_plan_params_ext(N, L, W, x0, Wz, z0, wmax, int(method), n_bins, &pp);
    if (!e.empty()) return fail(WSG_EINVAL, e);
    if (Nprime) *Nprime = pp.Nprime;
    if (t_lo) *t_lo = pp.t_lo;
    if (t_hi) *t_hi = pp.t_hi;
    if (n0) *n0 = pp.n0;
    if (n_scale) *n_scale = pp.n_scale;
    return WSG_OK;
}

void grid_destroy(wsg_plan* plan) {
    if (!plan) return;
    free_tables(plan);
    delete plan;
}

int grid_plan_info(const wsg_plan* plan, int* Nprime, int* n_layers, int* t_lo, double* n0, double* n_scale,
                   double* E) {
    if (!plan) return fail(WSG_EINVAL, "null plan");
    if (Nprime) *Nprime = plan->pp.Nprime;
    if (t_lo) *t_lo = plan->pp.t_lo;
    if (n_layers) *n_layers = plan->pp.n_layers();
    if (n0) *n0 = plan->pp.n0;
    if (n_scale) *n_scale = plan->pp.n_scale;
    if (E) *E = plan->kd.E;
    return WSG_OK;
}

size_t grid_workspace_bytes(const wsg_plan* plan, wsg_prec prec, int64_t M) {
    if (!plan || (prec != WSG_F32 && prec != WSG_F64) || M < 0 || M > 0x7fffffffLL) return 0;
    return layout_of(plan, prec, M, plan->nbt).total;
}

size_t grid_workspace_bytes_min(const wsg_plan* plan, wsg_prec prec, int64_t M) {
    if (!plan || (prec != WSG_F32 && prec != WSG_F64) || M < 0 || M > 0x7fffffffLL) return 0;
    return layout_of(plan, prec, M, 1).total;
}

int grid_layers_per_pass(const wsg_plan* plan, wsg_prec prec, int nch, int64_t M, size_t ws_bytes) {
    if (!plan || (prec != WSG_F32 && prec != WSG_F64) || M < 0 || M > 0x7fffffffLL || nch < 1 ||
        nch > kMaxChannels)
        return fail(WSG_EINVAL, "bad argument");
    int tiles = nch * plan->nbt;
    Layout L = layout_of(plan, prec, M, tiles, nch);
    while (tiles > 1 && ws_bytes < L.total) L = layout_of(plan, prec, M, --tiles, nch);
    if (ws_bytes < L.total) return fail(WSG_EWORKSPACE, "workspace too small");
    return L.pass_layers;
}

size_t grid_workspace_bytes_batch(const wsg_plan* plan, wsg_prec prec, int nch, int64_t M, int min_passes) {
    if (!plan || (prec != WSG_F32 && prec != WSG_F64) || M < 0 || M > 0x7fffffffLL || nch < 1 ||
        nch > kMaxChannels)
        return 0;
    return layout_of(plan, prec, M, min_passes ? 1 : nch * plan->nbt, nch).total;
}

int grid_visibilities_batch(const wsg_plan* plan, wsg_prec prec, int nch, const int64_t* M, const double* uvw,
                            const void* vis, void* dirty, void* ws, size_t ws_bytes, void* stream) {
    Layout L;
    int64_t tot = 0;
    int rc = check_call(plan, prec, nch, M, &tot, uvw, vis, true, dirty, false, ws, ws_bytes, &L);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    remember_call(plan, ws, stream);
    return prec == WSG_F32 ? run<float>(plan, true, M, tot, uvw, vis, dirty, ws, L, s)
                           : run<double>(plan, true, M, tot, uvw, vis, dirty, ws, L, s);
}

int degrid_visibilities_batch(const wsg_plan* plan, wsg_prec prec, int nch, const int64_t* M, const double* uvw,
                              const void* image, void* vis, void* ws, size_t ws_bytes, void* stream) {
    Layout L;
    int64_t tot = 0;
    int rc = check_call(plan, prec, nch, M, &tot, uvw, image, false, vis, true, ws, ws_bytes, &L);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    remember_call(plan, ws, stream);
    return prec == WSG_F32 ? run<float>(plan, false, M, tot, uvw, image, vis, ws, L, s)
                           : run<double>(plan, false, M, tot, uvw, image, vis, ws, L, s);
}

int grid_prepare(const wsg_plan* plan, wsg_prec prec, int nch, const int64_t* M, const double* uvw, void* ws,
                 size_t ws_bytes, void* stream) {
    Layout L;
    int64_t tot = 0;
    int rc = check_call(plan, prec, nch, M, &tot, uvw, uvw, true, ws, true, ws, ws_bytes, &L);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    remember_call(plan, ws, stream);
    if (prec == WSG_F32)
        bin_stage<float>(plan, false, 4, M, uvw, nullptr, ws, L, s);
    else
        bin_stage<double>(plan, false, 4, M, uvw, nullptr, ws, L, s);
    WSG_HIP(hipGetLastError());
    std::lock_guard<std::mutex> g(plan->last_mu);
    plan->prep_ws = ws;
    plan->prep_bytes = ws_bytes;
    plan->prep_prec = int(prec);
    plan->prep_M.assign(M, M + nch);
    return WSG_OK;
}

}  // extern "C"

namespace {

// A call on the binning grid_prepare left in `ws`: checks that it is there
// (same workspace, size and precision) and runs one direction on it.
int call_prepared(bool grid, const wsg_plan* plan, wsg_prec prec, const void* in, void* out, void* ws,
                  size_t ws_bytes, void* stream) {
    if (!plan) return fail(WSG_EINVAL, "null plan");
    std::vector<int64_t> Mc;
    {
        std::lock_guard<std::mutex> g(plan->last_mu);
        if (!ws || plan->prep_ws != ws || plan->prep_bytes != ws_bytes || plan->prep_prec != int(prec))
            return fail(WSG_EINVAL, "no binning of this plan and precision in this workspace: call grid_prepare "
                                    "first (any other call on the workspace replaces it)");
        Mc = plan->prep_M;
    }
    Layout L;
    int64_t tot = 0;
    int rc = grid ? check_call(plan, prec, int(Mc.size()), Mc.data(), &tot, nullptr, in, true, out, false, ws,
                               ws_bytes, &L, false)
                  : check_call(plan, prec, int(Mc.size()), Mc.data(), &tot, nullptr, in, false, out, true, ws,
                               ws_bytes, &L, false);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    remember_call(plan, ws, stream, true);
    return prec == WSG_F32 ? run_prepared<float>(plan, grid, tot, in, out, ws, L, s)
                           : run_prepared<double>(plan, grid, tot, in, out, ws, L, s);
}

}  // namespace

extern "C" {

int grid_visibilities_prepared(const wsg_plan* plan, wsg_prec prec, const void* vis, void* dirty, void* ws,
                               size_t ws_bytes, void* stream) {
    return call_prepared(true, plan, prec, vis, dirty, ws, ws_bytes, stream);
}

int degrid_visibilities_prepared(const wsg_plan* plan, wsg_prec prec, const void* image, void* vis, void* ws,
                                 size_t ws_bytes, void* stream) {
    return call_prepared(false, plan, prec, image, vis, ws, ws_bytes, stream);
}

}  // extern "C"

namespace {

// Runs of consecutive channels with one plan: [first channel, end channel).
int plan_runs(int nch, const wsg_plan* const* plans, std::vector<std::pair<int, int>>* runs) {
    if (nch < 1 || nch > kMaxChannels) return fail(WSG_EINVAL, "channels must be in [1, 64]");
    if (!plans) return fail(WSG_EINVAL, "null plan list");
    runs->clear();
    for (int c = 0; c < nch; ++c) {
        if (!plans[c]) return fail(WSG_EINVAL, "null plan for a channel");
        if (c > 0 && plans[c] == plans[c - 1]) {
            runs->back().second = c + 1;
            continue;
        }
        for (const auto& r : *runs)
            if (plans[r.first] == plans[c]) return fail(WSG_EINVAL, "channels sharing a plan must be consecutive");
        runs->push_back({c, c + 1});
    }
    return WSG_OK;
}

// One batched call per run; `a` advances over the inputs, `b` over the outputs
// (visibility-sized or map-sized by direction).
int run_multi(bool grid, int nch, const wsg_plan* const* plans, wsg_prec prec, const int64_t* M, const double* uvw,
              const void* in, void* out, void* ws, size_t ws_bytes, void* stream) {
    std::vector<std::pair<int, int>> runs;
    int rc = plan_runs(nch, plans, &runs);
    if (rc != WSG_OK) return rc;
    if (!M) return fail(WSG_EINVAL, "null visibility counts");
    const size_t cs = prec == WSG_F64 ? 16 : 8, rs = prec == WSG_F64 ? 8 : 4;
    int64_t voff = 0;
    size_t moff = 0;
    for (const auto& r : runs) {
        const wsg_plan* p = plans[r.first];
        const int n = r.second - r.first;
        int64_t mrun = 0;
        for (int c = r.first; c < r.second; ++c) mrun += M[c] < 0 ? 0 : M[c];
        const size_t map = size_t(p->pp.N) * size_t(p->pp.N) * size_t(n);
        const double* u = uvw ? uvw + 3 * voff : nullptr;
        if (grid) {
            const void* v = in ? static_cast<const char*>(in) + size_t(voff) * cs : nullptr;
            void* d = out ? static_cast<char*>(out) + moff * rs : nullptr;
            rc = grid_visibilities_batch(p, prec, n, M + r.first, u, v, d, ws, ws_bytes, stream);
        } else {
            const void* im = in ? static_cast<const char*>(in) + moff * rs : nullptr;
            void* v = out ? static_cast<char*>(out) + size_t(voff) * cs : nullptr;
            rc = degrid_visibilities_batch(p, prec, n, M + r.first, u, im, v, ws, ws_bytes, stream);
        }
        if (rc != WSG_OK) return rc;
        voff += mrun;
        moff += map;
    }
    return WSG_OK;
}

}  // namespace

extern "C" {

int grid_visibilities_multi(int nch, const wsg_plan* const* plans, wsg_prec prec, const int64_t* M,
                            const double* uvw, const void* vis, void* dirty, void* ws, size_t ws_bytes,
                            void* stream) {
    return run_multi(true, nch, plans, prec, M, uvw, vis, dirty, ws, ws_bytes, stream);
}

int degrid_visibilities_multi(int nch, const wsg_plan* const* plans, wsg_prec prec, const int64_t* M,
                              const double* uvw, const void* image, void* vis, void* ws, size_t ws_bytes,
                              void* stream) {
    return run_multi(false, nch, plans, prec, M, uvw, image, vis, ws, ws_bytes, stream);
}

size_t grid_workspace_bytes_multi(int nch, const wsg_plan* const* plans, wsg_prec prec, const int64_t* M,
                                  int min_passes) {
    std::vector<std::pair<int, int>> runs;
    if (plan_runs(nch, plans, &runs) != WSG_OK || !M) return 0;
    size_t best = 0;
    for (const auto& r : runs) {
        int64_t mrun = 0;
        for (int c = r.first; c < r.second; ++c) mrun += M[c];
        const size_t b = grid_workspace_bytes_batch(plans[r.first], prec, r.second - r.first, mrun, min_passes);
        if (b == 0) return 0;
        best = std::max(best, b);
    }
    return best;
}

int grid_visibilities(const wsg_plan* plan, wsg_prec prec, int64_t M, const double* uvw, const void* vis, void* dirty,
                      void* ws, size_t ws_bytes, void* stream) {
    return grid_visibilities_batch(plan, prec, 1, &M, uvw, vis, dirty, ws, ws_bytes, stream);
}

int grid_visibilities_noalloc(const wsg_plan* plan, wsg_prec prec, int64_t M, const double* uvw, const void* vis,
                              void* dirty, void* stream) {
    if (!plan) return fail(WSG_EINVAL, "null plan");
    if (prec != WSG_F32 && prec != WSG_F64) return fail(WSG_EINVAL, "prec must be WSG_F32 or WSG_F64");
    if (M < 0 || M > 0x7fffffffLL) return fail(WSG_EINVAL, "M must be in [0, 2^31)");
    const size_t need = grid_workspace_bytes_min(plan, prec, M);
    if (need > kScratchBytes)
        return fail(WSG_EWORKSPACE, "grid_visibilities_noalloc: the call needs " + std::to_string(need) +
                                        " bytes of workspace, the library's scratch holds " +
                                        std::to_string(kScratchBytes));
    void* ws = nullptr;
    const int rc = scratch_on(plan->device, &ws);
    if (rc != WSG_OK) return rc;
    return grid_visibilities_batch(plan, prec, 1, &M, uvw, vis, dirty, ws, kScratchBytes, stream);
}

int degrid_visibilities(const wsg_plan* plan, wsg_prec prec, int64_t M, const double* uvw, const void* image, void* vis,
                        void* ws, size_t ws_bytes, void* stream) {
    return degrid_visibilities_batch(plan, prec, 1, &M, uvw, image, vis, ws, ws_bytes, stream);
}

int64_t grid_last_skipped(const wsg_plan* plan) {
    if (!plan) return fail(WSG_EINVAL, "null plan");
    const void* ws;
    void* stream;
    {
        std::lock_guard<std::mutex> g(plan->last_mu);
        ws = plan->last_ws;
        stream = plan->last_stream;
    }
    if (!ws) return fail(WSG_EINVAL, "the plan has made no grid/degrid call");
    return grid_skipped(plan, ws, stream);
}

int wsg_bandwidth_probe(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst || bytes % 16 || (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16)
        return fail(WSG_EINVAL, "probe: 16-byte aligned pointers and a multiple of 16 bytes are required");
    const char *a = static_cast<const char*>(src), *b = static_cast<const char*>(dst);
    if (a < b + bytes && b < a + bytes) return fail(WSG_EINVAL, "probe: overlapping buffers");
    const size_t n = bytes / 16;
    if (n == 0) return WSG_OK;
    const unsigned blocks = unsigned(std::min<size_t>((n + kProbeThreads * kProbeUnroll - 1) /
                                                          (kProbeThreads * kProbeUnroll), 256 * 64));
    hipLaunchKernelGGL(k_copy_probe, dim3(blocks), dim3(kProbeThreads), 0, static_cast<hipStream_t>(stream),
                       static_cast<const probe_vec*>(src), static_cast<probe_vec*>(dst), n);
    WSG_HIP(hipGetLastError());
    return WSG_OK;
}

int64_t grid_skipped(const wsg_plan* plan, const void* ws, void* stream) {
    if (!plan || !ws) return fail(WSG_EINVAL, "null plan or workspace");
    uint32_t n = 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    WSG_HIP(hipMemcpyAsync(&n, ws, sizeof(n), hipMemcpyDeviceToHost, s));   // counter at offset 0
    WSG_HIP(hipStreamSynchronize(s));
    return int64_t(n);
}

}  // extern "C"
