/*
 * wsgrid.h -- improved W-stacking gridding and degridding on one MI355X (gfx950).
 *
 * Implements the two operators of Ye, Gull, Tan & Nikolic, "High accuracy wide
 * field imaging method in radio interferometry" (MNRAS 2021):
 *
 *   grid    (Algorithm 5): visibilities -> real dirty map
 *       D[j][i] ~= h_x h_y h_z * Re sum_t [IFFT2 G_t](i, j) exp(+i 2 pi t z_ji),
 *       G_t = sum_k V_k exp(+i 2 pi w_k (n0 - 1)) C(r - u'_k) C(s - v'_k) C(t - w'_k)
 *       (Sec. 5.2 eqs. gridded-dirty-map and gridded_vis, Sec. 5.4);
 *   degrid  (Algorithm 6): real model image -> visibilities, the exact adjoint.
 *
 * Both approximate the direct Fourier pair of eq. fourier_visibility
 *     V_k = sum_ji f_ji exp[-i 2 pi (u_k l_i + v_k m_j + w_k (n_ji - 1))],
 *     D_ji = Re sum_k V_k exp[+i 2 pi (u_k l_i + v_k m_j + w_k (n_ji - 1))],
 * with RMS relative error about sqrt(3) E(W, x0) (Sec. 6.3), E the 1-D error
 * bound of eq. norm_bound for the least-misfit functions C, h (Sec. 3.3).
 *
 * Conventions shared by every entry point:
 *   - image f / dirty map D: N x N real, row-major, row j <-> m_j, column i <-> l_i,
 *     l_i = (i - N/2) L/N (same for m);  f is I/n (Sec. 5.2); no 1/M weights.
 *   - uvw: M x 3 float64, row-major (u, v, w) in wavelengths, any sign and size
 *     (u, v are taken modulo the FFT grid; Sec. 5.2).  w < 0 is folded to
 *     (-u, -v, -w, conj V) (Sec. 5.4).  |w| > wmax (or a non-finite coordinate)
 *     is skipped: grid ignores it, degrid returns 0 for it.
 *   - vis: M complex values, interleaved (re, im): complex64 for WSG_F32,
 *     complex128 for WSG_F64.  Image/dirty: float32 for WSG_F32, float64 for WSG_F64.
 *   - all array pointers given to grid_visibilities / degrid_visibilities (and
 *     their _batch forms) are HIP device pointers owned by the caller; the call
 *     only enqueues work on `stream` (a hipStream_t, NULL = default stream) and
 *     returns.  Host memory is used only for the plan, the channel counts of a
 *     batched call and the error message; the library allocates device memory
 *     only in grid_create (its tables).
 *   - memory: the caller's workspace holds the binned visibilities, the layer
 *     stack and the FFT intermediates; a workspace smaller than the one that
 *     holds every layer makes the call take the layers in passes of whole tile
 *     layers (16 w-layers), with the same results.
 *   - return value 0 on success, or a negative WSG_E* code; the message is in
 *     grid_last_error() (thread-local).
 */
#ifndef WSGRID_H
#define WSGRID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wsg_plan wsg_plan;

/* arithmetic precision of a call: float32 or float64 data and arithmetic */
typedef enum wsg_prec { WSG_F32 = 0, WSG_F64 = 1 } wsg_prec;

enum {
    WSG_OK = 0,
    WSG_EINVAL = -1,      /* bad argument (size, precision, null pointer, plan)   */
    WSG_EWORKSPACE = -2,  /* workspace smaller than grid_workspace_bytes_min()    */
    WSG_ENOMEM = -3,      /* host allocation failed                               */
    WSG_EHIP = -4         /* HIP runtime error (no device, launch failure, ...)   */
};

/* w-layer method of a plan (see grid_create_axes) */
typedef enum wsg_method {
    WSG_IMPROVED = 0,             /* improved W-stacking, z offset (eq. n_params)         */
    WSG_IMPROVED_NO_OFFSET = 1,   /* improved W-stacking without z offset (Sec. 5.3)     */
    WSG_ORIGINAL = 2              /* original W-stacking, Algorithms 3 and 4 (Sec. 4)    */
} wsg_method;

/*
 * Create a plan for an N x N image spanning L in direction cosine (l, m in
 * [-L/2, L/2)), gridding width W in u, v and w, cropping parameter x0 (= y0 =
 * z0, Sec. 6.2) and largest |w| = wmax wavelengths.
 *   - FFT length N' = N / (2 x0) (Algorithm 1); must be 2^a or 3 2^a (radix-3
 *     transforms, e.g. x0 = 1/3, Sec. 6.3) in [64, 8192].
 *   - n_scale = (1 - n_min) / (2 z0), n0 = 1 - z0 n_scale (eq. n_params).
 *   - w-layers t = t_lo .. t_hi with t_lo = floor(W/2) - W + 1 and
 *     t_hi = floor(n_scale wmax + W/2) (Algorithm 5 step 1; every layer a
 *     folded visibility can touch).
 *   - designs the least-misfit C, h for (W, x0) in float64 on the host
 *     (Sec. 3.3, eqs. csum2 / norm_bound) and uploads the kernel polynomials,
 *     the per-pixel correction h_x h_y h_z (Algorithm 5 step 5) and the FFT
 *     twiddles to the current HIP device (blocking, ~N^2 x 12 bytes).
 * Valid ranges: N even, 1 <= W <= 16, 0 < x0 <= 1/2, 0 < L < sqrt(2), wmax >= 0.
 * Returns NULL on error (see grid_last_error()).  The plan is immutable and may
 * be used from several threads with distinct workspaces; it is bound to the
 * device that was current at creation.
 */
wsg_plan* grid_create(int N, double L, int W, double x0, double wmax);

/*
 * As grid_create, choosing the placement of the z = 0 plane (Sec. 5.3).
 * z_offset != 0: eq. n_params, exactly grid_create (z in [-z0, z0], the fewest
 * layers).  z_offset == 0: the variant without z offset, eq.
 * n_params_no_offset: n_scale = (1 - n_min) / z0 and n0 = 1, so z = 0 at the
 * map centre, where the correction h_z is smallest, and z in [-z0, 0]; the
 * layer spacing in w halves, so about twice as many layers, and the
 * per-visibility phase exp(+-i 2 pi w (n0 - 1)) is 1.  Same ranges, errors and
 * ownership as grid_create.
 */
wsg_plan* grid_create_variant(int N, double L, int W, double x0, double wmax, int z_offset);

/*
 * Plan with the gridding function chosen per axis and the w-layer method
 * (Sec. 5.2: eqs. gridded-dirty-map and gridded_vis allow separate C_x, C_y,
 * C_z; Sec. 6.1 trades W_z against z0; Sec. 4 and 6.2: the original method is
 * the W_z = 1 top hat).
 *   W, x0    width and cropping on u and v (the image axes);
 *   Wz, z0   width and cropping on w (improved methods): n_scale = (1 -
 *            n_min) / (2 z0) and n0 = 1 - z0 n_scale (WSG_IMPROVED) or n_scale
 *            = (1 - n_min) / z0 and n0 = 1 (WSG_IMPROVED_NO_OFFSET); layers
 *            t = floor(Wz/2) - Wz + 1 .. floor(n_scale wmax + Wz/2); the
 *            correction is h_x h_y h_z with h_z of the (Wz, z0) design;
 *   method   WSG_ORIGINAL: Algorithms 3 and 4 -- Wz must be 1 (z0 ignored),
 *            n_bins bins over [0, wmax] after the Hermitian fold (0: the
 *            smallest count of eq. N_w, ceil(2 pi (1 - n_min) wmax)); a
 *            visibility goes to bin t = floor(w / dw), dw = wmax / n_bins (the
 *            last bin closed), with weight 1 and the bin phase exp(+-i 2 pi
 *            w[t] (n - 1)) at the midpoint w[t] = (t + 1/2) dw; the correction
 *            is h_x h_y only.
 * Compiled width pairs: Wz = W with z0 = x0 (W = 1 .. 16); otherwise W = 7 with
 * Wz = 1 .. 7, or Wz = 1 with W = 3 .. 8.  Other pairs give WSG_EINVAL.
 * grid_create(N, L, W, x0, wmax) is grid_create_axes(N, L, W, x0, W, x0, wmax,
 * WSG_IMPROVED, 0).  NULL on error; ownership as for grid_create.
 */
wsg_plan* grid_create_axes(int N, double L, int W, double x0, int Wz, double z0, double wmax, wsg_method method,
                           int n_bins);

/*
 * Axis parameters of a plan (any output pointer may be NULL): W, x0, W_z, z0
 * (0 for the original method), the method, n_bins (original method, else 0)
 * and the error bound E of the w-axis design (NaN for the top hat).
 */
int grid_plan_axes(const wsg_plan* plan, int* W, double* x0, int* Wz, double* z0, int* method, int* n_bins,
                   double* E_z);

/* Free a plan and its device tables (blocking).  NULL is ignored. */
void grid_destroy(wsg_plan* plan);

/*
 * Plan parameters (any output pointer may be NULL): FFT length N', number of
 * w-layers N_w' (t_lo .. t_hi), first layer t_lo, n0, n_scale (Sec. 5.3, eq.
 * n_params) and the design's error bound E (eq. norm_bound).
 */
int grid_plan_info(const wsg_plan* plan, int* Nprime, int* n_layers, int* t_lo,
                   double* n0, double* n_scale, double* E);

/*
 * Device workspace (bytes) for one grid_visibilities or degrid_visibilities
 * call with M visibilities at precision `prec` that holds every w-layer at
 * once: the w-layer stack (n_layers N'^2 complex; only tiles some visibility
 * reaches are touched), the FFT intermediate before and after its transpose
 * (2 n_layers N N' complex), the binned visibility records (2 M records), the
 * degrid per-tile parts (8 M complex) and the bin tables.  0 on a bad argument.
 */
size_t grid_workspace_bytes(const wsg_plan* plan, wsg_prec prec, int64_t M);

/*
 * Smallest workspace (bytes) a call accepts: the same buffers with the stack
 * and FFT intermediates sized for one tile layer (16 w-layers).  A call given
 * ws_bytes between this and grid_workspace_bytes() processes the layers in
 * passes of as many tile layers as fit (Algorithm 5 steps 3a-4 and Algorithm 6
 * steps 3-4 are independent per layer; gridding sums the passes' maps, so the
 * result differs from one pass only by rounding order; degridding is the same
 * arithmetic).  0 on a bad argument.
 */
size_t grid_workspace_bytes_min(const wsg_plan* plan, wsg_prec prec, int64_t M);

/*
 * Dirty map by Algorithm 5.
 *   uvw   [M][3] float64 device;  vis [M] complex (prec) device;
 *   dirty [N][N] real (prec) device, overwritten;
 *   ws    device workspace of ws_bytes >= grid_workspace_bytes_min(plan, prec, M),
 *         contents on entry ignored (the call owns it until the stream reaches
 *         the end of the call's work).
 * M = 0 gives an all-zero map (uvw and vis may then be NULL).
 */
int grid_visibilities(const wsg_plan* plan, wsg_prec prec, int64_t M, const double* uvw,
                      const void* vis, void* dirty, void* ws, size_t ws_bytes, void* stream);

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: as
 * grid_visibilities, with the workspace taken from the library's own static
 * device buffer of WSG_SCRATCH_BYTES, which every device the library runs on
 * holds (its own copy) until the process ends.  The call allocates nothing
 * and makes no blocking HIP call; the buffer's device address is looked up
 * once per device when the first plan is created there.
 *   uvw, vis, dirty: as for grid_visibilities (caller's device memory).
 *   Returns WSG_EWORKSPACE when grid_workspace_bytes_min(plan, prec, M)
 *   exceeds WSG_SCRATCH_BYTES (the layers are taken in passes, as with a
 *   small workspace; only small plans and visibility counts fit, e.g. N' =
 *   512 with 13 layers and 5,000 visibilities in float64).
 * Every call on a device shares that device's buffer: the call clears what
 * must start at zero itself, and calls that overlap on one device (several
 * streams or threads) race and give wrong results.  grid_last_skipped(plan)
 * reads the count of skipped visibilities from the buffer.
 */
#define WSG_SCRATCH_BYTES ((size_t)128 << 20)
int grid_visibilities_noalloc(const wsg_plan* plan, wsg_prec prec, int64_t M, const double* uvw,
                              const void* vis, void* dirty, void* stream);

/*
 * Model visibilities by Algorithm 6 (exact adjoint of grid_visibilities under
 * Re <., .> on visibilities and <., .> on real images).
 *   uvw [M][3] float64 device;  image [N][N] real (prec) device;
 *   vis [M] complex (prec) device, overwritten;  ws as for grid_visibilities.
 * M = 0 does nothing but the layer transforms (uvw and vis may then be NULL).
 */
int degrid_visibilities(const wsg_plan* plan, wsg_prec prec, int64_t M, const double* uvw,
                        const void* image, void* vis, void* ws, size_t ws_bytes, void* stream);

/*
 * Batched channels: nch (1..64) channels on one plan, each with its own
 * visibilities (uvw in wavelengths at its own frequency, |w| <= wmax), gridded
 * to or degridded from its own map in one call whose binning, tile and FFT
 * stages are each one launch over all channels (Algorithms 5 and 6 applied per
 * channel; channels are independent).  Internally channel c's w-layers follow
 * channel c - 1's on one layer axis, so the workspace holds the channels'
 * layers together and the layer passes of grid_workspace_bytes_min run across
 * channel boundaries.
 *   M     [nch] visibility counts (host memory), any may be 0;
 *   uvw   [sum M][3] float64 device, the channels' visibilities one after the
 *         other (channel 0 first); vis [sum M] complex (prec) device, same order;
 *   dirty [nch][N][N] real (prec) device, overwritten (grid);
 *   image [nch][N][N] real (prec) device (degrid); vis overwritten (degrid);
 *   ws    device workspace of ws_bytes >= grid_workspace_bytes_batch(plan,
 *         prec, nch, sum M, 1); with grid_workspace_bytes_batch(..., 0) every
 *         layer of every channel is held at once.
 * The result of channel c equals grid_visibilities / degrid_visibilities on
 * channel c alone (degrid: bit for bit; grid: up to the rounding order of the
 * sum over layer passes).  Errors as for the single-channel calls, plus
 * WSG_EINVAL for nch outside [1, 64], a sum of M of 2^31 or more, or more than
 * 2^25 tiles over the channels.
 */
int grid_visibilities_batch(const wsg_plan* plan, wsg_prec prec, int nch, const int64_t* M, const double* uvw,
                            const void* vis, void* dirty, void* ws, size_t ws_bytes, void* stream);
int degrid_visibilities_batch(const wsg_plan* plan, wsg_prec prec, int nch, const int64_t* M, const double* uvw,
                              const void* image, void* vis, void* ws, size_t ws_bytes, void* stream);

/*
 * One binning shared by several gridding and degridding calls on the same
 * visibilities.  The fold (Sec. 5.4), the normalised coordinates, the support
 * boxes, the tile binning and the phase e^{+-i 2 pi w (n0 - 1)} of Algorithm 5
 * step 2 and Algorithm 6 steps 4-5 depend on uvw alone, so an imaging loop
 * that grids and degrids the same visibilities many times (Sec. 7: the
 * gridding/degridding pair inside a reconstruction) bins them once.
 * grid_prepare bins nch channels' visibilities (as grid_visibilities_batch:
 * M [nch] host counts, uvw [sum M][3] float64 device) into ws, a device
 * workspace of ws_bytes >= grid_workspace_bytes_batch(plan, prec, nch, sum M,
 * 1), and keeps the binning there for this plan.  The prepared calls then take
 * only the values:
 *   grid_visibilities_prepared:   vis [sum M] complex (prec) -> dirty [nch][N][N];
 *   degrid_visibilities_prepared: image [nch][N][N] real (prec) -> vis [sum M],
 * with the same ws, ws_bytes and prec.  Their results equal those of
 * grid_visibilities_batch / degrid_visibilities_batch on the prepared uvw
 * (degrid bit for bit; grid up to the rounding of the value's phase product,
 * which the scatter forms in FP64 from the stored phase).  The binning stays valid until another call is
 * made on ws: any grid_prepare or plain call of this plan on ws replaces it (the
 * library notices and the prepared calls then fail with WSG_EINVAL); calls of
 * other plans on the same memory are the caller's to avoid.  The plan keeps one
 * binning (the most recent grid_prepare).  grid_last_skipped and grid_skipped
 * report the visibilities skipped by the binning.  uvw may change after
 * grid_prepare returns; the binning keeps what it read.
 * Errors: as for the batched calls; WSG_EINVAL from a prepared call when this
 * plan holds no binning in ws for ws_bytes and prec.
 */
int grid_prepare(const wsg_plan* plan, wsg_prec prec, int nch, const int64_t* M, const double* uvw, void* ws,
                 size_t ws_bytes, void* stream);
int grid_visibilities_prepared(const wsg_plan* plan, wsg_prec prec, const void* vis, void* dirty, void* ws,
                               size_t ws_bytes, void* stream);
int degrid_visibilities_prepared(const wsg_plan* plan, wsg_prec prec, const void* image, void* vis, void* ws,
                                 size_t ws_bytes, void* stream);

/*
 * Batched channels with plans of their own (image size N_c, wmax, widths):
 * channel c uses plans[c]; channels that share a plan must be consecutive and
 * each such run is one grid_visibilities_batch / degrid_visibilities_batch
 * (one launch per stage over the run's channels), the runs one after the
 * other on `stream` with the same workspace.  All plans on one device.
 *   M      [nch] visibility counts (host); uvw, vis: the channels' visibilities
 *          one after the other, as for the _batch calls;
 *   dirty / image: the channels' N_c x N_c maps one after the other (channel
 *          c at offset sum_{c' < c} N_c'^2 elements);
 *   ws     ws_bytes >= grid_workspace_bytes_multi(nch, plans, prec, M, 1).
 * Channel c's result equals the single-channel call with plans[c] (degrid:
 * bit for bit).  Errors as for the _batch calls, plus WSG_EINVAL when a plan
 * pointer is null or a plan recurs after another plan's run.
 */
int grid_visibilities_multi(int nch, const wsg_plan* const* plans, wsg_prec prec, const int64_t* M,
                            const double* uvw, const void* vis, void* dirty, void* ws, size_t ws_bytes,
                            void* stream);
int degrid_visibilities_multi(int nch, const wsg_plan* const* plans, wsg_prec prec, const int64_t* M,
                              const double* uvw, const void* image, void* vis, void* ws, size_t ws_bytes,
                              void* stream);

/*
 * Workspace (bytes) of the _multi calls: the largest over the runs of
 * grid_workspace_bytes_batch(run plan, prec, run channels, run visibilities,
 * min_passes).  0 on a bad argument.
 */
size_t grid_workspace_bytes_multi(int nch, const wsg_plan* const* plans, wsg_prec prec, const int64_t* M,
                                  int min_passes);

/*
 * Workspace (bytes) of a batched call with nch channels and M visibilities in
 * all: min_passes = 0 holds every layer of every channel at once, 1 gives the
 * smallest workspace the call accepts (one tile layer of 16 w-layers per
 * pass).  0 on a bad argument.
 */
size_t grid_workspace_bytes_batch(const wsg_plan* plan, wsg_prec prec, int nch, int64_t M, int min_passes);

/*
 * Virtual w-layers per layer pass that a call with nch channels, M
 * visibilities in all and a workspace of ws_bytes would use (the channels'
 * layers laid end to end, each channel padded to whole tile layers of 16);
 * WSG_EWORKSPACE when ws_bytes is below the minimum, WSG_EINVAL on a bad
 * argument.  Host only.
 */
int grid_layers_per_pass(const wsg_plan* plan, wsg_prec prec, int nch, int64_t M, size_t ws_bytes);

/*
 * Number of visibilities skipped (|w| > wmax or non-finite) by the last call
 * that used workspace `ws`.  Waits for `stream`.  Returns < 0 on error.  The
 * count lives in the caller's workspace, so calls on one plan with distinct
 * workspaces (several threads) each keep their own.
 */
int64_t grid_skipped(const wsg_plan* plan, const void* ws, void* stream);

/*
 * The same count for the most recent grid/degrid call made with this plan (on
 * any thread): the library remembers that call's workspace and stream, waits
 * for the stream and reads the counter there.  Valid while that workspace is
 * alive and not reused by another plan.  Returns < 0 when the plan has made no
 * call yet or on a HIP error.
 */
int64_t grid_last_skipped(const wsg_plan* plan);

/*
 * Measurement aid.  While enabled on the calling thread, every grid/degrid call
 * records HIP events on its stream around each stage:
 *   0 grid binning (fold, count, scan, scatter)   4 degrid binning
 *   1 grid 3-D scatter tiles                     5 degrid FFT pass along p (+ w-screen)
 *   2 grid FFT pass along v (+ crop)             6 degrid FFT pass along q
 *   3 grid FFT pass along u (+ w-screen, sum)    7 degrid 3-D gather tiles
 *   8 grid intermediate transpose                9 degrid intermediate transpose
 * grid_prepare's binning is timed as stage 4 (it is the degridding binning).
 * wsg_stage_times() waits for the recorded events, writes the summed
 * milliseconds and the number of timed sections of the first n stages (one per
 * layer pass; stage 7 one more for the final sum of parts; either pointer may
 * be NULL), clears the record and returns WSG_NSTAGES (or < 0 on error).
 */
#define WSG_NSTAGES 10
void wsg_stage_timing(int enable);
int wsg_stage_times(double* ms, int* launches, int n);

/*
 * Measurement aid: achievable HBM bandwidth.  Enqueues on `stream` one
 * streaming copy kernel dst[i] = src[i] over `bytes` bytes (16-byte vectors,
 * each byte read once and written once), so that bytes * 2 / its duration is
 * the read + write rate the memory system sustains for a plain stream.  src
 * and dst are device pointers, 16-byte aligned, not overlapping; bytes a
 * multiple of 16.  WSG_EINVAL otherwise.
 */
int wsg_bandwidth_probe(const void* src, void* dst, size_t bytes, void* stream);

/* Message of the last error on this thread ("" if none). */
const char* grid_last_error(void);

/*
 * Host-only inspection of the library's own least-misfit design (no GPU use):
 * for width W and cropping x0, writes c_a(nu_k) = C(a - (W-1)/2 - nu_k) for the
 * n_nu points nu (each in [-1/2, 1/2]) to c_out[k*W + a] (from the fitted
 * kernel polynomials the device evaluates), h(x_k) for the n_x points x (|x| <=
 * 1/2) to h_out, and E to *E_out (any output may be NULL when its count is 0).
 */
int wsg_design_eval(int W, double x0, int n_nu, const double* nu, double* c_out,
                    int n_x, const double* x, double* h_out, double* E_out);

/*
 * Host-only planner (no GPU use): the values grid_create_variant(..., z_offset)
 * would use (z_offset = 1: grid_create).  Any output pointer may be NULL.
 */
int wsg_plan_params(int N, double L, int W, double x0, double wmax, int z_offset,
                    int* Nprime, int* t_lo, int* t_hi, double* n0, double* n_scale);

/* Host-only planner of grid_create_axes (no GPU use, no design). */
int wsg_plan_params_axes(int N, double L, int W, double x0, int Wz, double z0, double wmax, wsg_method method,
                         int n_bins, int* Nprime, int* t_lo, int* t_hi, double* n0, double* n_scale);

#ifdef __cplusplus
}
#endif

#endif /* WSGRID_H */
