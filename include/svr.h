/*
 * svr -- spectral-cube volume rendering on MI355X (gfx950).
 *
 * C ABI of the hot path of Vohl, Fluke, Barnes & Hassan (2017), "Real-time colouring and
 * filtering with graphics shaders": per-pixel ray casting through a (RA, Dec, velocity)
 * cube with the paper's transfer functions, filters, smoothing and line-ratio passes.
 *
 * Conventions shared by every entry point
 *  - Cubes are C-order [z][y][x]: x = RA (fastest), y = Dec, z = velocity.  Voxel (i,j,l)
 *    is centred at (i,j,l); the volume box is [-0.5, n-0.5] on each axis.
 *  - Pointers named *_host are host memory; every other data pointer is device memory
 *    owned by the caller, except the opaque handles (svr_volume, svr_batch), which the
 *    library owns and frees in the matching *_destroy call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the legacy default stream).  Work
 *    is enqueued asynchronously unless the entry point says it synchronises.
 *  - Every function returns an svr_status; no exception crosses the ABI.  Arguments are
 *    validated on the host before anything is enqueued; a call that fails validation has
 *    written nothing.  svr_last_error() returns a message for the calling thread's last
 *    failure.  Asynchronous device faults surface at the next synchronising call
 *    (svr_sync, svr_minmax, svr_volume_clim) as SVR_EHIP.
 */
#ifndef SVR_H
#define SVR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SVR_OK = 0,
    SVR_EINVAL = 1,        /* an argument is out of its documented range */
    SVR_ENOMEM = 2,        /* device allocation failed or a workspace is too small */
    SVR_EHIP = 3,          /* the HIP runtime reported an error */
    SVR_EUNSUPPORTED = 4   /* valid but not implemented (e.g. non-contiguous smooth input) */
} svr_status;

/* Storage / element types. */
typedef enum { SVR_F32 = 0, SVR_F16 = 1, SVR_BF16 = 2 } svr_dtype;

/* Transfer functions of Section 3: zeroth-moment (MIP0, AVIP0, Alg. MIP0/AVIP0),
 * first-moment (MIP1, AVIP1, Alg. MIP1/AVIP1) and RGB-cube (Alg. MIP_RGB/AVIP_RGB). */
typedef enum {
    SVR_MIP0 = 0, SVR_MIP1 = 1, SVR_MIPRGB = 2, SVR_AVIP0 = 3, SVR_AVIP1 = 4, SVR_AVIPRGB = 5
} svr_mode;

/* filter() of Alg. 1: Section 4.3 intensity clipping, Section 4.4 domain scaling. */
typedef enum { SVR_FILTER_NONE = 0, SVR_FILTER_CLIP = 1, SVR_FILTER_SCALE = 2 } svr_filter;

#define SVR_MAX_LUT 1024      /* entries of a colour table */
#define SVR_MAX_BOX_ARM 15    /* Section 4.1 filterArm */
#define SVR_MAX_TAPS 63       /* smoothing kernel length */

const char* svr_status_string(int status);
const char* svr_last_error(void);
/* Library version string; also a cheap "is the library loadable" probe. */
const char* svr_version(void);

/* A strided view of a cube in device memory.  Strides are in elements; all three zero means
 * C-contiguous [z][y][x]. */
typedef struct {
    const void* data;
    int32_t dtype;            /* svr_dtype */
    int32_t nx, ny, nz;
    int64_t sx, sy, sz;
} svr_cube_view;

/* Finite minimum and maximum of a cube (NaN and +-inf ignored): the default colour-map
 * domain, whose minimum is the paper's DATAMIN (Alg. intensity clipping).  Writes
 * lo_hi_host[2]; if no value is finite both are NaN.  Synchronises `stream`. */
svr_status svr_minmax(const svr_cube_view* cube, float* lo_hi_host, void* stream);

/* Allocation-free variant of svr_minmax, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * The same finite minimum and maximum as svr_minmax, written to lo_hi_dev[2] in DEVICE
 * memory owned by the caller, asynchronously on `stream` (no copy to the host, no
 * synchronisation).  It calls no hipMalloc, hipFree or other allocating routine: the
 * per-workgroup partials of the reduction live in a fixed library array of 3 x 2048 floats
 * (24 KiB) on each GPU, set up on the first call on that GPU and held until the process
 * ends.  The reduction never uses more than 2048 workgroups, so every cube size fits;
 * SVR_EINVAL (with a message) if a launch would need more partials than the array holds.
 * Calls that overlap on one GPU share the array and race: serialise them (one stream, or
 * events between streams). */
svr_status svr_minmax_noalloc(const svr_cube_view* cube, float* lo_hi_dev, void* stream);

/* ---------------------------------------------------------------- volumes (upload)
 * A volume is the library's copy of a cube laid out for the ray-march: cubic bricks of
 * `brick` voxels per edge, each stored with a one-voxel apron on its +x/+y/+z faces (so a
 * trilinear stencil never leaves its brick; beyond the cube's last voxel the apron repeats
 * it, i.e. clamp-to-edge), converted to `storage` with round-to-nearest-even.  NaN voxels
 * (masked mosaics, Section 5.2) are stored as `nan_fill`, or as the finite minimum
 * (DATAMIN) when nan_fill is NaN.  The volume also keeps its finite min/max on the device.
 * brick: 8 or 16 (0 selects 8).  Library-owned device memory; the source may be released
 * once `stream` has passed the call.  Creation is asynchronous on `stream`. */
typedef struct svr_volume svr_volume;
svr_status svr_volume_create(const svr_cube_view* src, int32_t storage, int32_t brick,
                             float nan_fill, void* stream, svr_volume** out);
svr_status svr_volume_destroy(svr_volume* vol);
/* Re-upload a cube of the same dims into an existing volume (same storage and brick, no
 * allocation): the upload pass alone, asynchronous on `stream`. */
svr_status svr_volume_upload(svr_volume* vol, const svr_cube_view* src, float nan_fill,
                             void* stream);
/* dims_zyx[3] = (nz, ny, nx); bytes = device bytes held.  Host-only query. */
svr_status svr_volume_info(const svr_volume* vol, int32_t* dims_zyx, int32_t* storage,
                           int32_t* brick, int64_t* bytes);
/* The volume's finite min/max (after quantisation).  Synchronises `stream`. */
svr_status svr_volume_clim(const svr_volume* vol, float* lo_hi_host, void* stream);
/* Copy the stored values back as a C-contiguous [z][y][x] cube of the storage dtype. */
svr_status svr_volume_export(const svr_volume* vol, void* out, void* stream);

/* ---------------------------------------------------------------- rendering
 * Camera (Appendix A).  Pixel (px, py) gives u = 2(px+0.5)/width - 1 and
 * v = 2(py+0.5)/height - 1.  type 0 (parallel): origin eye + uU + vV, direction W.
 * type 1 (perspective): origin eye, direction W + uU + vV.  Directions are normalised, so
 * the step dt is in voxels.  The ray runs over t >= 0 inside the volume box. */
typedef struct {
    int32_t type;
    float eye[3], U[3], V[3], W[3];
    int32_t width, height;
} svr_camera;

/* Colour map (Section 2.1): n RGBA float entries, entry j at s = j/(n-1), linearly
 * interpolated; 2 <= n <= SVR_MAX_LUT.  Device memory, 16-byte aligned (SVR_EINVAL
 * otherwise). */
typedef struct {
    const float* rgba;
    int32_t n;
} svr_lut;

#define SVR_MAX_STAR 4

/* Parameters of Alg. 1 and its smooth()/filter()/transferFunction()/setFragment().
 *  mode            svr_mode.
 *  filter          svr_filter, thresholds min_t/max_t (Sections 4.3, 4.4); for the ratio
 *                  methods clipping uses min_t/max_t on cube 1 and min_t2/max_t2 on cube 2.
 *  box_arm         Section 4.1 filterArm: the mean of the 2*box_arm+1 samples centred on
 *                  each sample along the ray, taken before filter(); 0 = off.
 *  mip_alpha       MIP alpha: 0 = colour-table alpha (MIP0) or s_max (MIP1, MIP_RGB);
 *                  1 = opaque; 2 = opaque where s_max exceeds the scaled min_t, s_max (MIP1,
 *                  MIP_RGB) or table alpha (MIP0) elsewhere (the transparency workaround of
 *                  the Discussion, Section 5.7).
 *  ratio           0 = none; 1/2 = line-ratio method 1/2 of Section 4.5 (needs vol2, mode
 *                  SVR_MIP0, box_arm 0, filter none or clip); the ratio is mapped onto
 *                  [ratio_lo, ratio_hi].
 *  opacity_from_lut AVIP opacity weight: 0 = k*s (Alg. AVIP0), 1 = k*table(s).a.
 *  k, min_val, ert AVIP weighting factor in [0,1], minVal > 0, termination threshold (the
 *                  ray stops after the sample whose alpha exceeds ert; 0.99 in the paper).
 *  clim_lo/hi      colour-map domain [lo, hi]; DATAMIN = lo.  clim_hi <= clim_lo selects
 *                  the volume's own finite min/max.
 *  dt              sample spacing along the ray, voxels (> 0).  Samples t_k = t_enter +
 *                  k*dt for k = 0 .. ceil((t_exit - t_enter)/dt) - 1.
 *  star_n, star_c0, star_off, star_w
 *                  in-ray 3-axis Gaussian of Section 4.2 (Alg. 9-tap smoothing), the
 *                  alternative to box_arm: each sample value v at point p becomes, for the
 *                  axes e = x, then y, then z, v <- c0 v + sum_{k < star_n} w_k (cube[p +
 *                  off_k e] + cube[p - off_k e]), every lookup a trilinear fetch of the raw
 *                  cube (1 + 6 star_n fetches per sample; the paper's 9-tap form has star_n
 *                  = 2, off = (1.3846153846, 3.2307692308), w = (0.3162162162, 0.0702702703),
 *                  c0 = 0.2270270270).  star_n = 0 (up to SVR_MAX_STAR) disables it; offsets
 *                  in voxels, finite, in [0, 64]; needs box_arm 0 and ratio 0. */
typedef struct {
    int32_t mode;
    int32_t filter;
    int32_t box_arm;
    int32_t mip_alpha;
    int32_t ratio;
    int32_t opacity_from_lut;
    float k, min_val, ert;
    float clim_lo, clim_hi;
    float dt;
    float min_t, max_t;
    float min_t2, max_t2;
    float ratio_lo, ratio_hi;
    int32_t star_n;
    float star_c0;
    float star_off[SVR_MAX_STAR];
    float star_w[SVR_MAX_STAR];
} svr_params;

/* Host-only check of a parameter set (everything that does not depend on a volume):
 * SVR_OK or SVR_EINVAL with svr_last_error() naming the offending field. */
svr_status svr_params_validate(const svr_params* params);

/* Render one image: rgba_out[height][width][4] float32 (row py = v), 16-byte aligned
 * (SVR_EINVAL otherwise).  A ray that misses the
 * volume gives (0,0,0,0).  samples_out (may be NULL) receives, per pixel, the number of
 * samples the transfer function consumed (all N for MIP, up to and including the
 * terminating sample for AVIP).  vol2 is the second line cube for ratio methods (same
 * dims and storage as vol), NULL otherwise. */
svr_status svr_render(const svr_volume* vol, const svr_volume* vol2, const svr_camera* cam,
                      const svr_lut* lut, const svr_params* params, float* rgba_out,
                      int32_t* samples_out, void* stream);

/* Host-only: the number of segments svr_render splits each ray of this view into.  1 is one
 * pass per ray.  For the MIP transfer functions (raw or box-smoothed), oblique views
 * with few rays and many samples split each ray's samples over up to 8 workgroups, so more
 * loads are in flight (parallel views along a volume axis stay one pass: they stream the
 * bricks in order); a per-pixel 64-bit maximum of (s, k) keys then selects the same sample
 * as the one-pass render (Eq. MIP, later sample on ties), and the image is bit-identical to
 * it.  The split render runs three kernels on the stream (clear, march, finalise) and uses
 * the output image as its scratch. */
svr_status svr_render_segments(const svr_volume* vol, const svr_camera* cam,
                               const svr_params* params, int32_t* segments);

/* ---------------------------------------------------------------- smoothing pre-pass
 * Separable 3D smoothing (Section 4.2: the 1D kernel applied successively along x, y, z)
 * with clamp-to-edge borders and float32 accumulation.  taps_host[ntaps] (odd ntaps <=
 * SVR_MAX_TAPS) is centred: out[x] = sum_j taps[j] * in[x + j - ntaps/2].  `in` must be
 * C-contiguous; `out` is C-contiguous with the same dims and dtype.  workspace: device
 * buffer of at least svr_smooth_workspace(in, ntaps) bytes: 0 for the tap counts with a
 * fused single-pass kernel (5, 7, 9, 13, 19; workspace may then be NULL), two float32 cubes
 * otherwise. */
svr_status svr_smooth_workspace(const svr_cube_view* in, int32_t ntaps, size_t* bytes);
svr_status svr_smooth(const svr_cube_view* in, const float* taps_host, int32_t ntaps,
                      void* out, void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------- moment maps
 * Moment maps of every spectrum of a cube over the channel window [z0, z0 + nz_w)
 * (Section 2.2, Eq. mom0 and Eq. mom1, and the argmax variant described with them).  A
 * channel counts when its value is finite and inside [min_t, max_t] (pass -inf / +inf for
 * no clipping).  For the spectrum at (x, y):
 *   m0_out[y][x]     = dv * sum of the counted values (dv: channel width);
 *   m1_out[y][x]     = sum z v / sum v over the counted channels, z the cube's channel index
 *                      (NaN when no channel counts or the sum is zero);
 *   argmax_out[y][x] = the last channel holding the largest counted value (the MIP tie rule),
 *                      -1 when no channel counts.
 * Sums are formed in float64 in channel order and rounded to float32 at the end.  Outputs are
 * C-contiguous [ny][nx] device buffers owned by the caller; any of them may be NULL, not all.
 * SVR_EINVAL: window outside the cube, NaN dv / min_t / max_t, min_t > max_t, ny > 65535. */
svr_status svr_moments(const svr_cube_view* cube, int32_t z0, int32_t nz_w, float dv,
                       float min_t, float max_t, float* m0_out, float* m1_out,
                       int32_t* argmax_out, void* stream);

/* ---------------------------------------------------------------- line ratio pass
 * Voxel-wise emission-line ratio of two spectral windows of one cube (Section 4.5,
 * method 2 computed per voxel): with a = cube[z0_a + j], b = cube[z0_b + j] (j < nz_w),
 * each first clipped (a < min_t_a -> datamin, b < min_t_b -> datamin),
 * ratio_out[j][y][x] = b / a where a > 0, else datamin.  float32 output, C-contiguous. */
svr_status svr_line_ratio(const svr_cube_view* cube, int32_t z0_a, int32_t z0_b,
                          int32_t nz_w, float min_t_a, float min_t_b, float datamin,
                          float* ratio_out, void* stream);

/* ---------------------------------------------------------------- differentiable render
 * AVIP0 with a piecewise-linear RGBA transfer function `tf` (colour = tf(s).rgb, opacity
 * weight = k * tf(s).a; filter none, box_arm 0, ratio 0), whose forward pass stores the
 * ray state every 32 samples in a caller-owned workspace, and its hand-written adjoint.
 * The paper leaves the choice of k and of the transfer function to the user and names
 * its automation as future work (Section 7); the adjoint lets it be fitted by gradient
 * descent. */
svr_status svr_render_train_workspace(const svr_volume* vol, const svr_camera* cam,
                                      const svr_params* params, size_t* bytes);
svr_status svr_render_train(const svr_volume* vol, const svr_camera* cam, const svr_lut* tf,
                            const svr_params* params, float* rgba_out, void* workspace,
                            size_t workspace_bytes, void* stream);
/* rgba_out, the workspace and grad_rgba are 16-byte aligned (SVR_EINVAL otherwise).
 * grad_rgba[height][width][4] = dL/dRGBA.  grad_tf[n*4] and grad_vox[nz*ny*nx] (float32,
 * C-contiguous [z][y][x]; may be NULL) are ACCUMULATED with atomics: zero them first.
 * The termination index, the interval of the table and the minVal clamp are held at the
 * forward pass's values. */
svr_status svr_render_backward(const svr_volume* vol, const svr_camera* cam, const svr_lut* tf,
                               const svr_params* params, const void* workspace,
                               size_t workspace_bytes, const float* grad_rgba,
                               float* grad_tf, float* grad_vox, void* stream);

/* ---------------------------------------------------------------- batched rendering
 * Render n volumes, each with its own camera and output image, in ONE persistent launch:
 * a device work queue of (volume, tile) items ordered by estimated cost is drained by
 * workgroups that claim items with an atomic counter.  The launch pair (counter reset,
 * persistent kernel) is captured once into a HIP graph; svr_batch_launch replays it.  The
 * lut/params/volumes/outputs (16-byte aligned) must stay alive and unchanged in shape until
 * destroy.  Each
 * image equals, bit for bit, what svr_render gives for that volume and camera.  The
 * many detection sub-cubes of a survey (Section 1) motivate the form.
 * tune: 0 = the default shape (the volumes' brick edge, 16 x 16 pixel tiles, 4 workgroups
 * per CU); 1 = the autotuner's choice for the batch's size class, taken from the tuning
 * cache when it holds one, else searched and stored; 2 = always search (and store).  The
 * search times every combination of brick edge (8, 16) x tile (8 x 32, 16 x 16, 32 x 8
 * pixels) x grid (2, 4, 8 workgroups per CU) as the median of three launches on `stream`
 * (synchronising it).  When the other brick edge wins, the batch keeps library-owned
 * copies of the volumes re-bricked to it (freed by svr_batch_destroy).  The size class is
 * the storage type, transfer function, box smoothing on/off and the log2 buckets of n, the
 * median voxel count and the median image size (and the CU count). */
typedef struct svr_batch svr_batch;
svr_status svr_batch_create(const svr_volume* const* vols, const svr_camera* cams, int32_t n,
                            const svr_lut* lut, const svr_params* params,
                            float* const* rgba_outs, int32_t tune, void* stream,
                            svr_batch** out);
svr_status svr_batch_launch(svr_batch* batch, void* stream);
/* The launch the batch replays.  items = work-queue length, grid = workgroups of the
 * persistent launch, tile_waves_x = width of the 4-wave (8 x 8 pixels per wave) tile in
 * waves: 1 (8 x 32 pixels), 2 (16 x 16) or 4 (32 x 8); brick = brick edge of the volumes it
 * reads; from_cache = 1 when the choice came from the tuning cache; default_ms / tuned_ms =
 * median launch time of the default shape and of the chosen one when the batch searched
 * (0 otherwise). */
typedef struct {
    int64_t items;
    int32_t grid;
    int32_t tile_waves_x;
    int32_t brick;
    int32_t from_cache;
    float default_ms;
    float tuned_ms;
} svr_batch_stats;
svr_status svr_batch_info(const svr_batch* batch, svr_batch_stats* stats);
/* Tuning cache file (text, one line per size class, appended to): `path`, or none when
 * path is NULL or empty.  Until this is called the environment variable SVR_TUNE_CACHE
 * names it (none when unset).  Process-wide. */
svr_status svr_set_tune_cache(const char* path);
svr_status svr_batch_destroy(svr_batch* batch);

/* Wait for `stream` and report any pending asynchronous HIP error. */
svr_status svr_sync(void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SVR_H */
