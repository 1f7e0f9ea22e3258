/*
 * lc.h - time-sliced retarded-time (light-cone) radiation field on a
 * periodic 3D grid, for AMD Instinct MI355X (gfx950).
 *
 * The library computes, for every band b of every periodic box,
 *
 *     J_b = IDFT( sum_k  G^_{k,b} . DFT(S_k) ) / N^3
 *
 * which is the time-sliced field of Sec. 2.1 (Eqs. 9-10) discretised on a
 * uniform grid (Sec. 2.2, Eq. 11) and evaluated by the convolution theorem
 * (Eqs. 12-13, algorithm steps 2-6). S_k is the source grid of lookback
 * slice k (luminosity per cell; the cell volume is absorbed, Eq. 11), and
 * G_{k,b} the periodic retarded-time shell kernel of slice k (Eq. 10):
 *
 *   G_{k,b}(c) = (1/m^3) sum_{subpoints} sum_{images u}
 *                [r_k <= rho < r_{k+1}] pref * phi_b(rho) / (4 pi rho^2)
 *
 * summed over the periodic images of a unit source (algorithm step 2) and
 * averaged over m^3 subpoints of the cell (m = 1 is the paper's node rule).
 * Membership is decided exactly: with h = L/(2 m N) a subpoint at integer
 * half-subcell offsets q has n = q.q (an exact integer) and lies in slice k
 * iff T_k <= n < T_{k+1}, T_k = (r_k/h)*(r_k/h) in IEEE double. When
 * r_0 = 0 the unit source's own cell takes the exact cube average of
 * pref * phi/(4 pi r^2), finite although the integrand is singular.
 *
 * DFT convention (Eq. 12): forward exp(-2 pi i (ip+jq+kr)/N), unnormalised;
 * inverse exp(+...), scaled by 1/N^3.
 *
 * Grid layout: cell (i, j, k) at flat index (i*N + j)*N + k, k contiguous;
 * its position is (i, j, k) * l with l = L/N (node convention, Sec. 2.2).
 *
 * Conventions shared by every call:
 *   - Every function returns an lc_status (0 = success, < 0 = error); no
 *     call throws or aborts. On error the plan is left unchanged and
 *     lc_last_error() describes the failure.
 *   - Arguments are validated on the host before any device work.
 *   - All device work is enqueued on the plan's HIP stream; device pointers
 *     passed in must stay valid and unmodified until the stream reaches the
 *     call. Host-pointer sources are consumed before the call returns;
 *     host-pointer outputs make lc_field synchronise the stream.
 *   - The caller owns all memory passed in (workspace, sources, outputs).
 *     The plan owns host tables only and sub-allocates inside the
 *     caller's workspace; lc_destroy frees no caller memory.
 *   - A plan is not thread-safe: use one host thread per plan.
 */
#ifndef LC_H
#define LC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LC_OK = 0,
    LC_EINVAL = -1,        /* invalid argument or descriptor field */
    LC_ENOMEM = -2,        /* workspace smaller than lc_workspace_bytes() */
    LC_EDEVICE = -3,       /* no usable gfx950 device, or a HIP call failed */
    LC_ESTATE = -4,        /* call out of order (e.g. field before kernels built) */
    LC_EUNSUPPORTED = -5,  /* valid but unsupported size or combination */
    LC_ENONFINITE = -6     /* a slice's sources hold a NaN or an infinity (their FP64
                              sum is not finite); reported by lc_field with host
                              outputs and by lc_check_sources */
} lc_status;

/* Arithmetic of the transforms and the slice sum. */
typedef enum {
    /* FP64 everywhere; unfused passes (forward x, y, z per slice, then a
     * separate multiply-accumulate over slices, then one inverse). */
    LC_PREC_FP64 = 0,
    /* FP32 everywhere, twiddles computed in FP32, plain FP32 slice sum,
     * same unfused passes as LC_PREC_FP64. */
    LC_PREC_FP32_PLAIN = 1,
    /* FP32 butterflies with twiddles generated in FP64; the forward z
     * transform, the multiply-accumulate over slices (compensated,
     * Kahan) and the inverse z transform fused in one pass; the mean
     * (DC) mode summed in FP64 and added back in FP64; kernels built in
     * FP64 and stored in FP32. */
    LC_PREC_FP32 = 2
} lc_precision;

typedef enum { LC_F32 = 0, LC_F64 = 1 } lc_dtype;
typedef enum { LC_MEM_HOST = 0, LC_MEM_DEVICE = 1 } lc_mem;

/* One periodic box. */
typedef struct {
    int32_t n;            /* grid side N: 8..512, N = 2^a 3^b, N even     */
    int32_t n_slices;     /* K >= 1 lookback slices (algorithm step 1)    */
    int32_t n_bands;      /* B >= 1 radial factors sharing the sources    */
    int32_t supersample;  /* m: 1 (node rule) .. 8 subpoints per axis     */
    int32_t conserve;     /* 1: rescale G_{k,b} so l^3 sum_c G = shell
                             integral of phi_b over [r_k, r_{k+1})         */
    int32_t rule;         /* mesh kernel G_{k,b} at a cell (Eq. 10 over the
                             cell): 0 = average over m^3 subpoints
                             (supersample m); 1 = exact cell average, the
                             m -> infinity limit (supersample unused; build
                             cost ~20-100x rule 0)                        */
    double box;           /* L, same length unit as radii                 */
    const double *radii;  /* K+1 strictly increasing, r_0 >= 0 (host);
                             slice k <-> shell [r_k, r_{k+1}), k = 0 the
                             most recent (Eq. 9: tau - tau_{n+1} .. tau - tau_n) */
} lc_box_desc;

typedef struct {
    int32_t n_boxes;              /* >= 1                                  */
    int32_t precision;            /* lc_precision                          */
    const lc_box_desc *boxes;     /* n_boxes entries (host)                */
    void *hip_stream;             /* hipStream_t; NULL = default stream    */
    void *workspace;              /* device memory, >= lc_workspace_bytes  */
    size_t workspace_bytes;
    int32_t use_graph;            /* 1: lc_step replays a captured graph   */
    int32_t autotune;             /* 1: lc_plan times every compiled launch
                                     shape of the tunable passes on this
                                     plan's buffers and keeps the fastest
                                     (see lc_schedule); 0: built-in choice */
} lc_plan_desc;

/* Radial factor phi_b (Eqs. 14-17). G = prefactor * phi / (4 pi r^2).
 *   kind 0: phi = 1
 *   kind 1: phi = max(0, a exp(-(r/s)^p) - c)            (continuous)
 *   kind 2: phi = a exp(-(r/s)^p) - c if r <= cut else 0  (Eq. 15 as printed,
 *           with s = 116.29 alpha and cut = 97.39 alpha)
 * Requires a, s, p > 0 for kinds 1-2; prefactor finite. */
typedef struct {
    int32_t kind;
    int32_t reserved;             /* must be 0 */
    double a, s, p, c, cut;
    double prefactor;             /* 1.0 for the bare 1/(4 pi r^2) dilution */
} lc_atten;

/* Sources of one slice (Eq. 17's sum of point luminosities, deposited to
 * the nearest grid point; several sources in a cell add).
 *   kind 0: dense grid, `grid` holds N^3 values in the grid layout above.
 *   kind 1: point list, n entries: cell[i] in [0, N^3) (flat index, int64),
 *           lum[i] of type `dtype`. A device point list is deposited with
 *           FP64 atomics (summation order of coincident sources varies).
 *   kind 2: positioned point list, n entries: `grid` points to 3n FP64
 *           positions (i, j, k axis order, k contiguous, in length units,
 *           any real values: wrapped periodically), lum[i] of type `dtype`;
 *           deposited to the nearest node, round(x / l) mod N. The same
 *           list feeds the near-field correction (lc_near_field).
 * `dtype` gives the value type of grid / lum, `mem` where they live. */
typedef struct {
    int32_t kind;
    int32_t dtype;                /* lc_dtype */
    int32_t mem;                  /* lc_mem   */
    int32_t reserved;             /* must be 0 */
    const void *grid;
    int64_t n;
    const int64_t *cell;
    const void *lum;
} lc_sources;

typedef struct lc_plan_s lc_plan_t;

/* Bytes of device workspace the plan needs (0 on an invalid descriptor;
 * the workspace fields of desc are ignored). Host only, no device call.
 * The storage follows the algorithm of Sec. 2.2: the transformed sources of
 * every lookback slice (step 4, kept for the slice sum of step 6), the
 * kernel spectra G^_{k,b} of every (slice, band) (step 3, precomputed once
 * and stored, as the paragraph after the algorithm proposes), one
 * accumulator spectrum per band, and builder scratch for step 2. */
size_t lc_workspace_bytes(const lc_plan_desc *desc);

/* Algorithm step 1: fix the box, the grid and the lookback slices of each
 * box (radii r_k of the shells [r_k, r_{k+1}), Eq. 9 and the shell of step
 * 2). Validates desc, carves the workspace, computes the FP64 host constants
 * (thresholds T_k, twiddle tables, self-cell averages) and uploads them.
 * Errors: LC_EINVAL (bad field), LC_EUNSUPPORTED (N not 2^a 3^b in
 * 8..512, m > 8, or r_0 = 0 with r_1 < (sqrt(3)/2) l so that the self
 * cell would straddle two slices), LC_ENOMEM (workspace too small or
 * misaligned to 256 bytes), LC_EDEVICE (no gfx950 device). A plan of
 * several boxes also creates up to three side streams (default priority) on
 * the current device for lc_step; lc_destroy releases them. */
int lc_plan(const lc_plan_desc *desc, lc_plan_t **out);

/* Build G_{k,b} for all K slices of one (box, band) - algorithm steps 2-3:
 * direct summation over images inside the shells (FP64), FP64 forward
 * transform, real part of its non-redundant octant kept (G is real and
 * even, so G^ is real and even). G^_{k,b}(0) is kept in FP64. Must be
 * called for every (box, band) before lc_field / lc_step. Enqueued on the
 * stream; uses the workspace's builder scratch. */
int lc_build_greens(lc_plan_t *plan, int32_t box, int32_t band, const lc_atten *atten);

/* Stage slice k of a box - algorithm step 4 up to the passes that do not
 * depend on the kernel: deposit (point list) or read (dense grid), then the
 * forward transform (x and y passes for LC_PREC_FP32, all three passes for
 * the unfused forms). Replaces whatever the slice held; slices never
 * pushed are zero. */
int lc_push_sources(lc_plan_t *plan, int32_t box, int32_t slice, const lc_sources *src);

/* Move the observing time forward by one slice (the paragraph after the
 * algorithm of Sec. 2.2: the field is wanted at a sequence of observing
 * times, and with slices of equal width aligned to the steps, the slice
 * that was lookback k becomes lookback k+1). The plan's slice spectra form
 * a ring: the oldest (lookback K-1) is dropped, every other slice moves one
 * lookback slot older without being transformed again, and `src` becomes
 * lookback slice 0 (step 4 for the new slice only). The kernels G^_{k,b}
 * stay attached to the lookback index; rebuild them with lc_build_greens
 * where they depend on the observing time (Eq. 17). A following lc_field
 * then costs one forward transform, the slice sum over all K slices and one
 * inverse per band. Errors as lc_push_sources; on error the ring is
 * unchanged. */
int lc_advance(lc_plan_t *plan, int32_t box, const lc_sources *src);

/* Evaluate the field - algorithm steps 5-6 with the slice sum taken in
 * spectral space (linearity; one inverse per band instead of one per
 * slice). box = -1 selects all boxes, band = -1 all bands. out holds one
 * pointer per selected (box, band), box-major, each to N^3 values of
 * `dtype` in `mem`. Errors: LC_ESTATE if a selected kernel is not built. */
int lc_field(lc_plan_t *plan, int32_t box, int32_t band, void *const *out,
             int32_t dtype, int32_t mem);

/* One whole step for every box - algorithm steps 4-6 for every slice and
 * band: push all slices from srcs (box-major, lookback order,
 * sum_b K_b entries, device memory only) and evaluate every band into out
 * (box-major, band, device memory). With use_graph = 1 the launch sequence
 * is captured in a HIP graph on first use and replayed while the argument
 * pointers are unchanged. With dense sources only, the boxes of a
 * multi-box plan run concurrently on the plan's stream and its side
 * streams, forked from and joined back to the plan's stream: as for every
 * call, the work is complete when the plan's stream reaches the end of the
 * call. Outputs of different boxes must not overlap. */
int lc_step(lc_plan_t *plan, const lc_sources *srcs, void *const *out, int32_t dtype);

/* Evaluate the field with the sources frozen at one lookback slice: every
 * slice k uses the sources of lookback slice `slice` (normally 0, the
 * observing time) while the kernels G^_{k,b} keep their retarded-time
 * shells and radial factors - the instantaneously affected field of Sec. 3
 * (Eq. 18). Same outputs, errors and ordering as lc_field;
 * LC_EINVAL if slice is outside [0, K) of a selected box. */
int lc_field_frozen(lc_plan_t *plan, int32_t box, int32_t band, int32_t slice, void *const *out,
                    int32_t dtype, int32_t mem);

/* Near-field (particle-mesh) correction of one band's field for sources
 * with positions inside their cells (Sec. 4: direct summation for nearby
 * sources, the FFT method for the far field). srcs holds the K slices'
 * positioned point lists (kind 2, device memory, lookback order; n = 0 for
 * none) that were pushed for the field in `out` (device, N^3 values of
 * `dtype`, as written by lc_field / lc_step for this box and band). For
 * every source s of slice k, nearest node c_s, and every node x = c_s + o
 * with 0 < max|o_d| <= near_cells, the mesh kernel's primary-image value
 * G_k(o) is replaced by the retarded kernel at the exact distance:
 *   out[x] += L_s (F_k(|x l - x_s|) - G^prim_k(o)),
 * F_k(r) = [r_k <= r < r_{k+1}] pref phi_k(r) / (4 pi r^2), and G^prim_k(o)
 * the m^3-subpoint average of the image u = 0 with the same shell rule as
 * the kernel. The source's own node keeps the cell-averaged mesh value.
 * Requires (near_cells + 1) sqrt(3) l < L/2 (one image), near_cells in
 * [1, 8]; corrections are summed with FP64 atomics (order varies).
 * Errors: LC_EINVAL, LC_ESTATE (band not built), LC_EUNSUPPORTED. */
int lc_near_field(lc_plan_t *plan, int32_t box, int32_t band, const lc_sources *srcs, int32_t near_cells,
                  void *out, int32_t dtype);

/* Fractional difference of two fields (Sec. 3, the comparison of the
 * instantaneous and the light-cone field): out[i] = (j_inst[i] - j[i]) / j[i]
 * where j[i] != 0, else 0. count values of `dtype` (LC_F32/LC_F64) in
 * device memory, computed in FP64 on hip_stream (NULL: default stream).
 * out may alias either input. */
int lc_fdiff(const void *j, const void *j_inst, void *out, int64_t count, int32_t dtype, void *hip_stream);

/* Background cosmology: a flat universe of matter and a cosmological
 * constant (Omega_L = 1 - omega_m), H0 = 100 h km/s/Mpc. */
typedef struct {
    double h;
    double omega_m;      /* (0, 1] */
} lc_cosmo;

/* Lookback slices of equal cosmic time dt_myr (Myr) before an observing
 * redshift z_obs (algorithm step 1 with the conformal time of Eqs. 4-5):
 * slice k covers cosmic times [t_obs - (k+1) dt, t_obs - k dt]; z_edge[k]
 * (K+1 values, may be NULL) is the redshift at t_obs - k dt, radii[k] (K+1
 * values) the comoving distance light travels from it to z_obs, c (tau_obs -
 * tau_k), in comoving Mpc (radii[0] = 0), and z_src[k] (K values, may be
 * NULL) the redshift at the slice's middle time t_obs - (k + 1/2) dt.
 * Host only. Errors: LC_EINVAL (bad cosmology, z_obs < 0, dt <= 0, K
 * outside [1, 1024], slices reaching t = 0). */
int lc_cosmo_slices(const lc_cosmo *c, double z_obs, double dt_myr, int32_t K, double *radii, double *z_edge,
                    double *z_src);

/* Lyman-Werner radial factors of K slices (Sec. 3): for source redshift
 * z_src[k], alpha_k of Eq. 16, the modulation of Eq. 15 with scale
 * 116.29 alpha_k and horizon 97.39 alpha_k (kind 2: as printed, hard cut;
 * kind 1: the continuous form max(0, .), whose zero lies 0.15% beyond the
 * printed horizon), and prefactor (1+z_obs)^3 / (1+z_src[k]) / (4 pi) so
 * that the kernel's 1/(4 pi r^2) completes Eq. 14's 1/((4 pi)^2 r^2). r is
 * in comoving Mpc, so the box length and radii must be too. The factor is
 * held fixed over each slice at its middle redshift. Host only. */
int lc_lw_factors(const lc_cosmo *c, double z_obs, int32_t K, const double *z_src, int32_t kind,
                  lc_atten *out);

/* As lc_build_greens with one radial factor per slice (per_slice[k], K
 * entries): the dilution factor of Eq. 8 depends on the source time as well
 * (Eq. 17: (1+z_s) and alpha(z_s)). The self cell of slice 0 uses
 * per_slice[0]. */
int lc_build_greens_slices(lc_plan_t *plan, int32_t box, int32_t band, const lc_atten *per_slice);

/* Non-finite source check (LC_ENONFINITE): every field evaluation reduces
 * each slice's sources in FP64 (the sum also gives the FP64 mean of the
 * FP32 form, S^_k(0) of Eq. 13) and flags a slice whose sum is NaN or
 * infinite. Synchronises the plan's stream, then returns LC_ENONFINITE if
 * any evaluation of box `box` (-1: all boxes) since the last check flagged
 * a slice, with the smallest flagged lookback index in *first_bad (may be
 * NULL; -1 when none), and clears the flags. lc_field with host outputs
 * performs the same check after its copies. */
int lc_check_sources(lc_plan_t *plan, int32_t box, int32_t *first_bad);

/* Size of the device scratch of lc_step_static, per GPU. */
#define LC_STATIC_SCRATCH_BYTES (128u * 1024u * 1024u)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one whole
 * step of one box - lc_plan, lc_build_greens for every band (atten[b]),
 * lc_step - with no workspace from the caller and no allocation. The plan's
 * buffers live in a static device array of LC_STATIC_SCRATCH_BYTES per GPU,
 * held until the process ends (looked up once per GPU on the first call on
 * it). desc: one box; workspace NULL, workspace_bytes 0, use_graph 0,
 * autotune 0 (built-in launch shapes). srcs, out, dtype as lc_step (device
 * memory). Work is enqueued on desc->hip_stream and the call synchronises
 * that stream before it returns. Every call on a GPU shares that GPU's
 * scratch and leaves its contents behind (each call clears what must start
 * at zero): calls that overlap on one GPU (several host threads, or streams
 * used by other callers at the same time) race and must be serialised by
 * the caller. Errors as lc_plan/lc_build_greens/lc_step, plus LC_ENOMEM when
 * the box needs more than LC_STATIC_SCRATCH_BYTES (lc_workspace_bytes of the
 * same desc) and LC_EINVAL for a caller workspace, several boxes, graphs or
 * autotuning. */
int lc_step_static(const lc_plan_desc *desc, const lc_atten *atten, const lc_sources *srcs, void *const *out,
                   int32_t dtype);

/* Release the plan's host state and its side streams (no caller memory is
 * freed). NULL is a no-op. */
void lc_destroy(lc_plan_t *plan);

/* Text of the last error on the calling thread; valid until the next
 * library call on this thread. Never NULL. */
const char *lc_last_error(void);

/* Largest |Im G^| / max|G^| seen by lc_build_greens for (box, band) (the
 * kernel spectrum is real up to rounding); synchronises the stream. */
int lc_greens_imag_ratio(lc_plan_t *plan, int32_t box, int32_t band, double *ratio);

/* Copy G^_{k,b}(0) = sum_c G_{k,b}(c) (FP64) for all K slices to host
 * memory dc[K]; synchronises the stream. */
int lc_greens_dc(lc_plan_t *plan, int32_t box, int32_t band, double *dc);

/* Kernels of the path, for lc_time_kernel. */
typedef enum {
    LC_KERNEL_X_FWD = 0,      /* forward x pass of one slice (reads the source grid) */
    LC_KERNEL_COL_Y_FWD = 1,  /* forward y pass of one slice, in place               */
    LC_KERNEL_COL_Z_FWD = 2,  /* forward z pass of one slice (unfused forms)          */
    LC_KERNEL_FUSED_Z = 3,    /* fused z pass + slice sum over all slices (FP32 form)  */
    LC_KERNEL_MAC = 4,        /* plain multiply-accumulate of one slice (unfused)     */
    LC_KERNEL_COL_Z_INV = 5,  /* inverse z pass of one band (unfused forms)           */
    LC_KERNEL_COL_Y_INV = 6,  /* inverse y pass of one band                           */
    LC_KERNEL_X_INV = 7,      /* inverse x pass + epilogue of one band                */
    LC_KERNEL_XY_FWD = 8,     /* fused forward x + y pass of one slice (FP32 form,
                                 N in {64, 96, 128, 192, 256}, where the step uses it
                                 in place of LC_KERNEL_X_FWD + LC_KERNEL_COL_Y_FWD)   */
    LC_KERNEL_YX_INV = 9      /* fused inverse y + x pass + epilogue of one band (FP32
                                 form with a parity-layout xy shape, where the step
                                 uses it in place of LC_KERNEL_COL_Y_INV +
                                 LC_KERNEL_X_INV)                                      */
} lc_kernel_id;

/* Launch shapes of one box's tunable passes (a6: radix schedule, columns
 * per tile and LDS layout are compiled per shape; the plan picks one).
 *   xy_variant     fused forward x + y pass: shape in [0, n_xy), or -1 for
 *                  separate x and y passes (always -1 when n_xy = 0). At
 *                  N = 256, shapes 4..6 take half a z-plane (the rows of one
 *                  parity) per workgroup and leave the y transforms of the
 *                  even and the odd rows apart (parity layout); the fused z
 *                  pass applies the last radix-2 step of the y transform.
 *   fused_variant  fused z pass register schedule in [0, n_fused)
 *                  (FP32 form; -1 in the other forms)
 *   fused_rounds   1: persistent workgroups take whole tiles in rounds; the
 *                  tiles left over after the last whole round are split by
 *                  slices over all workgroups and their parts merged by a
 *                  small kernel. 0: all (tile, slice) pairs are split evenly
 *                  between the workgroups; a tile's second part is merged by
 *                  the inverse y pass
 *   push_group     slices per batched forward launch in lc_step, 1..64
 *   fused_bands    bands that one fused z launch takes (each launch reads
 *                  the slice spectra once), 1..n_fused_bands (FP32 form; -1
 *                  in the other forms). With 1 or 2 the sum over slices is
 *                  compensated (Kahan); with 3 or 4 (N = 384, 512) it is a
 *                  plain FP32 sum. Default n_fused_bands; not tuned.
 *   spectra_3d     1: the slice spectra are stored transformed along z as
 *                  well (3D spectra, as in the plain forms): each push adds
 *                  the z pass, and a field is the product with G^ and the
 *                  sum over slices alone, then one inverse per band (the
 *                  regime of a rolling light-cone, where each observing
 *                  time pushes one slice and sums all K). Needs a
 *                  whole-plane xy shape. 0 (default): the fused z pass
 *                  transforms every slice along z at each field. FP32 form
 *                  only (-1 in the other forms); not tuned. The plan-time
 *                  autotuner times the fused schedules on the default
 *                  layout; with 3D spectra, time each fused_variant with
 *                  lc_time_kernel(LC_KERNEL_FUSED_Z) to pick one
 *   n_xy, n_fused, n_fused_bands  (lc_get_schedule only) shapes compiled
 *                  for this N/form; n_fused_bands = min(B, 4 at N = 384,
 *                  512, else 2)
 * lc_set_schedule validates every field (LC_EINVAL) and applies them to
 * later launches; the next lc_step captures a new graph. Changing whether
 * the fused xy pass is used, between whole-plane and parity-layout shapes,
 * or spectra_3d, clears the box's pushed slices (they read as zero until
 * pushed again). FP64 input grids (and point lists) use the first shape of the
 * same layout (0 or 4). */
typedef struct {
    int32_t xy_variant;
    int32_t fused_variant;
    int32_t fused_rounds;
    int32_t push_group;
    int32_t n_xy;
    int32_t n_fused;
    int32_t fused_bands;
    int32_t n_fused_bands;
    int32_t spectra_3d;
} lc_schedule;

int lc_get_schedule(lc_plan_t *plan, int32_t box, lc_schedule *out);
int lc_set_schedule(lc_plan_t *plan, int32_t box, const lc_schedule *s);

/* Diagnostic: launch one kernel of the path `reps` times back to back on
 * the plan's stream and return the mean duration per launch measured with
 * HIP events recorded on that stream. Per-slice kernels cycle over the
 * box's slices; LC_KERNEL_X_FWD and LC_KERNEL_XY_FWD read the dense device
 * grid most recently pushed for the slice (a zeroed scratch grid if none);
 * LC_KERNEL_XY_FWD runs in the step's configuration, min(push_group, K)
 * slices per launch (lc_schedule), and its time is per launch; per-band
 * kernels
 * use band 0 (the fused pass handles bands 0 .. fused_bands-1); the output of
 * LC_KERNEL_X_INV goes to the workspace scratch. Kernels must be built.
 * The plan's spectra and accumulators are left unspecified: push every
 * slice again before the next lc_field. Synchronises the stream.
 * Errors: LC_EINVAL (bad id, reps < 1, kernel not part of this plan's
 * form), LC_ESTATE (kernels not built). */
int lc_time_kernel(lc_plan_t *plan, int32_t box, int32_t kernel, int32_t reps, double *avg_ms);

#ifdef __cplusplus
}
#endif

#endif /* LC_H */
