// Internal interface between the host plan code and the HIP kernel
// launchers. Not installed; the public interface is include/lc.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lc {

// Spectrum of one real N^3 grid, x (contiguous) axis halved:
//   main: [z][y][p],  p in [0, N/2)      N*N*(N/2) complex
//   nyq : [z][y]      (p = N/2)          N*N complex
__host__ __device__ inline int64_t spec_main(int n) { return (int64_t)n * n * (n / 2); }
__host__ __device__ inline int64_t spec_elems(int n) { return spec_main(n) + (int64_t)n * n; }
// Kernel spectrum octant (real, folded |r|, |q| in [0, N/2]):
//   main: [r][q][p], p in [0, N/2)       H*H*(N/2) reals, H = N/2+1
//   nyq : [r][q]                         H*H reals
inline int64_t oct_main(int n) { int64_t h = n / 2 + 1; return h * h * (n / 2); }
inline int64_t oct_elems(int n) { int64_t h = n / 2 + 1; return h * h * (n / 2 + 1); }

bool supported_n(int n);

// Number of workgroups of the forward x pass with an FP32 spectrum (rows per
// WG depends on N; the row-batched pass at N = 512); the DC partial array of
// one slice has this many doubles.
int x_pass_wgs(int n);

// Source grid pointers of a batch of slices (passed by value as a kernel
// argument, so no device table has to be written before a launch).
struct SrcTab {
    static constexpr int kMax = 64;
    const void *p[kMax];
};

// Forward x pass of `count` slices: slice i reads in.p[i] and writes the
// spectrum at spec + i*spec_stride (complex elements); DC partials at
// dcpart + i*x_pass_wgs(n).
hipError_t launch_x_fwd_batch(int n, bool t_f64, const SrcTab &in, int count, bool in_f64, void *spec,
                              int64_t spec_stride, const void *tw_half, const void *twist, double *dcpart,
                              hipStream_t st);
// Fused forward x + y pass of `count` slices (FP32 form, N in {64, 96, 128,
// 192, 256}; xy_supported): one workgroup per z-plane. Slice i reads in.p[i],
// writes its y-transformed spectrum at spec + i*spec_stride and one FP64 sum
// of the input per plane at dcpart + i*dc_stride + z.
// `variant` selects one of xy_variants(n) compiled launch shapes (FP64
// input runs the first shape of the same layout).
// Parity-layout shapes (xy_parity) take half a plane per workgroup, the rows y of one
// parity s (y = 2m + s): rows r < N/2 of every z-plane of the spectrum then
// hold the N/2-point y transform E of the even rows and rows N/2 + r that
// of the odd rows O, so that the length-N y transform is
//   T[q] = E[q mod N/2] + W_N^q O[q mod N/2]
// (completed by the fused z pass, FusedArgs::parity), and the plane sums go
// to dcpart + i*dc_stride + 2z + s (2N per slice).
// Forward x pass alone with an FP32 spectrum for N = 512 (x_rows_supported):
// x_rows_wgs(n) workgroups per slice, each with one FP64 partial in dcpart
// (dcpart + i*x_rows_wgs(n) for slice i); otherwise as launch_x_fwd_batch.
bool x_rows_supported(int n);
int x_rows_wgs(int n);
hipError_t launch_x_rows_batch(int n, const SrcTab &in, int count, bool in_f64, void *spec, int64_t spec_stride,
                               const void *tw_half, const void *twist, double *dcpart, hipStream_t st);
bool xy_supported(int n);
int xy_variants(int n);
bool xy_parity(int n, int variant);
// Inverse y + x passes and epilogue of one band's FP32 accumulator in the
// parity layout left by the fused z pass with parity input (rows q and
// N/2 + q hold U_0 = T[q] + T[q+N/2] and U_1 = W_N^-q (T[q] - T[q+N/2])):
// out = IDFT(acc) * scale + *mu, N^3 reals (FP32 or FP64). With part
// non-null the second parts of split fused tiles (split_tab) are added.
bool yx_inv_supported(int n);
hipError_t launch_yx_inv(int n, const void *acc, void *out, bool out_f64, const void *tw_half, const void *twist,
                         const void *tw_full, double scale, const double *mu, const int *split_tab,
                         const void *part, hipStream_t st);
hipError_t launch_xy_fwd_batch(int n, const SrcTab &in, int count, bool in_f64, void *spec, int64_t spec_stride,
                               const void *tw_half, const void *twist, const void *tw_full, double *dcpart,
                               int64_t dc_stride, int variant, hipStream_t st);
// Column pass over `count` spectra at spec + i*stride (complex elements).
hipError_t launch_col_batch(int n, bool t_f64, int axis, bool fwd, void *spec, int64_t stride, int count,
                            const void *tw_full, hipStream_t st);

// Forward x pass: real rows -> main/nyq. in_f64 selects the input type,
// t_f64 the working precision. dcpart (nullable) receives one FP64 partial
// sum of the input per workgroup.
hipError_t launch_x_fwd(int n, bool t_f64, const void *in, bool in_f64, void *spec,
                        const void *tw_half, const void *twist, double *dcpart,
                        hipStream_t st);

// Inverse x pass + epilogue: out = scale * x + (mu ? *mu : 0), cast to out type.
hipError_t launch_x_inv(int n, bool t_f64, const void *spec, void *out, bool out_f64,
                        const void *tw_half, const void *twist, double scale, const double *mu,
                        hipStream_t st);

// Column pass along y (axis 1) or z (axis 2), forward or inverse, in place,
// main and nyq together. tw_full is the length-N table.
hipError_t launch_col(int n, bool t_f64, int axis, bool fwd, void *spec, const void *tw_full,
                      hipStream_t st);

// z forward pass of one FP32 spectrum `in` (y-transformed, whole-plane
// layout) into `out` in the tile order of the slice-sum pass (3D spectra,
// lc_schedule.spectra_3d): per column set, tiles of fused_cpw(n) columns
// (the last narrower), each tile's N rows contiguous. in != out.
hipError_t launch_col_z_tiled(int n, const void *in, void *out, const void *tw_full, hipStream_t st);

// Plain multiply-accumulate A (+)= G^ S over one slice (first: A = G^ S).
hipError_t launch_mac_plain(int n, bool t_f64, void *A, const void *S, const void *ghat, bool first,
                            hipStream_t st);

// Fused z pass for FP32: for each column of the y-transformed slices,
// forward z transform of every slice k < kcount[b], multiply by G^_{k,b},
// sum over k (compensated with one or two bands per launch, plain with
// three or four), inverse z transform, store to acc[b].
struct FusedArgs {
    const void *spec;        // K slices, stride spec_elems(n)
    int64_t spec_stride;
    const void *ghat;        // slice k band b at ghat + (k*B + b)*oct_stride
    int64_t oct_stride;
    int32_t K, B;            // slices, total bands in ghat layout
    int32_t band0, nband;    // bands handled by this launch (nband 1..fused_max_bands(n))
    int32_t kcount[4];       // slices with nonzero kernel, per handled band
    void *acc;               // handled band j at acc + j*acc_stride (complex elements)
    int64_t acc_stride;
    void *part;              // second parts of split tiles: [band j][slot][N*CPW] complex
    int64_t part_stride;     // per band, >= max_parts * N * CPW
    int64_t max_parts;       // slots available in part (caps the persistent grid)
    void *split_tab;         // int32 per tile: slot holding its second part, or -1 (written in
                             // stream-K mode only; the rounds mode splits no tile)
    int32_t zero_dc;         // 1: drop the (0,0,0) bin (FP64 mean added later)
    int32_t kahan;           // 1: compensated sum
    int32_t variant;         // register schedule: 0 default, 1 eight elements per thread
    int32_t rounds;          // 1: whole tiles in rounds instead of the balanced split
    int32_t parity;          // 1: spectra in the parity y layout of the half-plane xy shapes
    int32_t pre = 0;         // 1: spectra already transformed along z (3D): product and sum only
    int32_t ring = 0;        // lookback slice k is stored in spectrum slot (k + ring) mod K
    int32_t frozen = -1;     // >= 0: every lookback slice reads spectrum slot `frozen`
    // band means mu[band0 + j] = inv_n3 * sum_k g0[k B + band0 + j] sk[k] (the FP64
    // DC mode), reduced by the first workgroup when mu is non-null
    const double *sk = nullptr, *g0 = nullptr;
    double inv_n3 = 0.0;
    double *mu = nullptr;
};
int fused_variants(int n);   // number of register schedules compiled for n
bool fused_parity_supported(int n);   // parity-layout input compiled for n
int fused_default_variant(int n, int nband);   // built-in choice for 1 or 2 bands per launch
int fused_max_bands(int n);  // bands one fused launch can take: 4 at N = 384, 512, else 2
hipError_t launch_fused_z(int n, const FusedArgs &a, const void *tw_full, hipStream_t st);
int64_t fused_tiles(int n);  // column tiles of the fused pass (main + nyq)
int fused_cpw(int n);        // columns per tile

// Inverse y pass of an accumulator whose fused z pass split some tiles: the
// second parts (split_tab, part) are added while loading. FP32 only.
hipError_t launch_col_y_inv_combine(int n, void *spec, const void *tw_full, const int *split_tab,
                                    const void *part, hipStream_t st);

// Shell kernel builder (FP64): G_k on the octant, mirrored into a full N^3
// FP64 grid.
// Exact cell average (kernel rule 1, the m -> infinity limit of the subpoint
// average) of one shell: pref / l^3 times the integral of phi(r) / (4 pi r^2)
// over the part of an image cell inside [r_lo, r_sup), r_sup = min(r_{k+1},
// end of phi's support). gx, gw: 16-point Gauss-Legendre rule on [0, 1].
struct ExactRule {
    double l, r_lo, r_sup, pref;
    int32_t kind;
    double a, s, p, c;
    double gx[16], gw[16];
};

struct BuildArgs {
    double *grid;             // N^3 FP64
    int32_t n, m;
    double l, h;
    double t_lo, t_hi;        // thresholds of [r_k, r_{k+1})
    double r_lo, r_hi;
    int32_t images;           // |u_d| <= images
    int32_t self_pair;        // 1: the self pair is replaced (r_0 == 0)
    double self_val;          // added at cell 0 when this is slice 0 and self_pair
    int32_t kind;
    double a, s, p, c, cut, pref;
    int32_t rule;             // 0: m^3 subpoints; 1: exact cell average (ex)
    ExactRule ex;
};
hipError_t launch_greens_build(const BuildArgs &a, hipStream_t st);

// Fold the FP64 spectrum of G_k to the octant store of the plan precision,
// scaled by (conserve ? target / (l^3 Re G^(0)) : 1); writes G^(0) (after
// scaling) to *dc and folds max|Im|, max|Re| into maxima[0..1] (atomic).
hipError_t launch_greens_fold(int n, const void *spec64, void *oct, bool oct_f64, int conserve,
                              double target_over_l3, double *dc, unsigned long long *maxima,
                              hipStream_t st);

// Near-field (particle-mesh) correction of one slice: its shell, thresholds
// and radial factor.
struct NearArgs {
    int32_t n, m, R;           // grid side, subpoints per axis, near radius in cells
    double l, h;
    double t_lo, t_hi;         // T_k, T_{k+1}
    double r_lo, r_hi;         // r_k, r_{k+1}
    int32_t kind;
    double a, s, p, c, cut, pref;
    double *table;             // (R+1)^3 primary-image mesh kernel of the slice (device)
    double *corr;              // N^3 FP64 correction accumulator (device)
    int32_t rule;              // mesh kernel rule of the box (BuildArgs::rule)
    ExactRule ex;
};
hipError_t launch_near_table(const NearArgs &a, hipStream_t st);
hipError_t launch_near_corr(const NearArgs &a, int64_t n_pts, const double *pos, const void *lum, bool lum_f64,
                            hipStream_t st);
hipError_t launch_deposit_pos(double *grid, int64_t n_pts, const double *pos, const void *lum, bool lum_f64, int n,
                              double l, hipStream_t st);
hipError_t launch_add_grid(void *out, bool out_f64, const double *corr, int64_t count, hipStream_t st);

hipError_t launch_fill_f64(double *p, int64_t count, double v, hipStream_t st);
hipError_t launch_fill_bytes(void *p, int64_t bytes, hipStream_t st);   // zero, bytes % 4 == 0
hipError_t launch_deposit(double *grid, int64_t n_pts, const int64_t *cell, const void *lum,
                          bool lum_f64, int64_t n_cells, hipStream_t st);
// sk[s] = sum_w dcpart[s*W + w] for slots s < K (FP64 per-slice input sums;
// the fused z pass forms the band means from them, FusedArgs::mu). A slot
// whose sum is not finite increments status[0] and lowers status[1] to its
// lookback index (s - ring) mod K; status starts as {0, INT32_MAX}.
hipError_t launch_dc_reduce(const double *dcpart, int K, int W, double *sk, int *status, int ring, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t st);
// out = (j_inst - j) / j elementwise (0 where j == 0), FP64 arithmetic
hipError_t launch_fdiff(const void *j, const void *j_inst, void *out, int64_t count, bool f64, hipStream_t st);
// The same sums and check for the plain forms, read from the DC bin of each
// slot's fully transformed spectrum (spec + s*stride, complex FP64 or FP32):
// a NaN or infinity anywhere in a slice's sources reaches that bin.
hipError_t launch_spec_dc(const void *spec, bool f64, int64_t stride, int K, double *sk, int *status, int ring,
                          hipStream_t st);

}  // namespace lc
