// Host side of the C ABI (include/lc.h): descriptor validation, workspace
// layout, FP64 host constants and the launch sequences of the four calls.
//
// Host constants computed here in FP64 (or wider):
//  * slice thresholds T_k = (r_k/h)^2, h = L/(2 m N)   (exact shell membership)
//  * twiddle tables exp(-2 pi i j/L) from long double sin/cos
//  * the self-cell value: cube average of pref*phi/(4 pi r^2) over one cell,
//    reduced by the six-pyramid split to a face integral of
//    (l/2) Phi(R) / (4 pi R^3), Phi(R) = int_0^R phi; Phi of the attenuated
//    forms via the lower incomplete gamma function
//  * shell integrals int_{r_k}^{r_{k+1}} phi (for the conserve option)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lc.h"
#include "lc_internal.h"

using namespace lc;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() {
    g_err = "no error";
    return LC_OK;
}

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(LC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

constexpr size_t kAlign = 256;
// persistent workgroups of the fused pass can never exceed this (256 CUs x 8)
constexpr int64_t kMaxParts = 2048;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
// part slots a box's fused pass can use: one per persistent workgroup, and
// never more workgroups than tiles
int64_t fused_parts(int n) { return std::min<int64_t>(kMaxParts, fused_tiles(n)); }

// ---- special functions (host, FP64) ---------------------------------------

// lower incomplete gamma gamma(a, x) for a > 0, x >= 0
double lower_gamma(double a, double x) {
    if (x <= 0.0) return 0.0;
    if (x < a + 1.0) {
        // series: x^a e^-x sum_n x^n / (a (a+1) ... (a+n))
        double term = 1.0 / a, sum = term;
        for (int n = 1; n < 500; ++n) {
            term *= x / (a + n);
            sum += term;
            if (std::fabs(term) < 1e-18 * std::fabs(sum)) break;
        }
        return sum * std::exp(a * std::log(x) - x);
    }
    // continued fraction for the upper function (modified Lentz)
    const double tiny = 1e-300;
    double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 500; ++i) {
        const double an = -i * (i - a);
        b += 2.0;
        d = an * d + b;
        if (std::fabs(d) < tiny) d = tiny;
        c = b + an / c;
        if (std::fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        const double del = d * c;
        h *= del;
        if (std::fabs(del - 1.0) < 1e-17) break;
    }
    const double upper = std::exp(a * std::log(x) - x) * h;
    return std::tgamma(a) - upper;
}

struct Atten {
    int kind;
    double a, s, p, c, cut, pref;
};

// end of the support of phi (first radius beyond which phi vanishes)
double support_end(const Atten &at) {
    if (at.kind == 0) return INFINITY;
    if (at.kind == 2) return at.cut;
    if (at.c <= 0.0) return INFINITY;
    if (at.a <= at.c) return 0.0;
    return at.s * std::pow(std::log(at.a / at.c), 1.0 / at.p);
}

// Phi(R) = int_0^R phi: for kinds 1-2, int_0^U a e^{-(r/s)^p} dr - c U with
// U = min(R, support end); the first term is a (s/p) gamma(1/p, (U/s)^p).
double Phi(const Atten &at, double R) {
    if (R <= 0.0) return 0.0;
    if (at.kind == 0) return R;
    const double U = std::min(R, support_end(at));
    if (U <= 0.0) return 0.0;
    return at.a * (at.s / at.p) * lower_gamma(1.0 / at.p, std::pow(U / at.s, at.p)) - at.c * U;
}

// Gauss-Legendre rule on [0, 1] (Newton on the three-term recurrence)
void gauss01(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        long double z = std::cos(pi * (i + 0.75L) / (n + 0.5L)), dp = 0;
        for (int it = 0; it < 60; ++it) {
            long double p1 = 1, p2 = 0;
            for (int j = 1; j <= n; ++j) {
                long double p3 = p2;
                p2 = p1;
                p1 = ((2 * j - 1) * z * p2 - (j - 1) * p3) / j;
            }
            dp = n * (z * p1 - p2) / (z * z - 1);
            long double dz = p1 / dp;
            z -= dz;
            if (std::fabs((double)dz) < 1e-19) break;
        }
        {
            long double p1 = 1, p2 = 0;
            for (int j = 1; j <= n; ++j) {
                long double p3 = p2;
                p2 = p1;
                p1 = ((2 * j - 1) * z * p2 - (j - 1) * p3) / j;
            }
            dp = n * (z * p1 - p2) / (z * z - 1);
        }
        x[i] = (double)(0.5L * (1 - z));
        w[i] = (double)(1.0L / ((1 - z * z) * dp * dp));   // 2/(..) on [-1,1], halved
    }
}

// Cube average of pref * phi / (4 pi r^2) over a cell of side l.
double self_cell(const Atten &at, double l) {
    const double pi = 3.141592653589793238462643383279502884;
    std::vector<double> x, w;
    if (at.kind == 0) {
        // (3 / (pi l^2)) J2, J2 = int_0^1 atan(1/sqrt(1+y^2)) / sqrt(1+y^2) dy
        gauss01(40, x, w);
        double j2 = 0.0;
        for (int i = 0; i < 40; ++i) {
            const double a = std::sqrt(1.0 + x[i] * x[i]);
            j2 += w[i] * std::atan(1.0 / a) / a;
        }
        return at.pref * 3.0 * j2 / (pi * l * l);
    }
    // (3 / (2 pi l^3)) * 4 * int_0^{l/2} int_0^{l/2} (l/2) Phi(R) / R^3, on 2 x 2 panels
    gauss01(24, x, w);
    const double hl = 0.5 * l, hp = 0.5 * hl;
    double acc = 0.0;
    for (int py = 0; py < 2; ++py)
        for (int pz = 0; pz < 2; ++pz)
            for (int i = 0; i < 24; ++i) {
                const double y = hp * (py + x[i]);
                for (int j = 0; j < 24; ++j) {
                    const double z = hp * (pz + x[j]);
                    const double R = std::sqrt(hl * hl + y * y + z * z);
                    acc += w[i] * w[j] * hl * Phi(at, R) / (R * R * R);
                }
            }
    acc *= hp * hp;
    return at.pref * 3.0 * 4.0 * acc / (2.0 * pi * l * l * l);
}

// ---- twiddle tables -----------------------------------------------------------

// exp(-2 pi i j / L) for j in [0, count), as (re, im) doubles
void twiddles64(int L, int count, double *out) {
    const long double pi2 = 6.283185307179586476925286766559005768L;
    for (int j = 0; j < count; ++j) {
        const long double ang = pi2 * (long double)j / (long double)L;
        out[2 * j] = (double)cosl(ang);
        out[2 * j + 1] = (double)(-sinl(ang));
    }
}

// same in FP32 arithmetic throughout (the plain FP32 form)
void twiddles32_plain(int L, int count, float *out) {
    const float pi2 = 6.28318530717958647692f;
    for (int j = 0; j < count; ++j) {
        const float ang = pi2 * (float)j / (float)L;
        out[2 * j] = cosf(ang);
        out[2 * j + 1] = -sinf(ang);
    }
}

bool is_2a3b(int n) {
    if (n <= 0) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

}  // namespace

// ---- plan --------------------------------------------------------------------

struct BoxPlan {
    int n = 0, K = 0, B = 0, m = 1, conserve = 0;
    int rule = 0;                // mesh kernel: 0 m^3 subpoints, 1 exact cell average
    // ring of slice spectra: lookback slice k is stored in slot (head + k) mod K
    // (lc_advance moves the head back by one, making the oldest slot the newest)
    int head = 0;
    int slot(int k) const { const int s = head + k; return s >= K ? s - K : s; }
    double L = 0, l = 0, h = 0;
    std::vector<double> radii, T;
    std::vector<int> built, kcount;
    std::vector<std::vector<Atten>> att;   // per band, per slice: the radial factors of the last build
    std::vector<uint8_t> pushed;          // per slot
    // dense device sources of the most recent push of each slot (diagnostic timing)
    std::vector<const void *> last_src;
    std::vector<uint8_t> last_src_f64;
    // device regions
    char *spec = nullptr, *acc = nullptr, *ghat = nullptr;
    double *ghat0 = nullptr, *dcpart = nullptr, *mu = nullptr, *sk = nullptr;
    // non-finite source sums seen by the DC reduction since the last query:
    // {count, smallest lookback index} (device, {0, INT32_MAX} when clear)
    int *status = nullptr;
    char *part = nullptr;        // FP32 form: second parts of split fused tiles, per band of a launch
    int *split_tab = nullptr;    // per fused launch of a field: tile -> part slot
    int64_t max_parts = 0, part_stride = 0, tiles = 0;
    int fused_variant = 0, fused_rounds = 1;
    int fused_bands = 1;         // bands per fused z launch (3-4: plain sums)
    // FP32 form: slice spectra stored transformed along z too (3D), so that a
    // field is the product and sum alone; every push adds the z pass
    bool spec3d = false;
    int xy_variant = 0;          // launch shape of the fused xy pass
    int push_group = 2;          // slices per batched forward launch in lc_step
    unsigned long long *maxima = nullptr;
    char *tw_half = nullptr, *tw_full = nullptr, *twist = nullptr;       // plan precision
    char *tw64_half = nullptr, *tw64_full = nullptr, *twist64 = nullptr; // FP64 (builder)
    int xwgs = 0;
    // FP32 form at N in {64, 96, 128, 192, 256}: x and y passes fused per plane
    bool use_xy = false;
    int dcw = 0;                 // FP64 DC partials per slice (x-pass workgroups, planes or half planes)
    // spectra in the parity y layout (half-plane xy shapes), completed by the fused z pass
    bool parity() const { return use_xy && xy_parity(n, xy_variant); }
    int dc_width() const { return use_xy ? (parity() ? 2 : 1) * n : xwgs; }
    int64_t dc_cap() const { return std::max<int64_t>(2 * (int64_t)n, xwgs); }   // dcpart entries per slice
};

struct lc_plan_s {
    int prec = LC_PREC_FP64;
    bool t_f64 = true;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int use_graph = 0;
    std::vector<BoxPlan> boxes;
    char *scratch_real = nullptr;    // FP64 N^3: builder grid / source staging / host-output staging
    char *scratch_spec = nullptr;    // FP64 spectrum for the builder
    // graph cache for lc_step
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<uint8_t> gkey;
    // side streams (default priority, created by the plan) on which lc_step
    // runs the boxes of a multi-box plan concurrently, forked from and joined
    // back to the plan's stream with events
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_done;
    hipEvent_t fork = nullptr;
    ~lc_plan_s() {
        for (hipEvent_t e : side_done) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        for (hipStream_t t : side) (void)hipStreamDestroy(t);
    }
};

namespace {

struct Layout {
    size_t total = 0;
    struct BoxOff {
        size_t spec, acc, ghat, ghat0, dcpart, mu, sk, status, part, split_tab, maxima, tw_half, tw_full, twist,
            tw64_half, tw64_full, twist64;
    };
    std::vector<BoxOff> box;
    size_t scratch_real = 0, scratch_spec = 0;
};

int validate(const lc_plan_desc *d) {
    if (!d) return fail(LC_EINVAL, "descriptor is NULL");
    if (d->autotune != 0 && d->autotune != 1) return fail(LC_EINVAL, "autotune must be 0 or 1");
    if (d->n_boxes < 1 || d->n_boxes > 4096) return fail(LC_EINVAL, "n_boxes must be in [1, 4096]");
    if (!d->boxes) return fail(LC_EINVAL, "boxes is NULL");
    if (d->precision != LC_PREC_FP64 && d->precision != LC_PREC_FP32_PLAIN && d->precision != LC_PREC_FP32)
        return fail(LC_EINVAL, "unknown precision %d", d->precision);
    if (d->use_graph != 0 && d->use_graph != 1) return fail(LC_EINVAL, "use_graph must be 0 or 1");
    for (int b = 0; b < d->n_boxes; ++b) {
        const lc_box_desc &x = d->boxes[b];
        if (x.rule != 0 && x.rule != 1) return fail(LC_EINVAL, "box %d: rule must be 0 or 1", b);
        if (x.n < 8 || x.n > 512 || (x.n % 2) || !is_2a3b(x.n) || !supported_n(x.n))
            return fail(LC_EUNSUPPORTED, "box %d: N=%d is not compiled in (even, 2^a 3^b, 8..512)", b, x.n);
        if (x.n_slices < 1 || x.n_slices > 1024)
            return fail(LC_EINVAL, "box %d: n_slices must be in [1, 1024]", b);
        if (x.n_bands < 1 || x.n_bands > 64) return fail(LC_EINVAL, "box %d: n_bands must be in [1, 64]", b);
        if (x.supersample < 1 || x.supersample > 8)
            return fail(LC_EUNSUPPORTED, "box %d: supersample must be in [1, 8]", b);
        if (x.conserve != 0 && x.conserve != 1) return fail(LC_EINVAL, "box %d: conserve must be 0 or 1", b);
        if (!(x.box > 0.0) || !std::isfinite(x.box)) return fail(LC_EINVAL, "box %d: box length must be > 0", b);
        if (!x.radii) return fail(LC_EINVAL, "box %d: radii is NULL", b);
        for (int k = 0; k <= x.n_slices; ++k)
            if (!std::isfinite(x.radii[k])) return fail(LC_EINVAL, "box %d: radius %d not finite", b, k);
        if (x.radii[0] < 0.0) return fail(LC_EINVAL, "box %d: r_0 must be >= 0", b);
        for (int k = 0; k < x.n_slices; ++k)
            if (!(x.radii[k + 1] > x.radii[k]))
                return fail(LC_EINVAL, "box %d: radii must be strictly increasing", b);
        const double l = x.box / x.n;
        // (the exact cell average splits the source's own cell between shells)
        if (x.rule == 0 && x.radii[0] == 0.0 && x.radii[1] < 0.5 * std::sqrt(3.0) * l)
            return fail(LC_EUNSUPPORTED,
                        "box %d: r_1 = %g < (sqrt 3 / 2) l = %g: the self cell would straddle slices", b,
                        x.radii[1], 0.5 * std::sqrt(3.0) * l);
        // image range and exact-integer headroom
        const double U = std::ceil(x.radii[x.n_slices] / x.box) + 1.0;
        const double qmax = 2.0 * x.supersample * (U + 1.0) * x.n + x.supersample;
        if (3.0 * qmax * qmax > 9.0e15)
            return fail(LC_EUNSUPPORTED, "box %d: outer radius too large for exact distances", b);
        if (U > 64) return fail(LC_EUNSUPPORTED, "box %d: outer radius spans more than 63 box lengths", b);
    }
    return LC_OK;
}

Layout layout_of(const lc_plan_desc *d) {
    Layout lay;
    const bool f64 = d->precision == LC_PREC_FP64;
    const size_t cs = f64 ? 16 : 8, rs = f64 ? 8 : 4;
    size_t off = 0, max_real = 0, max_spec = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    for (int b = 0; b < d->n_boxes; ++b) {
        const lc_box_desc &x = d->boxes[b];
        const int n = x.n, K = x.n_slices, B = x.n_bands;
        Layout::BoxOff o;
        o.spec = take((size_t)K * spec_elems(n) * cs);
        o.acc = take((size_t)B * spec_elems(n) * cs);
        o.ghat = take((size_t)K * B * oct_elems(n) * rs);
        o.ghat0 = take((size_t)K * B * 8);
        o.dcpart = take((size_t)K * std::max(x_pass_wgs(n), 2 * n) * 8);
        o.mu = take((size_t)B * 8);
        o.sk = take((size_t)K * 8);
        o.status = take(2 * sizeof(int32_t));
        if (d->precision == LC_PREC_FP32) {
            o.part = take((size_t)std::min(B, fused_max_bands(n)) * fused_parts(n) * n * fused_cpw(n) * 8);
            o.split_tab = take((size_t)B * fused_tiles(n) * 4);
        } else {
            o.part = o.split_tab = 0;
        }
        o.maxima = take((size_t)B * 2 * 8);
        o.tw_half = take((size_t)(n / 2) * cs);
        o.tw_full = take((size_t)n * cs);
        o.twist = take((size_t)(n / 2) * cs);
        o.tw64_half = take((size_t)(n / 2) * 16);
        o.tw64_full = take((size_t)n * 16);
        o.twist64 = take((size_t)(n / 2) * 16);
        lay.box.push_back(o);
        max_real = std::max(max_real, (size_t)n * n * n * 8);
        max_spec = std::max(max_spec, (size_t)spec_elems(n) * 16);
    }
    lay.scratch_real = take(max_real);
    lay.scratch_spec = take(max_spec);
    lay.total = off;
    return lay;
}

int check_device() {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) return fail(LC_EDEVICE, "no HIP device available");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(LC_EDEVICE, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(LC_EDEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(LC_EDEVICE, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
    return LC_OK;
}

int upload(void *dst, const void *src, size_t bytes, hipStream_t st) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return LC_OK;
}

Atten atten_of(const lc_atten *a) {
    Atten r;
    r.kind = a->kind; r.a = a->a; r.s = a->s; r.p = a->p; r.c = a->c; r.cut = a->cut;
    r.pref = a->prefactor;
    return r;
}

int valid_sources(const BoxPlan &bp, const lc_sources *s) {
    if (!s) return fail(LC_EINVAL, "sources is NULL");
    if (s->reserved != 0) return fail(LC_EINVAL, "sources.reserved must be 0");
    if (s->dtype != LC_F32 && s->dtype != LC_F64) return fail(LC_EINVAL, "bad source dtype");
    if (s->mem != LC_MEM_HOST && s->mem != LC_MEM_DEVICE) return fail(LC_EINVAL, "bad source mem");
    if (s->kind == 0) {
        if (!s->grid) return fail(LC_EINVAL, "dense source grid is NULL");
    } else if (s->kind == 1) {
        if (s->n < 0) return fail(LC_EINVAL, "point count must be >= 0");
        if (s->n > 0 && (!s->cell || !s->lum)) return fail(LC_EINVAL, "point list pointers are NULL");
        if (s->mem == LC_MEM_HOST) {
            const int64_t n3 = (int64_t)bp.n * bp.n * bp.n;
            for (int64_t i = 0; i < s->n; ++i)
                if (s->cell[i] < 0 || s->cell[i] >= n3)
                    return fail(LC_EINVAL, "point %lld: cell %lld outside [0, N^3)", (long long)i,
                                (long long)s->cell[i]);
        }
    } else if (s->kind == 2) {
        if (s->n < 0) return fail(LC_EINVAL, "point count must be >= 0");
        if (s->n > 0 && (!s->grid || !s->lum)) return fail(LC_EINVAL, "positioned point list pointers are NULL");
        if (s->mem == LC_MEM_HOST) {
            const double *pos = (const double *)s->grid;
            for (int64_t i = 0; i < 3 * s->n; ++i)
                if (!std::isfinite(pos[i])) return fail(LC_EINVAL, "point %lld: position not finite", (long long)(i / 3));
        }
    } else {
        return fail(LC_EINVAL, "unknown source kind %d", s->kind);
    }
    return LC_OK;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// Mean milliseconds per call of `launch`: one warm-up call, then `reps`
// calls between two events recorded on the plan's stream.
template <typename F> int time_calls(hipStream_t st, int reps, F &&launch, double *ms) {
    HIPCHK(launch());
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) HIPCHK(launch());
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)t / reps;
    return LC_OK;
}

// Inverse y pass of an FP32 accumulator after the fused z pass: the stream-K
// mode's split tiles are merged while loading; the rounds mode splits none.
hipError_t inv_y_fused(int n, void *acc, const void *tw_full, const int *tab, const void *part, bool rounds,
                       hipStream_t st) {
    return rounds ? launch_col(n, false, 1, false, acc, tw_full, st)
                  : launch_col_y_inv_combine(n, acc, tw_full, tab, part, st);
}

FusedArgs fused_args(const BoxPlan &bp) {
    FusedArgs fa;
    const int n = bp.n;
    fa.spec = bp.spec; fa.spec_stride = spec_elems(n); fa.ghat = bp.ghat; fa.oct_stride = oct_elems(n);
    fa.K = bp.K; fa.B = bp.B; fa.band0 = 0; fa.nband = bp.fused_bands;
    for (int j = 0; j < 4; ++j) fa.kcount[j] = j < fa.nband ? bp.kcount[j] : 0;
    fa.acc = bp.acc; fa.acc_stride = spec_elems(n); fa.zero_dc = 1; fa.kahan = fa.nband <= 2;
    fa.part = bp.part; fa.part_stride = bp.part_stride; fa.max_parts = bp.max_parts;
    fa.split_tab = bp.split_tab;
    fa.variant = bp.fused_variant;
    fa.rounds = bp.fused_rounds;
    fa.parity = bp.parity() ? 1 : 0;
    fa.pre = bp.spec3d ? 1 : 0;
    return fa;
}

// Forward launch (fused xy pass with shape xyv >= 0, else x + y passes) of
// `cnt` slices starting at output slice k0 of the box; the inputs are other
// slices' spectrum memory read as FP32 grids (K >= 2 cnt), so successive
// timed launches stream distinct memory as in a step.
hipError_t tune_forward(lc_plan_t *p, BoxPlan &bp, int xyv, int cnt, int k0) {
    const int n = bp.n;
    const int64_t se = spec_elems(n);
    SrcTab tab;
    // inputs: the spectrum memory of other slices, read as FP32 grids (a
    // slice's spectrum is larger than a grid). With cnt > K/2 some inputs
    // are also outputs of the same launch; the values are then meaningless
    // but every access stays inside the spectrum store, and the run time
    // does not depend on them.
    for (int j = 0; j < cnt; ++j)
        tab.p[j] = bp.K > 1 ? (const void *)(bp.spec + (size_t)((k0 + j + std::max(cnt, bp.K / 2)) % bp.K) * se * 8)
                            : (const void *)p->scratch_real;
    char *out = bp.spec + (size_t)k0 * se * 8;
    double *dcp = bp.dcpart + (size_t)k0 * bp.dc_cap();
    if (xyv >= 0)
        return launch_xy_fwd_batch(n, tab, cnt, false, out, se, bp.tw_half, bp.twist, bp.tw_full, dcp, bp.dc_cap(),
                                   xyv, p->stream);
    hipError_t e = launch_x_fwd_batch(n, false, tab, cnt, false, out, se, bp.tw_half, bp.twist, dcp, p->stream);
    if (e != hipSuccess) return e;
    return launch_col_batch(n, false, 1, true, out, se, cnt, bp.tw_full, p->stream);
}

// Plan-time choice of the launch shapes of one FP32-form box (a6): every
// compiled shape of the forward pass, the batching of the forward launches
// and the fused z pass schedule is timed on this plan's buffers (all zero
// at this point; the kernels' run time does not depend on the values).
// The forward shapes come in two spectrum layouts (whole planes, or the
// parity layout of the half-plane shapes, which the fused z pass completes
// at some cost), so the fastest forward shape and fused schedule are found
// per layout and the layout with the least K * (forward time per slice) +
// (fused pass time) is kept. Spectra and DC partials are cleared afterwards.
// Candidates are visited from the preferred end (lower shape numbers) and
// replace the current choice only when at least 2% faster, so that shapes
// within timing noise of each other do not change the choice from one plan
// to the next.
constexpr double kTuneMargin = 0.98;

// Shapes chosen by autotune_box, kept for the life of the process and reused
// by later plans with the same device, grid side, slice count and bands per
// fused launch (the trial launches take ~0.1-1 s per plan).
struct TunedShape {
    int xy_variant, push_group, fused_variant, fused_rounds;
};
using TuneKey = std::tuple<int, int, int, int>;   // device, N, K, bands per fused launch
std::mutex g_tune_mu;
std::map<TuneKey, TunedShape> g_tuned;

int autotune_box_uncached(lc_plan_t *p, BoxPlan &bp);

int autotune_box(lc_plan_t *p, BoxPlan &bp) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    const TuneKey key{dev, bp.n, bp.K, bp.fused_bands};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            bp.xy_variant = it->second.xy_variant;
            bp.push_group = it->second.push_group;
            bp.fused_variant = it->second.fused_variant;
            bp.fused_rounds = it->second.fused_rounds;
            bp.dcw = bp.dc_width();
            return LC_OK;
        }
    }
    int rc = autotune_box_uncached(p, bp);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = TunedShape{bp.xy_variant, bp.push_group, bp.fused_variant, bp.fused_rounds};
    return LC_OK;
}

int autotune_box_uncached(lc_plan_t *p, BoxPlan &bp) {
    const int n = bp.n;
    const int reps = 3;
    double ms = 0.0;
    int rot = 0;
    // forward pass shape and slices per launch, jointly (per slice time), per layout
    double fwd_best[2] = {1e30, 1e30};
    int fwd_v[2] = {-1, -1}, fwd_g[2] = {bp.push_group, bp.push_group};
    bool fwd_seen[2] = {false, false};
    {
        // all slices (up to the table size) in one launch: smaller groups
        // changed the per-slice time by about 1%, less than the trial-to-trial
        // spread, so tuning the grouping only made the choice unstable
        std::vector<int> cands{std::min(bp.K, SrcTab::kMax)};
        for (int v = bp.use_xy ? 0 : -1; v < (bp.use_xy ? xy_variants(n) : 0); ++v) {
            const int lay = v >= 0 && xy_parity(n, v) ? 1 : 0;
            if (lay == 1 && !fused_parity_supported(n)) continue;
            for (int g : cands) {
                int rc = time_calls(p->stream, reps, [&]() {
                    const int k0 = (rot++ * g) % std::max(1, bp.K - g + 1);
                    return tune_forward(p, bp, v, g, k0);
                }, &ms);
                if (rc) return rc;
                fwd_seen[lay] = true;
                if (ms / g < kTuneMargin * fwd_best[lay]) { fwd_best[lay] = ms / g; fwd_v[lay] = v; fwd_g[lay] = g; }
            }
        }
    }
    // fused z pass schedule and scheduling mode (with the inverse y pass
    // that merges split tiles), per layout
    double fz_best[2] = {1e30, 1e30};
    int fz_v[2] = {bp.fused_variant, bp.fused_variant}, fz_r[2] = {bp.fused_rounds, bp.fused_rounds};
    for (int lay = 0; lay < 2; ++lay) {
        if (!fwd_seen[lay]) continue;
        for (int v = 0; v < fused_variants(n); ++v)
            for (int r = 1; r >= 0; --r) {
                bp.fused_variant = v;
                bp.fused_rounds = r;
                FusedArgs fa = fused_args(bp);
                fa.parity = lay;
                // with the layout's own inverse pass (fused inverse y + x for the
                // parity layout; the inverse y pass otherwise, the x pass being
                // the same in both)
                int rc = time_calls(p->stream, 2, [&]() {
                    hipError_t e = launch_fused_z(n, fa, bp.tw_full, p->stream);
                    if (e != hipSuccess) return e;
                    if (lay)
                        return launch_yx_inv(n, bp.acc, p->scratch_real, false, bp.tw_half, bp.twist, bp.tw_full,
                                             1.0, bp.mu, bp.split_tab, r ? nullptr : bp.part, p->stream);
                    e = inv_y_fused(n, bp.acc, bp.tw_full, bp.split_tab, bp.part, r != 0, p->stream);
                    if (e != hipSuccess) return e;
                    return launch_x_inv(n, false, bp.acc, p->scratch_real, false, bp.tw_half, bp.twist, 1.0, nullptr,
                                        p->stream);
                }, &ms);
                if (rc) return rc;
                if (ms < kTuneMargin * fz_best[lay]) { fz_best[lay] = ms; fz_v[lay] = v; fz_r[lay] = r; }
            }
    }
    const int lay = fwd_seen[1] && (!fwd_seen[0] || bp.K * fwd_best[1] + fz_best[1] < bp.K * fwd_best[0] + fz_best[0])
                        ? 1 : 0;
    bp.xy_variant = fwd_v[lay] >= 0 ? fwd_v[lay] : 0;
    bp.push_group = fwd_g[lay];
    bp.fused_variant = fz_v[lay];
    bp.fused_rounds = fz_r[lay];
    bp.dcw = bp.dc_width();
    const size_t cs = 8;
    HIPCHK(launch_fill_bytes(bp.spec, (int64_t)bp.K * spec_elems(n) * cs, p->stream));
    HIPCHK(launch_fill_f64(bp.dcpart, (int64_t)bp.K * bp.dc_cap(), 0.0, p->stream));
    return LC_OK;
}

}  // namespace

extern "C" {

size_t lc_workspace_bytes(const lc_plan_desc *desc) {
    if (validate(desc) != LC_OK) return 0;
    ok();
    return layout_of(desc).total;
}

int lc_plan(const lc_plan_desc *d, lc_plan_t **out) {
    if (!out) return fail(LC_EINVAL, "out is NULL");
    int rc = validate(d);
    if (rc) return rc;
    const Layout lay = layout_of(d);
    if (!d->workspace) return fail(LC_EINVAL, "workspace is NULL");
    if (((uintptr_t)d->workspace) % kAlign) return fail(LC_ENOMEM, "workspace must be 256-byte aligned");
    if (d->workspace_bytes < lay.total)
        return fail(LC_ENOMEM, "workspace of %zu bytes < %zu required", d->workspace_bytes, lay.total);
    if ((rc = check_device())) return rc;

    std::unique_ptr<lc_plan_s> p(new lc_plan_s());
    p->prec = d->precision;
    p->t_f64 = d->precision == LC_PREC_FP64;
    p->stream = (hipStream_t)d->hip_stream;
    p->ws = (char *)d->workspace;
    p->ws_bytes = d->workspace_bytes;
    p->use_graph = d->use_graph;
    p->scratch_real = p->ws + lay.scratch_real;
    p->scratch_spec = p->ws + lay.scratch_spec;
    const size_t cs = p->t_f64 ? 16 : 8;
    for (int b = 0; b < d->n_boxes; ++b) {
        const lc_box_desc &x = d->boxes[b];
        const Layout::BoxOff &o = lay.box[b];
        BoxPlan bp;
        bp.n = x.n; bp.K = x.n_slices; bp.B = x.n_bands; bp.m = x.supersample; bp.conserve = x.conserve;
        bp.rule = x.rule;
        bp.L = x.box;
        bp.l = x.box / x.n;
        bp.h = x.box / (2.0 * x.supersample * x.n);
        bp.radii.assign(x.radii, x.radii + x.n_slices + 1);
        bp.T.resize(bp.K + 1);
        for (int k = 0; k <= bp.K; ++k) {
            const double q = bp.radii[k] / bp.h;
            bp.T[k] = q * q;
        }
        bp.built.assign(bp.B, 0);
        bp.att.assign(bp.B, std::vector<Atten>());
        bp.kcount.assign(bp.B, bp.K);
        bp.pushed.assign(bp.K, 0);
        bp.last_src.assign(bp.K, nullptr);
        bp.last_src_f64.assign(bp.K, 0);
        bp.spec = p->ws + o.spec; bp.acc = p->ws + o.acc; bp.ghat = p->ws + o.ghat;
        bp.ghat0 = (double *)(p->ws + o.ghat0); bp.dcpart = (double *)(p->ws + o.dcpart);
        bp.mu = (double *)(p->ws + o.mu); bp.sk = (double *)(p->ws + o.sk);
        bp.status = (int *)(p->ws + o.status);
        if (p->prec == LC_PREC_FP32) {
            bp.part = p->ws + o.part;
            bp.split_tab = (int *)(p->ws + o.split_tab);
            bp.max_parts = fused_parts(x.n);
            bp.part_stride = bp.max_parts * x.n * fused_cpw(x.n);
            bp.tiles = fused_tiles(x.n);
            bp.fused_bands = std::min(x.n_bands, fused_max_bands(x.n));
            bp.fused_variant = fused_default_variant(x.n, bp.fused_bands);
        }
        bp.maxima = (unsigned long long *)(p->ws + o.maxima);
        bp.tw_half = p->ws + o.tw_half; bp.tw_full = p->ws + o.tw_full; bp.twist = p->ws + o.twist;
        bp.tw64_half = p->ws + o.tw64_half; bp.tw64_full = p->ws + o.tw64_full;
        bp.twist64 = p->ws + o.twist64;
        bp.xwgs = x_pass_wgs(bp.n);
        bp.use_xy = p->prec == LC_PREC_FP32 && xy_supported(bp.n);
        bp.dcw = bp.dc_width();

        // tables
        const int n = bp.n;
        std::vector<double> th(n), tf(2 * n), tt(n);
        twiddles64(n / 2, n / 2, th.data());
        twiddles64(n, n, tf.data());
        twiddles64(n, n / 2, tt.data());
        if ((rc = upload(bp.tw64_half, th.data(), (size_t)n / 2 * 16, p->stream))) return rc;
        if ((rc = upload(bp.tw64_full, tf.data(), (size_t)n * 16, p->stream))) return rc;
        if ((rc = upload(bp.twist64, tt.data(), (size_t)n / 2 * 16, p->stream))) return rc;
        if (p->t_f64) {
            if ((rc = upload(bp.tw_half, th.data(), (size_t)n / 2 * 16, p->stream))) return rc;
            if ((rc = upload(bp.tw_full, tf.data(), (size_t)n * 16, p->stream))) return rc;
            if ((rc = upload(bp.twist, tt.data(), (size_t)n / 2 * 16, p->stream))) return rc;
        } else {
            std::vector<float> fh(n), ff(2 * n), ft(n);
            if (p->prec == LC_PREC_FP32) {
                for (int i = 0; i < n; ++i) fh[i] = (float)th[i];
                for (int i = 0; i < 2 * n; ++i) ff[i] = (float)tf[i];
                for (int i = 0; i < n; ++i) ft[i] = (float)tt[i];
            } else {
                twiddles32_plain(n / 2, n / 2, fh.data());
                twiddles32_plain(n, n, ff.data());
                twiddles32_plain(n, n / 2, ft.data());
            }
            if ((rc = upload(bp.tw_half, fh.data(), (size_t)n / 2 * 8, p->stream))) return rc;
            if ((rc = upload(bp.tw_full, ff.data(), (size_t)n * 8, p->stream))) return rc;
            if ((rc = upload(bp.twist, ft.data(), (size_t)n / 2 * 8, p->stream))) return rc;
        }
        // slices never pushed are zero
        HIPCHK(launch_fill_bytes(bp.spec, (int64_t)bp.K * spec_elems(n) * cs, p->stream));
        HIPCHK(launch_fill_f64(bp.dcpart, (int64_t)bp.K * bp.dc_cap(), 0.0, p->stream));
        HIPCHK(launch_fill_f64(bp.ghat0, (int64_t)bp.K * bp.B, 0.0, p->stream));
        HIPCHK(launch_fill_i32(bp.status, 1, 0, p->stream));
        HIPCHK(launch_fill_i32(bp.status + 1, 1, INT32_MAX, p->stream));
        p->boxes.push_back(std::move(bp));
    }
    if (d->autotune && p->prec == LC_PREC_FP32) {
        // boxes of equal N share the shapes measured on the first of them;
        // the slices per forward launch follow each box's own slice count,
        // as the tuner would set them (all slices, up to the table size)
        std::vector<int> done_n;
        std::vector<const BoxPlan *> done_bp;
        for (auto &bp : p->boxes) {
            size_t j = 0;
            while (j < done_n.size() && done_n[j] != bp.n) ++j;
            if (j < done_n.size()) {
                bp.xy_variant = done_bp[j]->xy_variant;
                bp.push_group = std::min(bp.K, SrcTab::kMax);
                bp.fused_variant = done_bp[j]->fused_variant;
                bp.fused_rounds = done_bp[j]->fused_rounds;
                bp.dcw = bp.dc_width();
                continue;
            }
            if ((rc = autotune_box(p.get(), bp))) return rc;
            done_n.push_back(bp.n);
            done_bp.push_back(&bp);
        }
    }
    // up to three side streams for concurrent boxes in lc_step (four lanes)
    const int nside = std::min<int>(3, (int)p->boxes.size() - 1);
    for (int i = 0; i < nside; ++i) {
        hipStream_t t = nullptr;
        hipEvent_t e = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));
        p->side.push_back(t);
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        p->side_done.push_back(e);
    }
    if (nside > 0) HIPCHK(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming));
    HIPCHK(hipStreamSynchronize(p->stream));
    *out = p.release();
    return ok();
}

void lc_destroy(lc_plan_t *p) {
    if (!p) return;
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
}

const char *lc_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

int check_atten(const lc_atten *at, int k) {
    if (at->reserved != 0) return fail(LC_EINVAL, "atten %d: reserved must be 0", k);
    if (at->kind < 0 || at->kind > 2) return fail(LC_EINVAL, "atten %d: unknown kind %d", k, at->kind);
    if (!std::isfinite(at->prefactor)) return fail(LC_EINVAL, "atten %d: prefactor must be finite", k);
    if (at->kind != 0) {
        if (!(at->a > 0) || !(at->s > 0) || !(at->p > 0) || !std::isfinite(at->c) || !std::isfinite(at->a) ||
            !std::isfinite(at->s) || !std::isfinite(at->p))
            return fail(LC_EINVAL, "atten %d needs finite a, s, p > 0 and finite c", k);
        if (at->kind == 2 && !(at->cut >= 0 && std::isfinite(at->cut)))
            return fail(LC_EINVAL, "atten %d: kind 2 needs a finite cut >= 0", k);
    }
    return LC_OK;
}

// Kernels of one (box, band), slice k with radial factor A[k] (algorithm
// steps 2-3). Slices past the last one whose shell meets its factor's
// support are skipped by the slice sum (kcount).
// Shell k's constants for the exact cell average (kernel rule 1).
ExactRule exact_rule(const BoxPlan &bp, const Atten &A, int k) {
    ExactRule e;
    e.l = bp.l;
    e.r_lo = bp.radii[k];
    e.r_sup = std::min(bp.radii[k + 1], support_end(A));
    e.pref = A.pref;
    e.kind = A.kind;
    e.a = A.a; e.s = A.s; e.p = A.p; e.c = A.c;
    std::vector<double> x, w;
    gauss01(16, x, w);
    for (int j = 0; j < 16; ++j) { e.gx[j] = x[j]; e.gw[j] = w[j]; }
    return e;
}

int build_impl(lc_plan_t *p, BoxPlan &bp, int band, const std::vector<Atten> &A) {
    const int n = bp.n, K = bp.K;
    int kc = 0;
    for (int k = 0; k < K; ++k)
        if (bp.radii[k] < support_end(A[k]) && A[k].pref != 0.0) kc = k + 1;
    // the unit source's own cell belongs to slice 0 (r_0 = 0)
    const double self = bp.radii[0] == 0.0 ? self_cell(A[0], bp.l) : 0.0;
    const double l3 = bp.l * bp.l * bp.l;
    const int U = (int)std::ceil(bp.radii[K] / bp.L) + 1;
    const bool oct_f64 = p->t_f64;
    const size_t rs = oct_f64 ? 8 : 4;
    hipStream_t st = p->stream;

    HIPCHK(launch_fill_bytes(bp.maxima + 2 * band, 16, st));
    for (int k = 0; k < K; ++k) {
        char *oct = bp.ghat + ((size_t)k * bp.B + band) * oct_elems(n) * rs;
        double *dc = bp.ghat0 + (size_t)k * bp.B + band;
        if (k >= kc || !(bp.radii[k] < support_end(A[k])) || A[k].pref == 0.0) {
            HIPCHK(launch_fill_bytes(oct, oct_elems(n) * rs, st));
            HIPCHK(launch_fill_f64(dc, 1, 0.0, st));
            continue;
        }
        BuildArgs a;
        a.grid = (double *)p->scratch_real;
        a.n = n; a.m = bp.m; a.l = bp.l; a.h = bp.h;
        a.t_lo = bp.T[k]; a.t_hi = bp.T[k + 1];
        a.r_lo = bp.radii[k]; a.r_hi = bp.radii[k + 1];
        a.images = U;
        a.self_pair = bp.radii[0] == 0.0 ? 1 : 0;
        a.self_val = (k == 0) ? self : 0.0;
        a.kind = A[k].kind; a.a = A[k].a; a.s = A[k].s; a.p = A[k].p; a.c = A[k].c; a.cut = A[k].cut;
        a.pref = A[k].pref;
        a.rule = bp.rule;
        a.ex = exact_rule(bp, A[k], k);
        HIPCHK(launch_greens_build(a, st));
        HIPCHK(launch_x_fwd(n, true, p->scratch_real, true, p->scratch_spec, bp.tw64_half, bp.twist64,
                            nullptr, st));
        HIPCHK(launch_col(n, true, 1, true, p->scratch_spec, bp.tw64_full, st));
        HIPCHK(launch_col(n, true, 2, true, p->scratch_spec, bp.tw64_full, st));
        const double target = bp.conserve ? (Phi(A[k], bp.radii[k + 1]) - Phi(A[k], bp.radii[k])) / l3 : 0.0;
        HIPCHK(launch_greens_fold(n, p->scratch_spec, oct, oct_f64, bp.conserve, target, dc,
                                  bp.maxima + 2 * band, st));
    }
    bp.kcount[band] = kc;
    bp.built[band] = 1;
    bp.att[band] = A;
    // a captured step holds this band's slice count (launch shapes of the
    // slice sum): the next lc_step captures again
    p->gkey.clear();
    return LC_OK;
}

}  // namespace

extern "C" {

int lc_build_greens(lc_plan_t *p, int32_t box, int32_t band, const lc_atten *at) {
    if (!p) return fail(LC_EINVAL, "plan is NULL");
    if (box < 0 || box >= (int)p->boxes.size()) return fail(LC_EINVAL, "box %d out of range", box);
    BoxPlan &bp = p->boxes[box];
    if (band < 0 || band >= bp.B) return fail(LC_EINVAL, "band %d out of range", band);
    if (!at) return fail(LC_EINVAL, "atten is NULL");
    int rc = check_atten(at, 0);
    if (rc) return rc;
    rc = build_impl(p, bp, band, std::vector<Atten>(bp.K, atten_of(at)));
    return rc ? rc : ok();
}

int lc_build_greens_slices(lc_plan_t *p, int32_t box, int32_t band, const lc_atten *per_slice) {
    if (!p) return fail(LC_EINVAL, "plan is NULL");
    if (box < 0 || box >= (int)p->boxes.size()) return fail(LC_EINVAL, "box %d out of range", box);
    BoxPlan &bp = p->boxes[box];
    if (band < 0 || band >= bp.B) return fail(LC_EINVAL, "band %d out of range", band);
    if (!per_slice) return fail(LC_EINVAL, "per_slice is NULL");
    std::vector<Atten> A(bp.K);
    for (int k = 0; k < bp.K; ++k) {
        int rc = check_atten(&per_slice[k], k);
        if (rc) return rc;
        A[k] = atten_of(&per_slice[k]);
    }
    int rc = build_impl(p, bp, band, A);
    return rc ? rc : ok();
}

// Stage lookback slice `slice` of a box (its ring slot) on the plan's stream.
static int push_impl(lc_plan_t *p, int box, int slice, const lc_sources *s) {
    BoxPlan &bp = p->boxes[box];
    const int n = bp.n;
    const int64_t n3 = (int64_t)n * n * n;
    hipStream_t st = p->stream;
    const void *in = nullptr;
    bool in_f64 = s->dtype == LC_F64;
    const int slot = bp.slot(slice);
    bp.last_src[slot] = nullptr;
    if (s->kind == 0) {
        if (s->mem == LC_MEM_DEVICE) {
            in = s->grid;
            bp.last_src[slot] = s->grid;
            bp.last_src_f64[slot] = in_f64 ? 1 : 0;
        } else {
            HIPCHK(hipMemcpyAsync(p->scratch_real, s->grid, (size_t)n3 * (in_f64 ? 8 : 4),
                                  hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
            in = p->scratch_real;
        }
    } else if (s->kind == 2) {
        // positioned sources: nearest-node deposit
        in_f64 = true;
        if (s->mem == LC_MEM_DEVICE) {
            HIPCHK(launch_fill_f64((double *)p->scratch_real, n3, 0.0, st));
            HIPCHK(launch_deposit_pos((double *)p->scratch_real, s->n, (const double *)s->grid, s->lum,
                                      s->dtype == LC_F64, n, bp.l, st));
        } else {
            std::vector<double> g((size_t)n3, 0.0);
            const double *pos = (const double *)s->grid;
            for (int64_t i = 0; i < s->n; ++i) {
                int64_t c[3];
                for (int d = 0; d < 3; ++d) {
                    double v = std::fmod(std::floor(pos[3 * i + d] / bp.l + 0.5), (double)n);
                    if (v < 0.0) v += n;
                    if (v >= n) v -= n;
                    c[d] = (int64_t)v;
                }
                g[(size_t)((c[0] * n + c[1]) * n + c[2])] += s->dtype == LC_F64 ? ((const double *)s->lum)[i]
                                                                               : (double)((const float *)s->lum)[i];
            }
            HIPCHK(hipMemcpyAsync(p->scratch_real, g.data(), (size_t)n3 * 8, hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        in = p->scratch_real;
    } else {
        in_f64 = true;
        if (s->mem == LC_MEM_DEVICE) {
            HIPCHK(launch_fill_f64((double *)p->scratch_real, n3, 0.0, st));
            HIPCHK(launch_deposit((double *)p->scratch_real, s->n, s->cell, s->lum, s->dtype == LC_F64, n3, st));
        } else {
            std::vector<double> g((size_t)n3, 0.0);
            for (int64_t i = 0; i < s->n; ++i)
                g[(size_t)s->cell[i]] += s->dtype == LC_F64 ? ((const double *)s->lum)[i]
                                                            : (double)((const float *)s->lum)[i];
            HIPCHK(hipMemcpyAsync(p->scratch_real, g.data(), (size_t)n3 * 8, hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        in = p->scratch_real;
    }
    const size_t cs = p->t_f64 ? 16 : 8;
    char *spec = bp.spec + (size_t)slot * spec_elems(n) * cs;
    // FP64 input sums (the FP32 form's FP64 mean and its non-finite check)
    double *dcp = p->prec == LC_PREC_FP32 ? bp.dcpart + (size_t)slot * bp.dcw : nullptr;
    // 3D spectra (FP32 form): the x and y passes write the plan's staging
    // spectrum, from which the z pass writes the slot in the slice-sum pass's
    // tile order
    const bool s3 = p->prec == LC_PREC_FP32 && bp.spec3d;
    char *fwd = s3 ? p->scratch_spec : spec;
    if (bp.use_xy) {
        SrcTab tab;
        tab.p[0] = in;
        HIPCHK(launch_xy_fwd_batch(n, tab, 1, in_f64, fwd, 0, bp.tw_half, bp.twist, bp.tw_full, dcp, bp.dcw,
                                   bp.xy_variant, st));
    } else {
        HIPCHK(launch_x_fwd(n, p->t_f64, in, in_f64, fwd, bp.tw_half, bp.twist, dcp, st));
        HIPCHK(launch_col(n, p->t_f64, 1, true, fwd, bp.tw_full, st));
    }
    if (p->prec != LC_PREC_FP32) HIPCHK(launch_col(n, p->t_f64, 2, true, spec, bp.tw_full, st));
    if (s3) HIPCHK(launch_col_z_tiled(n, fwd, spec, bp.tw_full, st));
    bp.pushed[slot] = 1;
    return LC_OK;
}

int lc_push_sources(lc_plan_t *p, int32_t box, int32_t slice, const lc_sources *s) {
    if (!p) return fail(LC_EINVAL, "plan is NULL");
    if (box < 0 || box >= (int)p->boxes.size()) return fail(LC_EINVAL, "box %d out of range", box);
    BoxPlan &bp = p->boxes[box];
    if (slice < 0 || slice >= bp.K) return fail(LC_EINVAL, "slice %d out of range", slice);
    int rc = valid_sources(bp, s);
    if (rc) return rc;
    rc = push_impl(p, box, slice, s);
    return rc ? rc : ok();
}

int lc_advance(lc_plan_t *p, int32_t box, const lc_sources *s) {
    if (!p) return fail(LC_EINVAL, "plan is NULL");
    if (box < 0 || box >= (int)p->boxes.size()) return fail(LC_EINVAL, "box %d out of range", box);
    BoxPlan &bp = p->boxes[box];
    int rc = valid_sources(bp, s);
    if (rc) return rc;
    // the oldest slot becomes lookback slice 0; every other slice moves one
    // lookback slot older
    const int prev = bp.head;
    bp.head = bp.head == 0 ? bp.K - 1 : bp.head - 1;
    rc = push_impl(p, box, 0, s);
    if (rc) {
        bp.head = prev;
        return rc;
    }
    return ok();
}

// Field of one box for bands [b0, b1) into device pointers outp[b - b0].
// frozen >= 0: every lookback slice reads the sources of ring slot `frozen`
// (the instantaneous field of Eq. 18).
static int field_box(lc_plan_t *p, int box, int b0, int b1, void *const *outp, bool out_f64, hipStream_t st,
                     int frozen = -1) {
    BoxPlan &bp = p->boxes[box];
    const int n = bp.n, K = bp.K;
    const size_t cs = p->t_f64 ? 16 : 8;
    const int64_t se = spec_elems(n);
    const double inv_n3 = 1.0 / ((double)n * n * n);
    // per-slice source sums (per ring slot), with the non-finite check: the
    // FP32 form reduces its FP64 input sums, from which the fused z pass
    // forms the FP64 band means; the plain forms read each spectrum's DC bin
    if (p->prec == LC_PREC_FP32)
        HIPCHK(launch_dc_reduce(bp.dcpart, K, bp.dcw, bp.sk, bp.status, bp.head, st));
    else
        HIPCHK(launch_spec_dc(bp.spec, p->t_f64, se, K, bp.sk, bp.status, bp.head, st));
    if (p->prec == LC_PREC_FP32) {
        for (int b = b0; b < b1;) {
            const int nb = std::min(bp.fused_bands, b1 - b);
            int *tab = bp.split_tab + (size_t)(b / bp.fused_bands) * bp.tiles;
            FusedArgs fa;
            fa.spec = bp.spec; fa.spec_stride = se;
            fa.ghat = bp.ghat; fa.oct_stride = oct_elems(n);
            fa.K = K; fa.B = bp.B; fa.band0 = b; fa.nband = nb;
            for (int j = 0; j < 4; ++j) fa.kcount[j] = j < nb ? bp.kcount[b + j] : 0;
            fa.acc = bp.acc + (size_t)b * se * cs; fa.acc_stride = se;
            fa.part = bp.part; fa.part_stride = bp.part_stride; fa.max_parts = bp.max_parts;
            fa.split_tab = tab;
            fa.zero_dc = 1; fa.kahan = nb <= 2; fa.variant = bp.fused_variant; fa.rounds = bp.fused_rounds;
            fa.parity = bp.parity() ? 1 : 0;
            fa.pre = bp.spec3d ? 1 : 0;
            fa.ring = bp.head;
            fa.frozen = frozen;
            fa.sk = bp.sk; fa.g0 = bp.ghat0; fa.inv_n3 = inv_n3; fa.mu = bp.mu;
            HIPCHK(launch_fused_z(n, fa, bp.tw_full, st));
            for (int j = 0; j < nb; ++j) {
                char *acc = bp.acc + (size_t)(b + j) * se * cs;
                char *part = bp.part + (size_t)j * bp.part_stride * 8;
                if (fa.parity) {
                    // parity-layout accumulator: inverse y + x fused per half plane
                    HIPCHK(launch_yx_inv(n, acc, outp[b + j - b0], out_f64, bp.tw_half, bp.twist, bp.tw_full,
                                         inv_n3, bp.mu + b + j, tab, fa.rounds ? nullptr : part, st));
                    continue;
                }
                HIPCHK(inv_y_fused(n, acc, bp.tw_full, tab, part, fa.rounds != 0, st));
                HIPCHK(launch_x_inv(n, false, acc, outp[b + j - b0], out_f64, bp.tw_half, bp.twist, inv_n3,
                                    bp.mu + b + j, st));
            }
            b += nb;
        }
    } else {
        for (int b = b0; b < b1; ++b) {
            char *acc = bp.acc + (size_t)b * se * cs;
            const size_t rs = p->t_f64 ? 8 : 4;
            const int kc = bp.kcount[b];
            if (kc == 0) HIPCHK(launch_fill_bytes(acc, se * cs, st));
            for (int k = 0; k < kc; ++k)
                HIPCHK(launch_mac_plain(n, p->t_f64, acc, bp.spec + (size_t)(frozen >= 0 ? frozen : bp.slot(k)) * se * cs,
                                        bp.ghat + ((size_t)k * bp.B + b) * oct_elems(n) * rs, k == 0, st));
            HIPCHK(launch_col(n, p->t_f64, 2, false, acc, bp.tw_full, st));
            HIPCHK(launch_col(n, p->t_f64, 1, false, acc, bp.tw_full, st));
            HIPCHK(launch_x_inv(n, p->t_f64, acc, outp[b - b0], out_f64, bp.tw_half, bp.twist, inv_n3, nullptr,
                                st));
        }
    }
    return LC_OK;
}

// Read and clear the non-finite source status of boxes [x0, x1) (the stream
// must have reached the reductions): LC_ENONFINITE naming the first box with
// a flagged slice, else LC_OK.
static int take_status(lc_plan_t *p, int x0, int x1, int32_t *first_bad) {
    int code = LC_OK;
    for (int x = x0; x < x1; ++x) {
        BoxPlan &bp = p->boxes[x];
        int32_t st[2];
        HIPCHK(hipMemcpyAsync(st, bp.status, sizeof(st), hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        if (st[0] == 0) continue;
        HIPCHK(launch_fill_i32(bp.status, 1, 0, p->stream));
        HIPCHK(launch_fill_i32(bp.status + 1, 1, INT32_MAX, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        if (code == LC_OK) {
            if (first_bad) *first_bad = st[1];
            code = fail(LC_ENONFINITE, "box %d: %d slice evaluation(s) with non-finite sources, first at lookback slice %d",
                        x, st[0], st[1]);
        }
    }
    return code;
}

static int field_impl(lc_plan_t *p, int32_t box, int32_t band, void *const *out, int32_t dtype, int32_t mem,
                      int frozen_lookback) {
    if (!p) return fail(LC_EINVAL, "plan is NULL");
    if (!out) return fail(LC_EINVAL, "out is NULL");
    if (dtype != LC_F32 && dtype != LC_F64) return fail(LC_EINVAL, "bad output dtype");
    if (mem != LC_MEM_HOST && mem != LC_MEM_DEVICE) return fail(LC_EINVAL, "bad output mem");
    const int nbx = (int)p->boxes.size();
    if (box < -1 || box >= nbx) return fail(LC_EINVAL, "box %d out of range", box);
    const int x0 = box < 0 ? 0 : box, x1 = box < 0 ? nbx : box + 1;
    size_t nout = 0;
    for (int x = x0; x < x1; ++x) {
        const BoxPlan &bp = p->boxes[x];
        if (band < -1 || band >= bp.B) return fail(LC_EINVAL, "band %d out of range for box %d", band, x);
        const int b0 = band < 0 ? 0 : band, b1 = band < 0 ? bp.B : band + 1;
        if (frozen_lookback >= bp.K)
            return fail(LC_EINVAL, "frozen slice %d out of range for box %d (K = %d)", frozen_lookback, x, bp.K);
        for (int b = b0; b < b1; ++b) {
            if (!bp.built[b]) return fail(LC_ESTATE, "kernel of box %d band %d not built", x, b);
            if (!out[nout]) return fail(LC_EINVAL, "output pointer %zu is NULL", nout);
            ++nout;
        }
    }
    const bool f64 = dtype == LC_F64;
    size_t o = 0;
    for (int x = x0; x < x1; ++x) {
        BoxPlan &bp = p->boxes[x];
        const int b0 = band < 0 ? 0 : band, b1 = band < 0 ? bp.B : band + 1;
        const int frozen = frozen_lookback >= 0 ? bp.slot(frozen_lookback) : -1;
        if (mem == LC_MEM_DEVICE) {
            int rc = field_box(p, x, b0, b1, out + o, f64, p->stream, frozen);
            if (rc) return rc;
        } else {
            const size_t bytes = (size_t)bp.n * bp.n * bp.n * (f64 ? 8 : 4);
            for (int b = b0; b < b1; ++b) {
                void *dev = p->scratch_real;
                int rc = field_box(p, x, b, b + 1, &dev, f64, p->stream, frozen);
                if (rc) return rc;
                HIPCHK(hipMemcpyAsync(out[o + (b - b0)], dev, bytes, hipMemcpyDeviceToHost, p->stream));
                HIPCHK(hipStreamSynchronize(p->stream));
            }
        }
        o += (size_t)(b1 - b0);
    }
    if (mem == LC_MEM_HOST) {
        // the stream is synchronised: report non-finite sources now
        int rc = take_status(p, x0, x1, nullptr);
        if (rc) return rc;
    }
    return ok();
}

int lc_field(lc_plan_t *p, int32_t box, int32_t band, void *const *out, int32_t dtype, int32_t mem) {
    return field_impl(p, box, band, out, dtype, mem, -1);
}

int lc_field_frozen(lc_plan_t *p, int32_t box, int32_t band, int32_t slice, void *const *out, int32_t dtype,
                    int32_t mem) {
    if (slice < 0) return fail(LC_EINVAL, "frozen slice %d must be >= 0", slice);
    return field_impl(p, box, band, out, dtype, mem, slice);
}

int lc_fdiff(const void *j, const void *j_inst, void *out, int64_t count, int32_t dtype, void *hip_stream) {
    if (count < 0) return fail(LC_EINVAL, "count must be >= 0");
    if (count > 0 && (!j || !j_inst || !out)) return fail(LC_EINVAL, "NULL field pointer");
    if (dtype != LC_F32 && dtype != LC_F64) return fail(LC_EINVAL, "bad dtype");
    HIPCHK(launch_fdiff(j, j_inst, out, count, dtype == LC_F64, (hipStream_t)hip_stream));
    return ok();
}

int lc_near_field(lc_plan_t *p, int32_t box, int32_t band, const lc_sources *srcs, int32_t near_cells, void *out,
                  int32_t dtype) {
    if (!p) return fail(LC_EINVAL, "plan is NULL");
    if (box < 0 || box >= (int)p->boxes.size()) return fail(LC_EINVAL, "box %d out of range", box);
    BoxPlan &bp = p->boxes[box];
    if (band < 0 || band >= bp.B) return fail(LC_EINVAL, "band %d out of range", band);
    if (!bp.built[band]) return fail(LC_ESTATE, "kernel of box %d band %d not built", box, band);
    if (!srcs || !out) return fail(LC_EINVAL, "srcs/out is NULL");
    if (dtype != LC_F32 && dtype != LC_F64) return fail(LC_EINVAL, "bad output dtype");
    const int R = near_cells;
    if (R < 1 || R > 8) return fail(LC_EINVAL, "near_cells must be in [1, 8]");
    // one periodic image: the farthest corrected node lies below half the box
    if (!((R + 1) * std::sqrt(3.0) * bp.l < 0.5 * bp.L))
        return fail(LC_EUNSUPPORTED, "near_cells = %d reaches beyond half the box (N = %d)", R, bp.n);
    for (int k = 0; k < bp.K; ++k) {
        const lc_sources &s = srcs[k];
        if (s.kind != 2) return fail(LC_EINVAL, "slice %d: near-field sources must be positioned (kind 2)", k);
        int rc = valid_sources(bp, &s);
        if (rc) return rc;
        if (s.mem != LC_MEM_DEVICE) return fail(LC_EINVAL, "slice %d: near-field sources must be in device memory", k);
    }
    const int n = bp.n;
    const int64_t n3 = (int64_t)n * n * n;
    hipStream_t st = p->stream;
    double *corr = (double *)p->scratch_real;
    HIPCHK(launch_fill_f64(corr, n3, 0.0, st));
    NearArgs a;
    a.n = n; a.m = bp.m; a.R = R; a.l = bp.l; a.h = bp.h;
    a.table = (double *)p->scratch_spec;
    a.corr = corr;
    for (int k = 0; k < bp.K; ++k) {
        const lc_sources &s = srcs[k];
        const Atten &A = bp.att[band][k];
        if (s.n == 0 || k >= bp.kcount[band] || A.pref == 0.0) continue;
        a.t_lo = bp.T[k]; a.t_hi = bp.T[k + 1];
        a.r_lo = bp.radii[k]; a.r_hi = bp.radii[k + 1];
        a.kind = A.kind; a.a = A.a; a.s = A.s; a.p = A.p; a.c = A.c; a.cut = A.cut; a.pref = A.pref;
        a.rule = bp.rule;
        a.ex = exact_rule(bp, A, k);
        HIPCHK(launch_near_table(a, st));
        HIPCHK(launch_near_corr(a, s.n, (const double *)s.grid, s.lum, s.dtype == LC_F64, st));
    }
    HIPCHK(launch_add_grid(out, dtype == LC_F64, corr, n3, st));
    return ok();
}

int lc_check_sources(lc_plan_t *p, int32_t box, int32_t *first_bad) {
    if (!p) return fail(LC_EINVAL, "plan is NULL");
    const int nbx = (int)p->boxes.size();
    if (box < -1 || box >= nbx) return fail(LC_EINVAL, "box %d out of range", box);
    if (first_bad) *first_bad = -1;
    HIPCHK(hipStreamSynchronize(p->stream));
    const int rc = take_status(p, box < 0 ? 0 : box, box < 0 ? nbx : box + 1, first_bad);
    return rc ? rc : ok();
}

// One box of lc_step on stream st: its slices' forward passes (groups of up
// to push_group consecutive dense slices of one value type per batched
// launch; point lists one by one, through the plan's staging grid, on the
// plan's stream only) and its field.
static int step_box(lc_plan_t *p, int x, const lc_sources *srcs, void *const *out, int32_t dtype, hipStream_t st) {
    const size_t cs = p->t_f64 ? 16 : 8;
    BoxPlan &bp = p->boxes[x];
    const int n = bp.n;
    const int64_t se = spec_elems(n);
    int k = 0;
    while (k < bp.K) {
        const lc_sources &s0 = srcs[k];
        if (s0.kind != 0 || bp.spec3d) {
            // (3D spectra go through the plan's staging spectrum one slice at a time)
            int rc = push_impl(p, x, k, &s0);
            if (rc) return rc;
            ++k;
            continue;
        }
        // a batch takes consecutive lookback slices in consecutive ring slots
        const int slot0 = bp.slot(k);
        int cnt = 0;
        SrcTab tab;
        while (k + cnt < bp.K && cnt < bp.push_group && srcs[k + cnt].kind == 0 && srcs[k + cnt].dtype == s0.dtype &&
               slot0 + cnt < bp.K) {
            tab.p[cnt] = srcs[k + cnt].grid;
            bp.last_src[slot0 + cnt] = srcs[k + cnt].grid;
            bp.last_src_f64[slot0 + cnt] = s0.dtype == LC_F64 ? 1 : 0;
            ++cnt;
        }
        char *spec = bp.spec + (size_t)slot0 * se * cs;
        double *dcp = p->prec == LC_PREC_FP32 ? bp.dcpart + (size_t)slot0 * bp.dcw : nullptr;
        if (bp.use_xy) {
            HIPCHK(launch_xy_fwd_batch(n, tab, cnt, s0.dtype == LC_F64, spec, se, bp.tw_half, bp.twist, bp.tw_full,
                                       dcp, bp.dcw, bp.xy_variant, st));
        } else {
            HIPCHK(launch_x_fwd_batch(n, p->t_f64, tab, cnt, s0.dtype == LC_F64, spec, se, bp.tw_half, bp.twist,
                                      dcp, st));
            HIPCHK(launch_col_batch(n, p->t_f64, 1, true, spec, se, cnt, bp.tw_full, st));
        }
        if (p->prec != LC_PREC_FP32) HIPCHK(launch_col_batch(n, p->t_f64, 2, true, spec, se, cnt, bp.tw_full, st));
        for (int j = 0; j < cnt; ++j) bp.pushed[slot0 + j] = 1;
        k += cnt;
    }
    return field_box(p, x, 0, bp.B, out, dtype == LC_F64, st);
}

// lc_step's work. With dense sources only and several boxes, the boxes run
// concurrently on up to four lanes (the plan's stream and its side
// streams): each box's work stays on one lane and touches only that box's
// part of the workspace, its sources and its outputs. The boxes go to the
// lanes largest first (N^3 K), each to the least loaded lane.
static int step_impl(lc_plan_t *p, const lc_sources *srcs, void *const *out, int32_t dtype) {
    const int nb = (int)p->boxes.size();
    std::vector<size_t> si(nb), oi(nb);
    bool dense = true;
    {
        size_t a = 0, o = 0;
        for (int x = 0; x < nb; ++x) {
            si[x] = a;
            oi[x] = o;
            for (int k = 0; k < p->boxes[x].K; ++k) dense = dense && srcs[a + k].kind == 0;
            dense = dense && !p->boxes[x].spec3d;   // (the staging spectrum is shared)
            a += p->boxes[x].K;
            o += p->boxes[x].B;
        }
    }
    if (!dense || p->side.empty()) {
        for (int x = 0; x < nb; ++x) {
            int rc = step_box(p, x, srcs + si[x], out + oi[x], dtype, p->stream);
            if (rc) return rc;
        }
        return LC_OK;
    }
    const int nl = (int)p->side.size() + 1;
    std::vector<int> order(nb), lane(nb);
    for (int x = 0; x < nb; ++x) order[x] = x;
    auto work = [&](int x) { return (double)p->boxes[x].n * p->boxes[x].n * p->boxes[x].n * p->boxes[x].K; };
    std::stable_sort(order.begin(), order.end(), [&](int u, int v) { return work(u) > work(v); });
    std::vector<double> load(nl, 0.0);
    for (int x : order) {
        int best = 0;
        for (int l = 1; l < nl; ++l)
            if (load[l] < load[best]) best = l;
        lane[x] = best;
        load[best] += work(x);
    }
    HIPCHK(hipEventRecord(p->fork, p->stream));
    for (hipStream_t t : p->side) HIPCHK(hipStreamWaitEvent(t, p->fork, 0));
    for (int x : order) {
        hipStream_t st = lane[x] == 0 ? p->stream : p->side[lane[x] - 1];
        int rc = step_box(p, x, srcs + si[x], out + oi[x], dtype, st);
        if (rc) return rc;
    }
    for (size_t i = 0; i < p->side.size(); ++i) {
        HIPCHK(hipEventRecord(p->side_done[i], p->side[i]));
        HIPCHK(hipStreamWaitEvent(p->stream, p->side_done[i], 0));
    }
    return LC_OK;
}

int lc_step(lc_plan_t *p, const lc_sources *srcs, void *const *out, int32_t dtype) {
    if (!p) return fail(LC_EINVAL, "plan is NULL");
    if (!srcs || !out) return fail(LC_EINVAL, "srcs/out is NULL");
    if (dtype != LC_F32 && dtype != LC_F64) return fail(LC_EINVAL, "bad output dtype");
    size_t ns = 0, no = 0;
    for (auto &bp : p->boxes) {
        for (int b = 0; b < bp.B; ++b)
            if (!bp.built[b]) return fail(LC_ESTATE, "a kernel is not built");
        for (int k = 0; k < bp.K; ++k) {
            const lc_sources *s = &srcs[ns++];
            int rc = valid_sources(bp, s);
            if (rc) return rc;
            if (s->mem != LC_MEM_DEVICE) return fail(LC_EINVAL, "lc_step takes device sources only");
        }
        for (int b = 0; b < bp.B; ++b)
            if (!out[no++]) return fail(LC_EINVAL, "output pointer is NULL");
    }
    if (!p->use_graph) {
        int rc = step_impl(p, srcs, out, dtype);
        return rc ? rc : ok();
    }
    // graph key: the argument bytes that determine the launch sequence
    std::vector<uint8_t> key(sizeof(int32_t));
    std::memcpy(key.data(), &dtype, sizeof(int32_t));
    key.insert(key.end(), (const uint8_t *)srcs, (const uint8_t *)(srcs + ns));
    key.insert(key.end(), (const uint8_t *)out, (const uint8_t *)(out + no));
    for (auto &bp : p->boxes) key.insert(key.end(), (const uint8_t *)&bp.head, (const uint8_t *)(&bp.head + 1));
    if (!p->gexec || key != p->gkey) {
        if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
        if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
        HIPCHK(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
        int rc = step_impl(p, srcs, out, dtype);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(p->stream, &g);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e != hipSuccess) return fail(LC_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        p->graph = g;
        HIPCHK(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
        p->gkey = key;
    }
    HIPCHK(hipGraphLaunch(p->gexec, p->stream));
    return ok();
}

int lc_greens_imag_ratio(lc_plan_t *p, int32_t box, int32_t band, double *ratio) {
    if (!p || !ratio) return fail(LC_EINVAL, "NULL argument");
    if (box < 0 || box >= (int)p->boxes.size()) return fail(LC_EINVAL, "box out of range");
    BoxPlan &bp = p->boxes[box];
    if (band < 0 || band >= bp.B) return fail(LC_EINVAL, "band out of range");
    if (!bp.built[band]) return fail(LC_ESTATE, "kernel not built");
    unsigned long long m[2];
    HIPCHK(hipMemcpyAsync(m, bp.maxima + 2 * band, 16, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    double mi, mr;
    std::memcpy(&mi, &m[0], 8);
    std::memcpy(&mr, &m[1], 8);
    *ratio = mr > 0 ? mi / mr : 0.0;
    return ok();
}

int lc_greens_dc(lc_plan_t *p, int32_t box, int32_t band, double *dc) {
    if (!p || !dc) return fail(LC_EINVAL, "NULL argument");
    if (box < 0 || box >= (int)p->boxes.size()) return fail(LC_EINVAL, "box out of range");
    BoxPlan &bp = p->boxes[box];
    if (band < 0 || band >= bp.B) return fail(LC_EINVAL, "band out of range");
    if (!bp.built[band]) return fail(LC_ESTATE, "kernel not built");
    std::vector<double> all((size_t)bp.K * bp.B);
    HIPCHK(hipMemcpyAsync(all.data(), bp.ghat0, all.size() * 8, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    for (int k = 0; k < bp.K; ++k) dc[k] = all[(size_t)k * bp.B + band];
    return ok();
}

int lc_time_kernel(lc_plan_t *p, int32_t box, int32_t kernel, int32_t reps, double *avg_ms) {
    if (!p || !avg_ms) return fail(LC_EINVAL, "NULL argument");
    if (box < 0 || box >= (int)p->boxes.size()) return fail(LC_EINVAL, "box out of range");
    if (reps < 1) return fail(LC_EINVAL, "reps must be >= 1");
    BoxPlan &bp = p->boxes[box];
    for (int b = 0; b < bp.B; ++b)
        if (!bp.built[b]) return fail(LC_ESTATE, "kernels not built");
    const bool fused = p->prec == LC_PREC_FP32;
    const bool plain_only = kernel == LC_KERNEL_COL_Z_FWD || kernel == LC_KERNEL_MAC || kernel == LC_KERNEL_COL_Z_INV;
    if (kernel < 0 || kernel > LC_KERNEL_YX_INV) return fail(LC_EINVAL, "unknown kernel id %d", kernel);
    if (kernel == LC_KERNEL_XY_FWD && !bp.use_xy)
        return fail(LC_EINVAL, "this plan does not use the fused xy pass (FP32 form, N in 64..256)");
    if (kernel == LC_KERNEL_YX_INV && !bp.parity())
        return fail(LC_EINVAL, "the fused inverse y + x pass belongs to the parity-layout schedule");
    if ((kernel == LC_KERNEL_COL_Y_INV || kernel == LC_KERNEL_X_INV) && bp.parity())
        return fail(LC_EINVAL, "the parity-layout schedule runs the fused inverse y + x pass instead");
    if (fused && plain_only) return fail(LC_EINVAL, "kernel %d is not part of the fused form", kernel);
    if (!fused && kernel == LC_KERNEL_FUSED_Z) return fail(LC_EINVAL, "the fused z pass belongs to LC_PREC_FP32");
    const int n = bp.n;
    const int64_t n3 = (int64_t)n * n * n, se = spec_elems(n);
    const size_t cs = p->t_f64 ? 16 : 8, rs = p->t_f64 ? 8 : 4;
    hipStream_t st = p->stream;
    if (kernel == LC_KERNEL_X_FWD || kernel == LC_KERNEL_XY_FWD)
        HIPCHK(launch_fill_bytes(p->scratch_real, n3 * (int64_t)rs, st));
    // per-slice kernels cycle over the slices (inputs of the most recent
    // pushes where known) so that their data stream from memory as in a step
    int rep = 0;
    auto one = [&]() -> hipError_t {
        const int k = rep++ % bp.K;
        char *speck = bp.spec + (size_t)k * se * cs, *acc0 = bp.acc;
        switch (kernel) {
            case LC_KERNEL_X_FWD: {
                const void *in = bp.last_src[k] ? bp.last_src[k] : p->scratch_real;
                const bool in_f64 = bp.last_src[k] ? bp.last_src_f64[k] != 0 : p->t_f64;
                return launch_x_fwd(n, p->t_f64, in, in_f64, speck, bp.tw_half, bp.twist,
                                    fused && !bp.use_xy ? bp.dcpart + (size_t)k * bp.dcw : nullptr, st);
            }
            case LC_KERNEL_XY_FWD: {
                // the step's launch configuration: push_group slices per launch
                const int g = std::min(bp.push_group, bp.K);
                const int kg = ((rep - 1) * g) % (bp.K - g + 1);
                SrcTab tab;
                bool in_f64 = false;
                for (int j = 0; j < g; ++j) {
                    tab.p[j] = bp.last_src[kg + j] ? bp.last_src[kg + j] : p->scratch_real;
                    in_f64 = bp.last_src[kg + j] ? bp.last_src_f64[kg + j] != 0 : false;
                }
                return launch_xy_fwd_batch(n, tab, g, in_f64, bp.spec + (size_t)kg * se * cs, se, bp.tw_half,
                                           bp.twist, bp.tw_full, bp.dcpart + (size_t)kg * bp.dcw, bp.dcw,
                                           bp.xy_variant, st);
            }
            case LC_KERNEL_COL_Y_FWD: return launch_col(n, p->t_f64, 1, true, speck, bp.tw_full, st);
            case LC_KERNEL_COL_Z_FWD: return launch_col(n, p->t_f64, 2, true, speck, bp.tw_full, st);
            case LC_KERNEL_FUSED_Z: {
                FusedArgs fa = fused_args(bp);
                fa.ring = bp.head;
                return launch_fused_z(n, fa, bp.tw_full, st);
            }
            case LC_KERNEL_MAC:
                return launch_mac_plain(n, p->t_f64, acc0, speck,
                                        bp.ghat + (size_t)k * bp.B * oct_elems(n) * rs, false, st);
            case LC_KERNEL_COL_Z_INV: return launch_col(n, p->t_f64, 2, false, acc0, bp.tw_full, st);
            case LC_KERNEL_COL_Y_INV:
                return fused ? inv_y_fused(n, acc0, bp.tw_full, bp.split_tab, bp.part, bp.fused_rounds != 0, st)
                             : launch_col(n, p->t_f64, 1, false, acc0, bp.tw_full, st);
            case LC_KERNEL_YX_INV:
                return launch_yx_inv(n, acc0, p->scratch_real, false, bp.tw_half, bp.twist, bp.tw_full,
                                     1.0 / (double)n3, bp.mu, bp.split_tab, bp.fused_rounds ? nullptr : bp.part, st);
            default:
                return launch_x_inv(n, p->t_f64, acc0, p->scratch_real, p->t_f64, bp.tw_half, bp.twist,
                                    1.0 / (double)n3, fused ? bp.mu : nullptr, st);
        }
    };
    HIPCHK(one());   // warm-up
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) HIPCHK(one());
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = (double)ms / reps;
    return ok();
}

int lc_get_schedule(lc_plan_t *p, int32_t box, lc_schedule *out) {
    if (!p || !out) return fail(LC_EINVAL, "NULL argument");
    if (box < 0 || box >= (int)p->boxes.size()) return fail(LC_EINVAL, "box out of range");
    const BoxPlan &bp = p->boxes[box];
    const bool fused = p->prec == LC_PREC_FP32;
    out->n_xy = fused ? xy_variants(bp.n) : 0;
    out->n_fused = fused ? fused_variants(bp.n) : 0;
    out->xy_variant = bp.use_xy ? bp.xy_variant : -1;
    out->fused_variant = fused ? bp.fused_variant : -1;
    out->fused_rounds = bp.fused_rounds;
    out->push_group = bp.push_group;
    out->fused_bands = fused ? bp.fused_bands : -1;
    out->n_fused_bands = fused ? std::min(bp.B, fused_max_bands(bp.n)) : 0;
    out->spectra_3d = fused ? (bp.spec3d ? 1 : 0) : -1;
    return ok();
}

int lc_set_schedule(lc_plan_t *p, int32_t box, const lc_schedule *s) {
    if (!p || !s) return fail(LC_EINVAL, "NULL argument");
    if (box < 0 || box >= (int)p->boxes.size()) return fail(LC_EINVAL, "box out of range");
    BoxPlan &bp = p->boxes[box];
    const bool fused = p->prec == LC_PREC_FP32;
    const int n_xy = fused ? xy_variants(bp.n) : 0, n_fused = fused ? fused_variants(bp.n) : 0;
    if (s->xy_variant < -1 || s->xy_variant >= n_xy)
        return fail(LC_EINVAL, "xy_variant %d outside [-1, %d)", s->xy_variant, n_xy);
    if (fused ? (s->fused_variant < 0 || s->fused_variant >= n_fused) : s->fused_variant != -1)
        return fail(LC_EINVAL, "fused_variant %d not available", s->fused_variant);
    if (s->fused_rounds != 0 && s->fused_rounds != 1) return fail(LC_EINVAL, "fused_rounds must be 0 or 1");
    if (s->push_group < 1 || s->push_group > SrcTab::kMax)
        return fail(LC_EINVAL, "push_group must be in [1, %d]", SrcTab::kMax);
    const int max_bands = fused ? std::min(bp.B, fused_max_bands(bp.n)) : 0;
    if (fused ? (s->fused_bands < 1 || s->fused_bands > max_bands) : s->fused_bands != -1)
        return fail(LC_EINVAL, "fused_bands %d not available (1..%d)", s->fused_bands, max_bands);
    if (fused ? (s->spectra_3d != 0 && s->spectra_3d != 1) : s->spectra_3d != -1)
        return fail(LC_EINVAL, "spectra_3d must be 0 or 1 (FP32 form), -1 otherwise");
    if (s->spectra_3d == 1 && s->xy_variant >= 0 && xy_parity(bp.n, s->xy_variant))
        return fail(LC_EINVAL, "spectra_3d needs a whole-plane xy shape (xy_variant %d is a parity-layout shape)",
                    s->xy_variant);
    const bool use_xy = s->xy_variant >= 0;
    const bool par = use_xy && xy_parity(bp.n, s->xy_variant);
    const bool s3 = fused && s->spectra_3d == 1;
    if (use_xy != bp.use_xy || par != bp.parity() || s3 != bp.spec3d) {
        // the spectrum and DC partial layouts change with the forward pass:
        // pushed slices are dropped
        const size_t cs = p->t_f64 ? 16 : 8;
        HIPCHK(launch_fill_bytes(bp.spec, (int64_t)bp.K * spec_elems(bp.n) * cs, p->stream));
        HIPCHK(launch_fill_f64(bp.dcpart, (int64_t)bp.K * bp.dc_cap(), 0.0, p->stream));
        std::fill(bp.pushed.begin(), bp.pushed.end(), 0);
        std::fill(bp.last_src.begin(), bp.last_src.end(), nullptr);
    }
    bp.use_xy = use_xy;
    if (use_xy) bp.xy_variant = s->xy_variant;
    bp.dcw = bp.dc_width();
    if (fused) {
        bp.fused_variant = s->fused_variant;
        bp.fused_bands = s->fused_bands;
        bp.spec3d = s3;
    }
    bp.fused_rounds = s->fused_rounds;
    bp.push_group = s->push_group;
    p->gkey.clear();   // the next lc_step captures the new launch sequence
    return ok();
}


// ---- cosmological slicing and Lyman-Werner radial factors ---------------------
//
// Flat universe of matter and a cosmological constant (Omega_L = 1 - Omega_m):
//  * cosmic time, closed form: t(z) = 2 / (3 H0 sqrt(OL)) asinh(sqrt(OL/Om) (1+z)^-1.5)
//    (the matter-only limit 2 / (3 H0 sqrt(Om)) (1+z)^-1.5 when OL = 0);
//  * conformal distance (Eq. 5 times c): chi(z1, z2) = (c/H0) int dz / E(z),
//    E = sqrt(Om (1+z)^3 + OL); with u = (1+z)^-1/2 the integrand becomes
//    2 / sqrt(Om + OL u^6), smooth on [u2, u1], integrated by Gauss-Legendre.
// Units: Myr (Julian year), comoving Mpc, c = 299792.458 km/s.

}  // extern "C"

namespace {

constexpr double kC_kms = 299792.458;
constexpr double kMpc_km = 3.0856775814913673e19;
constexpr double kMyr_s = 3.15576e13;

struct Bg {
    double om, ol, H0_myr, dh_mpc;
};

int bg_of(const lc_cosmo *c, Bg *b) {
    if (!c) return fail(LC_EINVAL, "cosmology is NULL");
    if (!(c->h > 0) || !std::isfinite(c->h)) return fail(LC_EINVAL, "h must be > 0");
    if (!(c->omega_m > 0 && c->omega_m <= 1)) return fail(LC_EINVAL, "omega_m must be in (0, 1]");
    b->om = c->omega_m;
    b->ol = 1.0 - c->omega_m;
    b->H0_myr = 100.0 * c->h / kMpc_km * kMyr_s;
    b->dh_mpc = kC_kms / (100.0 * c->h);
    return LC_OK;
}

double t_of_z(const Bg &b, double z) {
    const double x = std::pow(1.0 + z, -1.5);
    if (b.ol <= 0.0) return 2.0 / (3.0 * b.H0_myr * std::sqrt(b.om)) * x;
    return 2.0 / (3.0 * b.H0_myr * std::sqrt(b.ol)) * std::asinh(std::sqrt(b.ol / b.om) * x);
}

double z_of_t(const Bg &b, double t) {
    double x;
    if (b.ol <= 0.0) x = 1.5 * b.H0_myr * std::sqrt(b.om) * t;
    else x = std::sqrt(b.om / b.ol) * std::sinh(1.5 * b.H0_myr * std::sqrt(b.ol) * t);
    return std::pow(x, -2.0 / 3.0) - 1.0;
}

struct Rule32 {
    std::vector<double> x, w;
    Rule32() { gauss01(32, x, w); }
};

double chi(const Bg &b, double z1, double z2) {
    static const Rule32 rule;    // built once (thread-safe static initialisation)
    const std::vector<double> &gx = rule.x, &gw = rule.w;
    const double u1 = 1.0 / std::sqrt(1.0 + z1), u2 = 1.0 / std::sqrt(1.0 + z2);
    // four panels over [u2, u1]
    double acc = 0.0;
    for (int pnl = 0; pnl < 4; ++pnl) {
        const double a = u2 + (u1 - u2) * pnl / 4.0, w = (u1 - u2) / 4.0;
        for (size_t i = 0; i < gx.size(); ++i) {
            const double u = a + w * gx[i];
            const double u3 = u * u * u;
            acc += gw[i] * w * 2.0 / std::sqrt(b.om + b.ol * u3 * u3);
        }
    }
    return b.dh_mpc * acc;
}

}  // namespace

extern "C" {

int lc_cosmo_slices(const lc_cosmo *c, double z_obs, double dt_myr, int32_t K, double *radii, double *z_edge,
                    double *z_src) {
    Bg b;
    int rc = bg_of(c, &b);
    if (rc) return rc;
    if (!(z_obs >= 0) || !std::isfinite(z_obs)) return fail(LC_EINVAL, "z_obs must be finite and >= 0");
    if (!(dt_myr > 0) || !std::isfinite(dt_myr)) return fail(LC_EINVAL, "dt_myr must be > 0");
    if (K < 1 || K > 1024) return fail(LC_EINVAL, "K must be in [1, 1024]");
    if (!radii) return fail(LC_EINVAL, "radii is NULL");
    const double t0 = t_of_z(b, z_obs);
    if (!(t0 - K * dt_myr > 0.0))
        return fail(LC_EINVAL, "K = %d slices of %g Myr reach beyond t = 0 (t_obs = %g Myr)", K, dt_myr, t0);
    for (int k = 0; k <= K; ++k) {
        const double zk = k == 0 ? z_obs : z_of_t(b, t0 - k * dt_myr);
        radii[k] = k == 0 ? 0.0 : chi(b, z_obs, zk);
        if (z_edge) z_edge[k] = zk;
        if (z_src && k < K) z_src[k] = z_of_t(b, t0 - (k + 0.5) * dt_myr);
    }
    return ok();
}

int lc_lw_factors(const lc_cosmo *c, double z_obs, int32_t K, const double *z_src, int32_t kind, lc_atten *out) {
    Bg b;
    int rc = bg_of(c, &b);
    if (rc) return rc;
    if (K < 1 || !z_src || !out) return fail(LC_EINVAL, "K >= 1 and non-NULL z_src, out required");
    if (kind != 1 && kind != 2) return fail(LC_EINVAL, "kind must be 1 (continuous) or 2 (Eq. 15 as printed)");
    const double pi = 3.141592653589793238462643383279502884;
    for (int k = 0; k < K; ++k) {
        if (!(z_src[k] >= z_obs) || !std::isfinite(z_src[k]))
            return fail(LC_EINVAL, "z_src[%d] = %g must be finite and >= z_obs", k, z_src[k]);
        // Eq. 16
        const double alpha = std::pow(c->h / 0.7, -1.0) * std::pow(c->omega_m / 0.27, -0.5) *
                             std::pow((1.0 + z_src[k]) / 21.0, -0.5);
        lc_atten &a = out[k];
        a.kind = kind;
        a.reserved = 0;
        a.a = 1.7;               // Eq. 15
        a.s = 116.29 * alpha;
        a.p = 0.68;
        a.c = 0.7;
        a.cut = 97.39 * alpha;
        // Eq. 14: (1/(4 pi)^2) (1+z)^3 / (1+z_s); the kernel carries 1/(4 pi r^2)
        a.prefactor = std::pow(1.0 + z_obs, 3) / (1.0 + z_src[k]) / (4.0 * pi);
    }
    return ok();
}

// ---- allocation-free whole step (static device scratch) ----------------------

}  // extern "C"

// Device scratch of lc_step_static: one copy per GPU, held until the
// process ends. Host code never uses this name as an address (on the host it
// is only a stand-in for the symbol); the device address of each GPU's copy
// comes from hipGetSymbolAddress with that GPU current.
static __device__ __align__(256) char scratch[LC_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch, looked up on the first call
// on that GPU.
int scratch_ptr(void **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LC_EDEVICE, "device %d beyond the %d supported", dev, kMaxDevices);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(LC_EDEVICE, "no device address for the static scratch");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LC_OK;
}

}  // namespace

extern "C" {

int lc_step_static(const lc_plan_desc *desc, const lc_atten *atten, const lc_sources *srcs, void *const *out,
                   int32_t dtype) {
    if (!desc || !atten || !srcs || !out) return fail(LC_EINVAL, "NULL argument");
    int rc = validate(desc);
    if (rc) return rc;
    if (desc->n_boxes != 1) return fail(LC_EINVAL, "lc_step_static takes one box (n_boxes = %d)", desc->n_boxes);
    if (desc->workspace || desc->workspace_bytes)
        return fail(LC_EINVAL, "lc_step_static uses its static scratch: workspace must be NULL and 0 bytes");
    if (desc->use_graph || desc->autotune)
        return fail(LC_EINVAL, "lc_step_static runs eagerly with the built-in launch shapes (use_graph = autotune = 0)");
    const size_t need = layout_of(desc).total;
    if (need > (size_t)LC_STATIC_SCRATCH_BYTES)
        return fail(LC_ENOMEM, "this box needs %zu bytes of scratch, above the static maximum of %zu bytes "
                               "(use lc_plan with a caller workspace)", need, (size_t)LC_STATIC_SCRATCH_BYTES);
    if ((rc = check_device())) return rc;
    void *ws = nullptr;
    if ((rc = scratch_ptr(&ws))) return rc;
    lc_plan_desc d = *desc;
    d.workspace = ws;
    d.workspace_bytes = LC_STATIC_SCRATCH_BYTES;
    lc_plan_t *p = nullptr;
    if ((rc = lc_plan(&d, &p))) return rc;
    const int B = desc->boxes[0].n_bands;
    for (int b = 0; b < B && !rc; ++b) rc = lc_build_greens(p, 0, b, &atten[b]);
    if (!rc) rc = lc_step(p, srcs, out, dtype);
    if (!rc) {
        // the next call on this GPU reuses the scratch: this one's work
        // must be done with it first
        hipError_t e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) rc = fail(LC_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
    }
    const std::string msg = g_err;
    lc_destroy(p);
    if (rc) {
        g_err = msg;
        return rc;
    }
    return ok();
}

}  // extern "C"
