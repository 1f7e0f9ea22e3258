// Forward/inverse x passes (real <-> half spectrum) and strided column
// passes (y, z) of the 3D transform of Eq. 12, for gfx950.
//
// x pass, forward: a real row of N values is read as N/2 complex values
// z[n] = x[2n] + i x[2n+1]; after a length-N/2 FFT, the spectrum of the row
// is recovered for p in [0, N/2] from Z[p] and Z[N/2-p]:
//   E = (Z[p] + conj Z[N/2-p]) / 2,  O = (Z[p] - conj Z[N/2-p]) / (2i),
//   X[p] = E + W^p O,  X[N/2-p] = conj(E - W^p O),   W = exp(-2 pi i / N).
// x pass, inverse: the same relation run backwards (unnormalised), giving
// N x[2n] + i N x[2n+1] after a length-N/2 inverse FFT.
#include "lc_fft_device.h"
#include "lc_internal.h"

namespace lc {

// ---------------------------------------------------------------------------
// forward x pass
// ---------------------------------------------------------------------------
template <typename T, typename TIN, int N, bool DC>
__global__ __launch_bounds__((RowShape<T, N / 2>::NT)) void x_fwd_kernel(
    SrcTab srcs, cx<T> *__restrict__ spec0, int64_t spec_stride, int64_t n_rows, int wgs,
    const cx<T> *__restrict__ tw_g, const cx<T> *__restrict__ twist_g, double *__restrict__ dcpart0) {
    // workgroup blockIdx.x handles row block (blockIdx.x % wgs) of slice (blockIdx.x / wgs)
    const int slice = blockIdx.x / wgs, blk = blockIdx.x % wgs;
    const TIN *__restrict__ in = (const TIN *)srcs.p[slice];
    cx<T> *__restrict__ mainp = spec0 + slice * spec_stride;
    cx<T> *__restrict__ nyq = mainp + spec_main(N);
    double *__restrict__ dcpart = dcpart0 ? dcpart0 + (int64_t)slice * wgs : nullptr;
    constexpr int L = N / 2;
    using SH = RowShape<T, L>;
    constexpr int SK = SH::SK;
    using EN = Engine<T, L, true, Sched<L>, SK>;
    constexpr int TPL = SH::TPL, NT = SH::NT, RPW = SH::RPW, LS = SH::LS, E = EN::E;
    __shared__ cx<T> lds[RPW * LS];
    __shared__ cx<T> tws[L];
    __shared__ cx<T> twst[L];
    __shared__ double red[NT / 64];
    for (int i = threadIdx.x; i < L; i += NT) {
        tws[i] = tw_g[i];
        twst[i] = twist_g[i];
    }
    const int64_t row0 = (int64_t)blk * RPW;
    const int line = threadIdx.x / TPL, t = threadIdx.x % TPL;
    const int64_t row = row0 + line;
    const bool active = row < n_rows;
    double dsum = 0.0;
    cx<T> x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = EN::in_pos(t, e);
        if (active) {
            // one 2-element vector load (rows start 2-element aligned)
            const cx<TIN> ab = *(const cx<TIN> *)(in + row * N + 2 * p);
            x[e] = mk((T)ab.x, (T)ab.y);
            if (DC) dsum += (double)ab.x + (double)ab.y;
        } else {
            x[e] = mk((T)0, (T)0);
        }
    }
    EN::run(x, lds, line * LS, 1, t, tws);
    lds_barrier();
    cx<T> *z = lds + line * LS;
#pragma unroll
    for (int e = 0; e < E; ++e) z[lpos<SK>(EN::out_pos(t, e))] = x[e];
    lds_barrier();
    if (active) {
        for (int p = t; p <= L / 2; p += TPL) {
            const cx<T> A = z[lpos<SK>(p)], B = z[lpos<SK>((L - p) % L)];
            const cx<T> Ev = mk((A.x + B.x) * (T)0.5, (A.y - B.y) * (T)0.5);
            // O = (A - conj B) / (2i)
            const cx<T> O = mk((A.y + B.y) * (T)0.5, (B.x - A.x) * (T)0.5);
            const cx<T> WO = cmul(twst[p], O);
            mainp[row * L + p] = Ev + WO;
            const cx<T> Xm = conj(Ev - WO);
            if (p == 0) nyq[row] = Xm;
            else if (p != L - p) mainp[row * L + (L - p)] = Xm;
        }
    }
    if (DC) {
        // workgroup sum of the FP64 partials (fixed order: deterministic)
        for (int o = 32; o > 0; o >>= 1) dsum += __shfl_down(dsum, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dsum;
        lds_barrier();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += red[w];
            dcpart[blk] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// inverse x pass + epilogue
// ---------------------------------------------------------------------------
template <typename T, typename TOUT, int N>
__global__ __launch_bounds__((RowShape<T, N / 2>::NT)) void x_inv_kernel(
    const cx<T> *__restrict__ mainp, const cx<T> *__restrict__ nyq, TOUT *__restrict__ out,
    int64_t n_rows, const cx<T> *__restrict__ tw_g, const cx<T> *__restrict__ twist_g, double scale,
    const double *__restrict__ mu) {
    constexpr int L = N / 2;
    using SH = RowShape<T, L>;
    using EN = Engine<T, L, false, Sched<L>, SH::SK>;
    constexpr int TPL = SH::TPL, NT = SH::NT, RPW = SH::RPW, LS = SH::LS, E = EN::E;
    __shared__ cx<T> lds[RPW * LS];
    __shared__ cx<T> tws[L];
    __shared__ cx<T> twst[L];
    for (int i = threadIdx.x; i < L; i += NT) {
        tws[i] = tw_g[i];
        twst[i] = twist_g[i];
    }
    lds_barrier();
    const int64_t row0 = (int64_t)blockIdx.x * RPW;
    const int line = threadIdx.x / TPL, t = threadIdx.x % TPL;
    const int64_t row = row0 + line;
    const bool active = row < n_rows;
    cx<T> x[E];
    // Z[p] = E'_p + i O'_p with E'_p = X[p] + conj X[L-p],
    // O'_p = (X[p] - conj X[L-p]) conj(W^p); at p = 0 the real parts of X[0], X[L]
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = EN::in_pos(t, e);
        if (!active) {
            x[e] = mk((T)0, (T)0);
        } else if (p == 0) {
            const T x0 = mainp[row * L].x, xl = nyq[row].x;
            x[e] = mk(x0 + xl, x0 - xl);
        } else {
            const cx<T> Xp = mainp[row * L + p], Xm = mainp[row * L + (L - p)];
            const cx<T> Ep = Xp + conj(Xm);
            const cx<T> Op = cmul(Xp - conj(Xm), conj(twst[p]));
            x[e] = mk(Ep.x - Op.y, Ep.y + Op.x);
        }
    }
    EN::run(x, lds, line * LS, 1, t, tws);
    if (active) {
        const double m = mu ? *mu : 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            cx<TOUT> o;
            o.x = (TOUT)((double)x[e].x * scale + m);
            o.y = (TOUT)((double)x[e].y * scale + m);
            *(cx<TOUT> *)(out + row * N + 2 * EN::out_pos(t, e)) = o;
        }
    }
}

// ---------------------------------------------------------------------------
// column passes (y or z), in place; grid = main WGs then nyq WGs.
// Lanes walk the columns (col_stride 1) or, for row-contiguous sets, the
// rows of a column, so that global accesses stay coalesced either way.
// With COMBINE (inverse y pass of a fused FP32 accumulator) the second part
// of a tile that the persistent fused pass split between two workgroups is
// added while loading: element (z, y=q, p) belongs to fused tile
// (q*H + p) / cpw_z (main) or tiles_main + q / cpw_z (nyq), at row z.
// ---------------------------------------------------------------------------
template <int CPW, int TPL>
__device__ __forceinline__ void col_lane(bool rowfast, int &c, int &t) {
    if (rowfast) { c = threadIdx.x / TPL; t = threadIdx.x % TPL; }
    else { c = threadIdx.x % CPW; t = threadIdx.x / CPW; }
}

// TILED (z forward into the slice-sum pass's tile order): the transformed
// columns go to `out`, each set (main, nyq) as consecutive tiles of tcpw
// columns (the last one narrower), a tile's rows contiguous:
//   element (row r, column col) at set_off + c0 L + r w + (col - c0),
//   c0 = col - col mod tcpw, w = min(tcpw, n_cols - c0).
template <typename T, int L, bool FWD, bool COMBINE, bool TILED = false>
__global__ __launch_bounds__((ColShape<T, L>::NT)) void col_kernel(
    cx<T> *data0, int64_t data_stride, ColSet s0, ColSet s1, const cx<T> *__restrict__ tw_g,
    const int *__restrict__ tab, const cx<T> *__restrict__ part, int64_t tiles_main, int cpw_z,
    cx<T> *__restrict__ out = nullptr, int tcpw = 1) {
    // workgroup blockIdx.x handles tile (blockIdx.x % per) of spectrum (blockIdx.x / per)
    const int per = s0.n_wgs + s1.n_wgs;
    const int bid = blockIdx.x % per;
    cx<T> *data = data0 + (int64_t)(blockIdx.x / per) * data_stride;
    using SH = ColShape<T, L>;
    using EN = Engine<T, L, FWD>;
    constexpr int CPW = SH::CPW, NT = SH::NT, ES = CPW + SH::PAD, E = EN::E, TPL = SH::TPL;
    __shared__ cx<T> lds[L * ES];
    __shared__ cx<T> tws[L];
    for (int i = threadIdx.x; i < L; i += NT) tws[i] = tw_g[i];
    const bool first = bid < s0.n_wgs;
    const ColSet &s = first ? s0 : s1;
    const int64_t col0 = (int64_t)(first ? bid : bid - s0.n_wgs) * CPW;
    int c, t;
    col_lane<CPW, TPL>(s.rowfast, c, t);
    const int64_t col = col0 + c;
    const bool ok = col < s.n_cols;
    const int64_t base = ok ? col_base(s, col) : 0;
    cx<T> x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = EN::in_pos(t, e);
        x[e] = ok ? data[base + j * s.row_stride] : mk((T)0, (T)0);
        if constexpr (COMBINE) {
            if (ok) {
                int zt, zc, z;
                if (first) {
                    const int H = L / 2;
                    z = (int)(col / H);
                    const int q = j * H + (int)(col % H);
                    zt = q / cpw_z; zc = q % cpw_z;
                } else {
                    z = (int)col;
                    zt = (int)(tiles_main + j / cpw_z); zc = j % cpw_z;
                }
                const int w = tab[zt];
                if (w >= 0) x[e] = x[e] + part[((int64_t)w * L + z) * cpw_z + zc];
            }
        }
    }
    EN::run(x, lds, c, ES, t, tws);
    if constexpr (TILED) {
        if (ok) {
            const int64_t c0 = col - col % tcpw;
            const int64_t w = s.n_cols - c0 < tcpw ? s.n_cols - c0 : tcpw;
            cx<T> *o = out + (first ? 0 : spec_main(L)) + c0 * L + (col - c0);
#pragma unroll
            for (int e = 0; e < E; ++e) o[EN::out_pos(t, e) * w] = x[e];
        }
    } else if (ok) {
#pragma unroll
        for (int e = 0; e < E; ++e) data[base + EN::out_pos(t, e) * s.row_stride] = x[e];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
bool supported_n(int n) {
    switch (n) {
        case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96:
        case 128: case 192: case 256: case 384: case 512: return true;
        default: return false;
    }
}

#define LC_DISPATCH_N(n, MACRO)                                                  \
    switch (n) {                                                                 \
        case 8: MACRO(8); break;     case 12: MACRO(12); break;                  \
        case 16: MACRO(16); break;   case 24: MACRO(24); break;                  \
        case 32: MACRO(32); break;   case 48: MACRO(48); break;                  \
        case 64: MACRO(64); break;   case 96: MACRO(96); break;                  \
        case 128: MACRO(128); break; case 192: MACRO(192); break;                \
        case 256: MACRO(256); break; case 384: MACRO(384); break;                \
        case 512: MACRO(512); break;                                             \
        default: return hipErrorInvalidValue;                                    \
    }

template <int N> static int x_wgs_t() {
    using SH = RowShape<float, N / 2>;
    return (int)(((int64_t)N * N + SH::RPW - 1) / SH::RPW);
}

int x_pass_wgs(int n) {
    if (x_rows_supported(n)) return x_rows_wgs(n);   // the FP32 x pass there
    switch (n) {
#define W_(N) case N: return x_wgs_t<N>();
        W_(8) W_(12) W_(16) W_(24) W_(32) W_(48) W_(64) W_(96) W_(128) W_(192) W_(256) W_(384) W_(512)
#undef W_
        default: return 0;
    }
}

template <typename T, typename TIN, int N>
static hipError_t x_fwd_t(const SrcTab &in, int count, void *spec, int64_t spec_stride, const void *tw,
                          const void *twist, double *dcpart, hipStream_t st) {
    using SH = RowShape<T, N / 2>;
    static_assert(SH::RPW == RowShape<float, N / 2>::RPW, "rows per WG must not depend on T");
    const int64_t rows = (int64_t)N * N;
    const int wgs = (int)((rows + SH::RPW - 1) / SH::RPW);
    const dim3 grid((unsigned)(wgs * count));
    if (dcpart)
        hipLaunchKernelGGL((x_fwd_kernel<T, TIN, N, true>), grid, dim3(SH::NT), 0, st, in, (cx<T> *)spec,
                           spec_stride, rows, wgs, (const cx<T> *)tw, (const cx<T> *)twist, dcpart);
    else
        hipLaunchKernelGGL((x_fwd_kernel<T, TIN, N, false>), grid, dim3(SH::NT), 0, st, in, (cx<T> *)spec,
                           spec_stride, rows, wgs, (const cx<T> *)tw, (const cx<T> *)twist, dcpart);
    return hipGetLastError();
}

hipError_t launch_x_fwd_batch(int n, bool t_f64, const SrcTab &in, int count, bool in_f64, void *spec,
                              int64_t spec_stride, const void *tw_half, const void *twist, double *dcpart,
                              hipStream_t st) {
    if (count < 1 || count > SrcTab::kMax) return hipErrorInvalidValue;
    if (!t_f64 && x_rows_supported(n))
        return launch_x_rows_batch(n, in, count, in_f64, spec, spec_stride, tw_half, twist, dcpart, st);
#define X_(N)                                                                                          \
    if (t_f64) return in_f64 ? x_fwd_t<double, double, N>(in, count, spec, spec_stride, tw_half, twist, dcpart, st) \
                             : x_fwd_t<double, float, N>(in, count, spec, spec_stride, tw_half, twist, dcpart, st); \
    else return in_f64 ? x_fwd_t<float, double, N>(in, count, spec, spec_stride, tw_half, twist, dcpart, st)       \
                       : x_fwd_t<float, float, N>(in, count, spec, spec_stride, tw_half, twist, dcpart, st);
    LC_DISPATCH_N(n, X_)
#undef X_
    return hipErrorInvalidValue;
}

hipError_t launch_x_fwd(int n, bool t_f64, const void *in, bool in_f64, void *spec,
                        const void *tw_half, const void *twist, double *dcpart, hipStream_t st) {
    SrcTab tab;
    tab.p[0] = in;
    return launch_x_fwd_batch(n, t_f64, tab, 1, in_f64, spec, 0, tw_half, twist, dcpart, st);
}

template <typename T, typename TOUT, int N>
static hipError_t x_inv_t(const void *spec, void *out, const void *tw, const void *twist,
                          double scale, const double *mu, hipStream_t st) {
    using SH = RowShape<T, N / 2>;
    const int64_t rows = (int64_t)N * N;
    const int wgs = (int)((rows + SH::RPW - 1) / SH::RPW);
    const cx<T> *sp = (const cx<T> *)spec;
    hipLaunchKernelGGL((x_inv_kernel<T, TOUT, N>), dim3(wgs), dim3(SH::NT), 0, st, sp,
                       sp + spec_main(N), (TOUT *)out, rows, (const cx<T> *)tw,
                       (const cx<T> *)twist, scale, mu);
    return hipGetLastError();
}

hipError_t launch_x_inv(int n, bool t_f64, const void *spec, void *out, bool out_f64,
                        const void *tw_half, const void *twist, double scale, const double *mu,
                        hipStream_t st) {
#define X_(N)                                                                                     \
    if (t_f64) return out_f64 ? x_inv_t<double, double, N>(spec, out, tw_half, twist, scale, mu, st) \
                              : x_inv_t<double, float, N>(spec, out, tw_half, twist, scale, mu, st); \
    else return out_f64 ? x_inv_t<float, double, N>(spec, out, tw_half, twist, scale, mu, st)       \
                        : x_inv_t<float, float, N>(spec, out, tw_half, twist, scale, mu, st);
    LC_DISPATCH_N(n, X_)
#undef X_
    return hipErrorInvalidValue;
}

// Column sets of the spectrum for a pass along axis 1 (y) or 2 (z).
template <typename T, int N>
static void col_sets(int axis, ColSet &s0, ColSet &s1) {
    using SH = ColShape<T, N>;
    const int64_t H = N / 2;
    const int64_t main_n = spec_main(N);
    if (axis == 1) {
        // main: columns (z, p); element (row y) at z*N*H + y*H + p
        s0.n_cols = (int64_t)N * H; s0.W = H; s0.plane_stride = (int64_t)N * H; s0.col_stride = 1;
        s0.row_stride = H; s0.off = 0; s0.rowfast = 0;
        // nyq: columns z; element (row y) at main_n + z*N + y
        s1.n_cols = N; s1.W = N; s1.plane_stride = 0; s1.col_stride = N; s1.row_stride = 1;
        s1.off = main_n; s1.rowfast = 1;
    } else {
        // main: columns (y, p) = flat y*H + p; element (row z) at z*N*H + col
        s0.n_cols = (int64_t)N * H; s0.W = (int64_t)N * H; s0.plane_stride = 0; s0.col_stride = 1;
        s0.row_stride = (int64_t)N * H; s0.off = 0; s0.rowfast = 0;
        // nyq: columns y; element (row z) at main_n + z*N + y
        s1.n_cols = N; s1.W = N; s1.plane_stride = 0; s1.col_stride = 1; s1.row_stride = N;
        s1.off = main_n; s1.rowfast = 0;
    }
    s0.n_wgs = (int32_t)((s0.n_cols + SH::CPW - 1) / SH::CPW);
    s1.n_wgs = (int32_t)((s1.n_cols + SH::CPW - 1) / SH::CPW);
}

template <typename T, int N>
static hipError_t col_t(int axis, bool fwd, void *spec, int64_t stride, int count, const void *tw,
                        hipStream_t st) {
    using SH = ColShape<T, N>;
    ColSet s0, s1;
    col_sets<T, N>(axis, s0, s1);
    const dim3 grid((unsigned)((s0.n_wgs + s1.n_wgs) * count));
    if (fwd)
        hipLaunchKernelGGL((col_kernel<T, N, true, false>), grid, dim3(SH::NT), 0, st, (cx<T> *)spec, stride,
                           s0, s1, (const cx<T> *)tw, nullptr, nullptr, (int64_t)0, 1);
    else
        hipLaunchKernelGGL((col_kernel<T, N, false, false>), grid, dim3(SH::NT), 0, st, (cx<T> *)spec, stride,
                           s0, s1, (const cx<T> *)tw, nullptr, nullptr, (int64_t)0, 1);
    return hipGetLastError();
}

// z forward of one FP32 spectrum into the tile order of the slice-sum pass
template <int N>
static hipError_t col_z_tiled_t(const void *in, void *out, const void *tw, hipStream_t st) {
    using SH = ColShape<float, N>;
    ColSet s0, s1;
    col_sets<float, N>(2, s0, s1);
    hipLaunchKernelGGL((col_kernel<float, N, true, false, true>), dim3(s0.n_wgs + s1.n_wgs), dim3(SH::NT), 0, st,
                       (cx<float> *)in, (int64_t)0, s0, s1, (const cx<float> *)tw, nullptr, nullptr, (int64_t)0, 1,
                       (cx<float> *)out, fused_cpw(N));
    return hipGetLastError();
}

hipError_t launch_col_z_tiled(int n, const void *in, void *out, const void *tw_full, hipStream_t st) {
    if (in == out) return hipErrorInvalidValue;
#define X_(N) return col_z_tiled_t<N>(in, out, tw_full, st)
    LC_DISPATCH_N(n, X_);
#undef X_
    return hipSuccess;
}

template <int N>
static hipError_t col_comb_t(void *spec, const void *tw, const int *tab, const void *part, hipStream_t st) {
    using SH = ColShape<float, N>;
    ColSet s0, s1;
    col_sets<float, N>(1, s0, s1);
    // the fused pass tiles its N*H main columns by fused_cpw(N) columns
    const int cpw_z = fused_cpw(N);
    const int64_t tiles_main = ((int64_t)N * (N / 2) + cpw_z - 1) / cpw_z;
    hipLaunchKernelGGL((col_kernel<float, N, false, true>), dim3(s0.n_wgs + s1.n_wgs), dim3(SH::NT), 0, st,
                       (cx<float> *)spec, (int64_t)0, s0, s1, (const cx<float> *)tw, tab,
                       (const cx<float> *)part, tiles_main, cpw_z);
    return hipGetLastError();
}

hipError_t launch_col_y_inv_combine(int n, void *spec, const void *tw_full, const int *split_tab,
                                    const void *part, hipStream_t st) {
#define X_(N) return col_comb_t<N>(spec, tw_full, split_tab, part, st);
    LC_DISPATCH_N(n, X_)
#undef X_
    return hipErrorInvalidValue;
}

hipError_t launch_col_batch(int n, bool t_f64, int axis, bool fwd, void *spec, int64_t stride, int count,
                            const void *tw_full, hipStream_t st) {
    if (count < 1) return hipErrorInvalidValue;
#define X_(N)                                                                        \
    if (t_f64) return col_t<double, N>(axis, fwd, spec, stride, count, tw_full, st); \
    else return col_t<float, N>(axis, fwd, spec, stride, count, tw_full, st);
    LC_DISPATCH_N(n, X_)
#undef X_
    return hipErrorInvalidValue;
}

hipError_t launch_col(int n, bool t_f64, int axis, bool fwd, void *spec, const void *tw_full,
                      hipStream_t st) {
    return launch_col_batch(n, t_f64, axis, fwd, spec, 0, 1, tw_full, st);
}

}  // namespace lc
