// Slice sum of the convolution theorem (Eq. 13 summed over slices, algorithm
// steps 5-6 with the sum taken before the inverse transform):
//   A_b(p) = sum_k G^_{k,b}(p) S^_k(p).
// G^ is real and even in every axis, so it is stored as its non-negative
// octant and each complex product costs two real multiplies.
//
//  * mac_plain:  one launch per slice, A read-modify-written in HBM (the
//                unfused method; FP64 and plain FP32).
//  * fused_z:    per column of the y-transformed slices, the forward z
//                transform of each slice, the multiply by G^ and a
//                compensated (Kahan) sum over slices are done in registers;
//                the inverse z transform follows and A is written once.
#include "lc_fft_device.h"
#include "lc_internal.h"

namespace lc {

__device__ __forceinline__ int fold(int v, int n) { return v <= n / 2 ? v : n - v; }

// ---------------------------------------------------------------------------
// plain multiply-accumulate
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void mac_plain_kernel(cx<T> *__restrict__ A, const cx<T> *__restrict__ S,
                                                        const T *__restrict__ G, int n, int first) {
    const int64_t H = n / 2, HP = H + 1;
    const int64_t main_n = (int64_t)n * n * H;
    const int64_t total = main_n + (int64_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t gi;
        if (e < main_n) {
            const int z = (int)(e / (n * H));
            const int64_t rem = e % (n * H);
            const int y = (int)(rem / H), p = (int)(rem % H);
            gi = ((int64_t)fold(z, n) * HP + fold(y, n)) * H + p;
        } else {
            const int64_t e2 = e - main_n;
            const int z = (int)(e2 / n), y = (int)(e2 % n);
            gi = HP * HP * H + (int64_t)fold(z, n) * HP + fold(y, n);
        }
        const T g = G[gi];
        const cx<T> s = S[e];
        cx<T> v = mk(g * s.x, g * s.y);
        if (!first) v = A[e] + v;
        A[e] = v;
    }
}

hipError_t launch_mac_plain(int n, bool t_f64, void *A, const void *S, const void *ghat, bool first,
                            hipStream_t st) {
    const int64_t total = spec_elems(n);
    int wgs = (int)std::min<int64_t>((total + 255) / 256, 8192);
    if (t_f64)
        hipLaunchKernelGGL(mac_plain_kernel<double>, dim3(wgs), dim3(256), 0, st, (cx<double> *)A,
                           (const cx<double> *)S, (const double *)ghat, n, first ? 1 : 0);
    else
        hipLaunchKernelGGL(mac_plain_kernel<float>, dim3(wgs), dim3(256), 0, st, (cx<float> *)A,
                           (const cx<float> *)S, (const float *)ghat, n, first ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fused z pass (FP32)
// ---------------------------------------------------------------------------
struct FusedDev {
    const cx<float> *spec;
    int64_t spec_stride;
    const float *ghat;
    int64_t oct_stride;
    int32_t B, band0, K0, K1;   // kcount of the two handled bands
    cx<float> *acc;
    int64_t acc_stride;
    int32_t zero_dc, kahan;
};

template <int L, int NB_>
__global__ __launch_bounds__((ColShape<float, L>::NT)) void fused_z_kernel(FusedDev a, ColSet s0, ColSet s1,
                                                                         const cx<float> *__restrict__ tw) {
    using SH = ColShape<float, L>;
    constexpr int CPW = SH::CPW, NT = SH::NT, PAD = SH::PAD, ES = CPW + PAD, TPL = SH::TPL;
    constexpr int NP = Sched<L>::NP;
    constexpr int RL = pass_radix<L, true>(NP - 1);          // last forward radix
    constexpr int NSL = ns_before<L, true>(NP - 1);           // = L / RL
    using PL = Pass<float, L, RL, NSL, TPL, true>;            // last forward pass
    using PI = Pass<float, L, RL, 1, TPL, false>;             // first inverse pass
    constexpr int BPT = PL::BPT;
    static_assert(NSL * RL == L, "schedule");
    __shared__ cx<float> lds[L * ES];

    const bool is_main = (int)blockIdx.x < s0.n_wgs;
    const ColSet &s = is_main ? s0 : s1;
    const int64_t col0 = (int64_t)(is_main ? blockIdx.x : blockIdx.x - s0.n_wgs) * CPW;
    const int c = threadIdx.x % CPW, t = threadIdx.x / CPW;
    const int64_t col = col0 + c;
    const bool col_ok = col < s.n_cols;
    const int H = L / 2, HP = H + 1;

    // octant offset of this thread's elements (rows r = out_pos) in one G^ slice
    int goff[BPT][RL];
    {
        int qf, p, base_main;
        if (is_main) {
            const int cc = col_ok ? (int)col : 0;
            qf = fold(cc / H, L); p = cc % H;
            base_main = 1;
        } else {
            qf = fold(col_ok ? (int)col : 0, L); p = H;
            base_main = 0;
        }
#pragma unroll
        for (int i = 0; i < BPT; ++i)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int row = PL::out_pos(t, i, r);
                const int rf = fold(row < L ? row : 0, L);
                goff[i][r] = base_main ? (rf * HP + qf) * H + p
                                       : HP * HP * H + rf * HP + qf;
            }
    }

    cx<float> sum[NB_][BPT][RL], cmp[NB_][BPT][RL];
#pragma unroll
    for (int b = 0; b < NB_; ++b)
#pragma unroll
        for (int i = 0; i < BPT; ++i)
#pragma unroll
            for (int r = 0; r < RL; ++r) { sum[b][i][r] = mk(0.f, 0.f); cmp[b][i][r] = mk(0.f, 0.f); }

    const int kmax = (NB_ > 1 && a.K1 > a.K0) ? a.K1 : a.K0;
    for (int k = 0; k < kmax; ++k) {
        tile_load<float, L, CPW, NT, PAD>(lds, a.spec + (int64_t)k * a.spec_stride, s, col0);
        __syncthreads();
        run_passes<float, L, true, 0, NP - 1>(lds, c, ES, t, true, tw);
        cx<float> v[BPT][RL];
        PL::read(lds, c, ES, t, tw, v);
        __syncthreads();   // LDS free for the next slice
#pragma unroll
        for (int b = 0; b < NB_; ++b) {
            const int kc = b == 0 ? a.K0 : a.K1;
            if (k >= kc) continue;
            const float *g = a.ghat + ((int64_t)k * a.B + a.band0 + b) * a.oct_stride;
#pragma unroll
            for (int i = 0; i < BPT; ++i)
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    const float gv = col_ok ? g[goff[i][r]] : 0.f;
                    const float px = gv * v[i][r].x, py = gv * v[i][r].y;
                    if (a.kahan) {
                        const float yx = px - cmp[b][i][r].x, yy = py - cmp[b][i][r].y;
                        const float tx = sum[b][i][r].x + yx, ty = sum[b][i][r].y + yy;
                        cmp[b][i][r].x = (tx - sum[b][i][r].x) - yx;
                        cmp[b][i][r].y = (ty - sum[b][i][r].y) - yy;
                        sum[b][i][r].x = tx;
                        sum[b][i][r].y = ty;
                    } else {
                        sum[b][i][r].x += px;
                        sum[b][i][r].y += py;
                    }
                }
        }
    }

    // the (0,0,0) bin: element row 0 of main column 0
    const bool has_dc = a.zero_dc && is_main && col == 0;

#pragma unroll
    for (int b = 0; b < NB_; ++b) {
        cx<float> v[BPT][RL];
#pragma unroll
        for (int i = 0; i < BPT; ++i)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                v[i][r] = a.kahan ? sum[b][i][r] - cmp[b][i][r] : sum[b][i][r];
                if (has_dc && PL::out_pos(t, i, r) == 0) v[i][r] = mk(0.f, 0.f);
            }
        // first inverse pass straight from registers (positions match)
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            const int bb = t + i * TPL;
            if (PI::EVEN || bb < PI::NB) dft<RL, false>(v[i]);
        }
        PI::write(lds, c, ES, t, v);
        __syncthreads();
        run_passes<float, L, false, 1, NP>(lds, c, ES, t, true, tw);
        tile_store<float, L, CPW, NT, PAD>(a.acc + (int64_t)b * a.acc_stride, lds, s, col0);
        __syncthreads();
    }
}

template <int N>
static hipError_t fused_t(const FusedArgs &fa, const void *tw, hipStream_t st) {
    using SH = ColShape<float, N>;
    const int64_t H = N / 2;
    ColSet s0, s1;
    // main: columns (q, p) flat q*H + p; element (row r) at r*N*H + col
    s0.n_cols = (int64_t)N * H; s0.W = (int64_t)N * H; s0.plane_stride = 0; s0.col_stride = 1;
    s0.row_stride = (int64_t)N * H; s0.off = 0; s0.rowfast = 0;
    // nyq: columns q; element (row r) at main + r*N + q
    s1.n_cols = N; s1.W = N; s1.plane_stride = 0; s1.col_stride = 1; s1.row_stride = N;
    s1.off = spec_main(N); s1.rowfast = 0;
    s0.n_wgs = (int32_t)((s0.n_cols + SH::CPW - 1) / SH::CPW);
    s1.n_wgs = (int32_t)((s1.n_cols + SH::CPW - 1) / SH::CPW);
    FusedDev d;
    d.spec = (const cx<float> *)fa.spec; d.spec_stride = fa.spec_stride;
    d.ghat = (const float *)fa.ghat; d.oct_stride = fa.oct_stride;
    d.B = fa.B; d.band0 = fa.band0; d.K0 = fa.kcount[0]; d.K1 = fa.kcount[1];
    d.acc = (cx<float> *)fa.acc; d.acc_stride = fa.acc_stride;
    d.zero_dc = fa.zero_dc; d.kahan = fa.kahan;
    const int wgs = s0.n_wgs + s1.n_wgs;
    if (fa.nband == 2)
        hipLaunchKernelGGL((fused_z_kernel<N, 2>), dim3(wgs), dim3(SH::NT), 0, st, d, s0, s1,
                           (const cx<float> *)tw);
    else
        hipLaunchKernelGGL((fused_z_kernel<N, 1>), dim3(wgs), dim3(SH::NT), 0, st, d, s0, s1,
                           (const cx<float> *)tw);
    return hipGetLastError();
}

hipError_t launch_fused_z(int n, const FusedArgs &a, const void *tw_full, hipStream_t st) {
    if (a.nband < 1 || a.nband > 2) return hipErrorInvalidValue;
    switch (n) {
#define X_(N) case N: return fused_t<N>(a, tw_full, st);
        X_(8) X_(12) X_(16) X_(24) X_(32) X_(48) X_(64) X_(96) X_(128) X_(192) X_(256) X_(384) X_(512)
#undef X_
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// FP64 mean (DC) of each band: mu_b = sum_k G^_{k,b}(0) S^_k(0) / N^3
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void dc_reduce_kernel(const double *__restrict__ dcpart, int K, int W,
                                                        const double *__restrict__ g0, int B,
                                                        double inv_n3, double *__restrict__ mu) {
    __shared__ double red[256];
    __shared__ double sk[1024];
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int w = threadIdx.x; w < W; w += 256) s += dcpart[(int64_t)k * W + w];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) sk[k] = red[0];
        __syncthreads();
    }
    if ((int)threadIdx.x < B) {
        double m = 0.0;
        for (int k = 0; k < K; ++k) m += g0[(int64_t)k * B + threadIdx.x] * sk[k];
        mu[threadIdx.x] = m * inv_n3;
    }
}

hipError_t launch_dc_reduce(const double *dcpart, int K, int W, const double *g0, int B,
                            double inv_n3, double *mu, hipStream_t st) {
    if (K > 1024 || B > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(dc_reduce_kernel, dim3(1), dim3(256), 0, st, dcpart, K, W, g0, B, inv_n3, mu);
    return hipGetLastError();
}

}  // namespace lc
