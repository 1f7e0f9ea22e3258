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
//                Slices left in the parity y layout by the half-plane xy
//                pass get their last y radix-2 step on the way in, two
//                output columns per input column.
#include <type_traits>

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
// fused z pass (FP32), persistent with a balanced ("stream-K") partition
//
// The work is the sequence of (tile, slice) pairs, tile-major; tile t covers
// CPW columns and its slices k < kmax. Workgroup w of P takes the pairs
// [w W / P, (w+1) W / P), W = tiles * kmax, so every workgroup gets the same
// number of slice-tiles up to one. Since W / P >= kmax, a tile is split
// between at most two workgroups: the part starting at k = 0 is written to
// the accumulator spectrum, the other part (starting at an interior k) to a
// side buffer slot owned by the workgroup that computed it; the inverse y
// pass adds it back when it loads the tile.
// ---------------------------------------------------------------------------
struct FusedDev {
    const cx<float> *spec;
    int64_t spec_stride;
    const float *ghat;
    int64_t oct_stride;
    int32_t B, band0, nb;       // bands in the G^ layout, first handled band, handled bands
    int32_t Kc[4];              // kcount of the handled bands (0 past nb)
    cx<float> *acc;
    int64_t acc_stride;
    cx<float> *part;            // [band][P][L * CPW]
    int64_t part_stride;
    int32_t zero_dc, kahan;
    int32_t kmax, P;
    int64_t W;
    int32_t rounds;            // 1: whole tiles w, w+P, ... (no split tiles)
    int64_t tiles;
    const double *sk, *g0;     // band means (mu non-null): see FusedArgs
    double inv_n3;
    double *mu;
    int32_t K;
    int32_t ring;              // lookback k lives in spectrum slot (k + ring) mod K
    int32_t frozen;            // >= 0: every lookback slice reads slot `frozen` (instantaneous field)
};

// Processing order of the main tiles in the rounds schedule. Main tile
// q*NPB + pb covers columns p in [pb*CPW, (pb+1)*CPW) of row q (NPB tiles
// per row). Its kernel octant rows (folded q) are CPW floats, so GP =
// 32 / CPW neighbouring p-blocks share each 128-byte octant line, and the
// rows q and q' = N - q (0 <-> N/2) fold to the same octant row: the 2*GP
// tiles {q, q'} x {GP p-blocks} read the same octant lines (and, for
// CPW < 16, the same spectrum lines). Workgroups w, w+8, w+16, ... run on
// one XCD (workgroups are dispatched to the 8 XCDs in turn), so slot s of
// a block of 16*GP consecutive slots takes member (s % (16 GP)) / 8 of
// group 8 * (s / (16 GP)) + s % 8: the readers of a line are resident
// together on one XCD and it comes from that XCD's L2 once. Other tile
// counts, and tiles that do not split rows evenly (npb = 0), keep the
// identity order; the result is always a main tile when slot is one.
// With spectra in the parity layout, a tile covers rows q and q + N/2
// (q < N/2) and the same pairing runs with N/2 in place of N: the octant
// rows of tiles q and N/2 - q are {q, N/2 - q} for both.
__device__ __forceinline__ int64_t fused_slot_tile(int64_t slot, int64_t main_tiles, int n, int npb, int gp) {
    const int bs = 16 * gp;
    if (slot >= main_tiles || gp < 1 || npb < gp || npb % gp || main_tiles % bs ||
        (int64_t)n * npb != main_tiles)
        return slot;
    const int64_t blk = slot / bs;
    const int xcd = (int)(slot & 7), j = (int)((slot % bs) >> 3);
    const int64_t g = blk * 8 + xcd;
    const int ngp = npb / gp;
    const int q = (int)(g / ngp), pb = gp * (int)(g % ngp) + (j % gp);
    const int row = j < gp ? q : (q == 0 ? n / 2 : n - q);
    const int64_t tile = (int64_t)row * npb + pb;
    return tile < main_tiles ? tile : slot;
}

// PAR: the slice spectra are in the parity layout of the half-plane xy
// shapes (rows r < N/2 of a z-plane hold the y transform E of the even rows,
// rows N/2 + r that of the odd rows O). A column (q, p) with q < N/2 then
// yields the two columns of rows q and q + N/2 of the length-N y transform,
//   T[q] = E + W_N^q O,   T[q + N/2] = E - W_N^q O
// (its last radix-2 step), formed on the way to the first butterfly: each
// input element is read once for both, and both go through the z transform,
// the kernel product and the compensated sum. Output o of a column is at
// o * (N/2 rows) after the first; a second part goes to part slot 2 w + o.
template <int L, int NB_, typename S, int PF, int IN>
__global__ __launch_bounds__((FusedShape<L, S>::NT)) void fused_z_kernel(FusedDev a, ColSet s0, ColSet s1,
                                                                        const cx<float> *__restrict__ tw_g) {
    // input: 0 y-transformed slices, 1 the same in the parity layout, 2
    // slices already transformed along z as well (3D spectra: no forward z
    // transform here, the slice loop is the product and the sum)
    constexpr bool PAR = IN == 1, PRE = IN == 2;
    using SH = FusedShape<L, S>;
    using EF = Engine<float, L, true, S>;     // forward z transform
    using EI = Engine<float, L, false, S>;    // inverse z transform
    constexpr int CPW = SH::CPW, NT = SH::NT, ES = CPW + SH::PAD, E = EF::E;
    static_assert(EI::E == E, "forward and inverse hold the same elements");
    constexpr int HP = L / 2 + 1;
    constexpr int RSTEP = NT / CPW;                        // = threads per column
    constexpr int GROWS = (HP + RSTEP - 1) / RSTEP;        // octant rows loaded per thread
    constexpr int NO = PAR ? 2 : 1;                        // output columns per input column
    // compensated (Kahan) sums for one or two bands per launch; four bands
    // per launch keep plain FP32 sums (their compensation terms would not
    // fit in registers beside the sums)
    constexpr bool CS = NB_ <= 2;
    // pair tiles of one band: the two outputs' transforms run interleaved
    // (Engine::first2_db / rest2_db), two barriers per slice instead of four
    constexpr bool IL = PAR && NB_ == 1 && EF::NP > 1;
    // z transform line buffers, alternated by exchange (Engine::run_db):
    // only the barriers after the writes remain in the slice loop; lds3 and
    // lds4 are the second output's pair in the interleaved form
    __shared__ cx<float> lds[L * ES], lds2[L * ES];
    __shared__ cx<float> lds3[IL ? L * ES : 1], lds4[IL ? L * ES : 1];
    __shared__ cx<float> tws[L];
    // kernel octant rows of the tile (all folded z frequencies), per output:
    // rows r and L-r of a column share one entry. Double buffered by slice;
    // one buffer in the interleaved form, which stores slice k's rows after
    // the first barrier of slice k (every reader of slice k-1's rows has
    // passed it) and reads them after the second.
    constexpr int GB = IL ? 1 : 2;
    __shared__ float gl[GB][NB_ * NO][HP * CPW];
    for (int i = threadIdx.x; i < L; i += NT) tws[i] = tw_g[i];
    // the FP64 band means (DC mode), once per launch, by the first wave of
    // workgroup 0: mu_b = inv_n3 sum_k G^_{k,b}(0) S^_k(0)
    if (a.mu && blockIdx.x == 0 && threadIdx.x < 64) {
#pragma unroll
        for (int b = 0; b < NB_; ++b) {
            if (b >= a.nb) break;
            double v = 0.0;
            for (int k = threadIdx.x; k < a.K; k += 64) {
                const int slot = a.frozen >= 0 ? a.frozen : (k + a.ring < a.K ? k + a.ring : k + a.ring - a.K);
                v += a.g0[(int64_t)k * a.B + a.band0 + b] * a.sk[slot];
            }
            for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
            if (threadIdx.x == 0) a.mu[a.band0 + b] = v * a.inv_n3;
        }
    }

    const int c = threadIdx.x % CPW, t = threadIdx.x / CPW;
    const int H = L / 2;
    const int w = blockIdx.x;
    int64_t pos = (int64_t)w * a.W / a.P;
    const int64_t end = (int64_t)(w + 1) * a.W / a.P;

    auto segment = [&](const int64_t tile, const int k0, const int k1) {

        // readers of the LDS buffers in the previous segment are done
        lds_barrier();
        const bool is_main = tile < s0.n_wgs;
        const ColSet &s = is_main ? s0 : s1;
        const int64_t col0 = (is_main ? tile : tile - s0.n_wgs) * CPW;
        const int64_t col = col0 + c;
        const bool col_ok = col < s.n_cols;
        // columns past the end compute on a valid column and are not stored
        const int64_t ccol = col_ok ? col : col0;
        const int64_t cbase = col_base(s, ccol);
        // row (y frequency) of the column; in the parity layout the second
        // output and the O input are obase elements further
        const int q = is_main ? (int)(ccol / H) : (int)ccol;
        const int64_t obase = is_main ? (int64_t)H * H : (int64_t)H;
        const cx<float> wq = tws[PAR ? q : 0];   // W_N^q

        // octant offset of this thread's column in one G^ slice; the row
        // part (folded z frequency) is added per element. The second output
        // (row q + N/2) is gdel floats further.
        int gbase, grow, gdel = 0;
        if (is_main) {
            const int cc = (int)ccol;
            gbase = fold(q, L) * H + cc % H;
            grow = HP * H;
            if constexpr (PAR) gdel = (fold(q + H, L) - fold(q, L)) * H;
        } else {
            gbase = HP * HP * H + fold(q, L);
            grow = HP;
            if constexpr (PAR) gdel = fold(q + H, L) - fold(q, L);
        }

        cx<float> sum[NO][NB_][E], cmp[NO][CS ? NB_ : 1][CS ? E : 1];
#pragma unroll
        for (int o = 0; o < NO; ++o)
#pragma unroll
            for (int b = 0; b < NB_; ++b)
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    sum[o][b][e] = mk(0.f, 0.f);
                    if constexpr (CS) cmp[o][b][e] = mk(0.f, 0.f);
                }

        // Byte offsets, off workgroup-uniform bases (a slice spectrum is below
        // 4 GiB): of this thread's first input element, the others being whole
        // rows further (compile-time row deltas, folded into the uniform base),
        // and of the kernel octant rows it loads (rows t + j*RSTEP of its
        // column: uniform deltas too, except the last row, which is clamped
        // for the threads past the octant's end). One offset register each
        // instead of one per element.
        // (3D spectra are read at the forward transform's output positions,
        // from the tile order their z pass writes: the tile's rows of w
        // columns contiguous, w = CPW except in a set's last tile)
        auto rowpos = [&](int e) { return PRE ? EF::out_pos(t, e) : EF::in_pos(t, e); };
        int64_t in0 = cbase, in_rs = s.row_stride;
        if constexpr (PRE) {
            const int64_t w = s.n_cols - col0 < CPW ? s.n_cols - col0 : CPW;
            in0 = (is_main ? 0 : spec_main(L)) + col0 * L + (ccol - col0);
            in_rs = w;
        }
        const uint32_t xoff0 = (uint32_t)((in0 + (int64_t)rowpos(0) * in_rs) * 8);
        const int64_t rs8 = in_rs * 8;
        auto xld = [&](const char *base, int e) {
            return *(const cx<float> *)(base + (int64_t)(rowpos(e) - rowpos(0)) * rs8 + xoff0);
        };
        constexpr bool GFULL = GROWS * RSTEP <= HP;   // every thread's last row exists
        const int rlast = t + (GROWS - 1) * RSTEP;
        const uint32_t goff0 = (uint32_t)((gbase + t * grow) * 4);
        const uint32_t goffl = (uint32_t)((gbase + (rlast < HP ? rlast : 0) * grow) * 4);
        const int64_t gr4 = (int64_t)grow * 4 * RSTEP;
        // LDS slot of each output element's kernel value (folded row)
        int gslot[E];
#pragma unroll
        for (int e = 0; e < E; ++e) gslot[e] = fold(EF::out_pos(t, e), L) * CPW + c;

        // The slice loop runs to a multiple of PF with no branch in its body:
        // slices past k1 read slice k1-1 again (valid, recently read memory)
        // with kernel weight 0, which leaves the compensated sum's value
        // unchanged. Branch-free, every wait for a load counts exactly the
        // loads issued after it, so the prefetched slices stay in flight.
        const int kend = k0 + (k1 - k0 + PF - 1) / PF * PF;
        auto spec_at = [&](int k) {
            int slot = (k < k1 ? k : k1 - 1) + a.ring;
            if (slot >= a.K) slot -= a.K;
            if (a.frozen >= 0) slot = a.frozen;
            return (const char *)(a.spec + (int64_t)slot * a.spec_stride);
        };
        // first-pass inputs of the next PF slices, kept in flight in a ring of
        // register buffers (PF slices of HBM latency hidden behind compute);
        // in the parity layout ob holds the O halves
        constexpr int PO = PAR ? PF : 1;
        cx<float> xb[PF][E], ob[PO][E];
        const int64_t obytes = obase * 8;
        auto fill = [&](int j, int k) {
            const char *src = spec_at(k);
#pragma unroll
            for (int e = 0; e < E; ++e) xb[j][e] = xld(src, e);
            if constexpr (PAR) {
                const char *srco = src + obytes;
#pragma unroll
                for (int e = 0; e < E; ++e) ob[j][e] = xld(srco, e);
            }
        };
#pragma unroll
        for (int j = 0; j < PF; ++j) fill(j, k0 + j);
        // kernel octant rows of slice k are loaded one slice ahead into
        // registers and stored to LDS during slice k; a band without a kernel
        // for slice k reads a valid octant with weight 0. The weight is
        // applied at the LDS store, not at the load: arithmetic on the loaded
        // values right away would wait for every load in flight before them,
        // the prefetched slices included.
        float gn[NB_][NO][GROWS], gw[NB_];
        auto load_g = [&](int k) {
#pragma unroll
            for (int b = 0; b < NB_; ++b) {
                const int kc = a.Kc[b];
                const bool on = k < kc && k < k1;
                const int kb = on ? k : 0;
                gw[b] = on ? 1.f : 0.f;
                // (a band past nb reads the first handled band's octant)
                const int bb = b < a.nb ? b : 0;
                const char *gp = (const char *)(a.ghat + ((int64_t)kb * a.B + a.band0 + bb) * a.oct_stride);
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    // the second output's rows are gdel floats away (gdel < 0
                    // for q > N/4): the offset is formed in 32 bits, where it
                    // wraps to the true (nonnegative) offset, before the add
                    const uint32_t od = (uint32_t)(o * gdel) * 4u;
#pragma unroll
                    for (int j = 0; j < GROWS; ++j)
                        gn[b][o][j] = (j < GROWS - 1 || GFULL)
                                          ? *(const float *)(gp + j * gr4 + (uint32_t)(goff0 + od))
                                          : *(const float *)(gp + (uint32_t)(goffl + od));
                }
            }
        };
        // octant rows of slice k go to LDS buffer k&1, whose previous
        // contents (slice k-2) were last read before the barriers of slice k-1
        auto store_g = [&](int k) {
            float *glk = &gl[(k & 1) % GB][0][0];
#pragma unroll
            for (int b = 0; b < NB_; ++b)
#pragma unroll
                for (int o = 0; o < NO; ++o)
#pragma unroll
                    for (int jj = 0; jj < GROWS; ++jj) {
                        const int rf = t + jj * RSTEP;
                        if (rf < HP) glk[(b * NO + o) * HP * CPW + rf * CPW + c] = gw[b] * gn[b][o][jj];
                    }
        };
        // compensated (Kahan) sum over slices of output o, or the plain sum
        auto mac = [&](int o, const float *glk, const cx<float>(&v)[E]) {
#pragma unroll
            for (int b = 0; b < NB_; ++b)
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const float gv = glk[(b * NO + o) * HP * CPW + gslot[e]];
                    if constexpr (CS) {
                        const float yx = gv * v[e].x - cmp[o][b][e].x, yy = gv * v[e].y - cmp[o][b][e].y;
                        const float tx = sum[o][b][e].x + yx, ty = sum[o][b][e].y + yy;
                        cmp[o][b][e].x = (tx - sum[o][b][e].x) - yx;
                        cmp[o][b][e].y = (ty - sum[o][b][e].y) - yy;
                        sum[o][b][e].x = tx;
                        sum[o][b][e].y = ty;
                    } else {
                        sum[o][b][e] = mk(fmaf(gv, v[e].x, sum[o][b][e].x), fmaf(gv, v[e].y, sum[o][b][e].y));
                    }
                }
        };
        load_g(k0);
        if constexpr (IL) {
            for (int kk = k0; kk < kend; kk += PF) {
#pragma unroll
                for (int j = 0; j < PF; ++j) {
                    const int k = kk + j;
                    // last radix-2 step of the y transform: E +- W_N^q O
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const cx<float> x = xb[j][e], y = ob[j][e];
                        const float ux = fmaf(wq.x, y.x, -wq.y * y.y), uy = fmaf(wq.x, y.y, wq.y * y.x);
                        xb[j][e] = mk(x.x + ux, x.y + uy);
                        ob[j][e] = mk(x.x - ux, x.y - uy);
                    }
                    EF::first2_db(xb[j], ob[j], lds, lds3, c, ES, t);
                    // buffer j is free: refill it with slice k + PF
                    fill(j, k + PF);
                    EF::rest2_db(
                        lds, lds2, lds3, lds4, c, ES, t, tws,
                        [&] {
                            // slice k's octant rows (loaded during slice k - 1),
                            // then slice k + 1's in flight
                            store_g(k);
                            load_g(k + 1);
                        },
                        [&](int o, const cx<float>(&v)[E]) { mac(o, &gl[0][0][0], v); });
                }
            }
        } else if constexpr (PRE) {
            store_g(k0);
            for (int kk = k0; kk < kend; kk += PF) {
#pragma unroll
                for (int j = 0; j < PF; ++j) {
                    const int k = kk + j;
                    const float *glk = &gl[k & 1][0][0];
                    load_g(k + 1);
                    // slice k's octant rows (stored at the end of slice k - 1)
                    // are visible, and every reader of slice k - 1's rows is
                    // done before they are overwritten at the end of this slice
                    lds_barrier();
                    cx<float> v[E];
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e] = xb[j][e];
                    fill(j, k + PF);
                    mac(0, glk, v);
                    store_g(k + 1);
                }
            }
        } else {
            store_g(k0);
            for (int kk = k0; kk < kend; kk += PF) {
#pragma unroll
                for (int j = 0; j < PF; ++j) {
                    const int k = kk + j;
                    const float *glk = &gl[k & 1][0][0];
                    // the next slice's octant rows are in flight during this slice
                    load_g(k + 1);
                    if constexpr (PAR) {
                        // last radix-2 step of the y transform: E +- W_N^q O
#pragma unroll
                        for (int e = 0; e < E; ++e) {
                            const cx<float> x = xb[j][e], y = ob[j][e];
                            const float ux = fmaf(wq.x, y.x, -wq.y * y.y), uy = fmaf(wq.x, y.y, wq.y * y.x);
                            xb[j][e] = mk(x.x + ux, x.y + uy);
                            ob[j][e] = mk(x.x - ux, x.y - uy);
                        }
                    }
                    EF::first_db(xb[j], lds, c, ES, t);
                    cx<float> v[E];
                    if constexpr (EF::NP == 1) {
#pragma unroll
                        for (int e = 0; e < E; ++e) v[e] = xb[j][e];
                        lds_barrier();    // kernel values in LDS visible
                    }
                    // buffer j is free (both halves once the second output has
                    // entered its transform): refill it with slice k + PF
                    if constexpr (!PAR) fill(j, k + PF);
                    if constexpr (EF::NP > 1) EF::rest_db(xb[j], v, lds, lds2, c, ES, t, tws);
                    mac(0, glk, v);
                    if constexpr (PAR) {
                        EF::first_db(ob[j], lds, c, ES, t);
                        if constexpr (EF::NP == 1) {
#pragma unroll
                            for (int e = 0; e < E; ++e) v[e] = ob[j][e];
                        }
                        fill(j, k + PF);
                        if constexpr (EF::NP > 1) EF::rest_db(ob[j], v, lds, lds2, c, ES, t, tws);
                        mac(1, glk, v);
                    }
                    // stored at the end of the slice, after the refill loads were
                    // issued, so that waiting for them does not wait for the refill
                    store_g(k + 1);
                }
            }
        }

        // the (0,0,0) bin: row 0 of main column 0
        const bool has_dc = a.zero_dc && is_main && col == 0;
        const bool primary = k0 == 0;
        auto put = [&](int b, int o, const cx<float>(&y)[E]) {
            if (primary) {
                cx<float> *dst = a.acc + (int64_t)b * a.acc_stride + o * obase;
                if (col_ok)
#pragma unroll
                    for (int e = 0; e < E; ++e)
                        dst[(uint32_t)(cbase + (int64_t)EI::out_pos(t, e) * s.row_stride)] = y[e];
            } else {
                cx<float> *dst = a.part + (int64_t)b * a.part_stride + (int64_t)(NO * w + o) * (L * CPW) + c;
#pragma unroll
                for (int e = 0; e < E; ++e) dst[EI::out_pos(t, e) * CPW] = y[e];
            }
        };
#pragma unroll
        for (int b = 0; b < NB_; ++b) {
            if (b >= a.nb) break;   // (uniform: the barriers below stay matched)
            cx<float> y[NO][E];
#pragma unroll
            for (int o = 0; o < NO; ++o) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if constexpr (CS) {
                        y[o][e] = sum[o][b][e] - cmp[o][b][e];
                    } else {
                        y[o][e] = sum[o][b][e];
                    }
                    if (o == 0 && has_dc && EF::out_pos(t, e) == 0) y[o][e] = mk(0.f, 0.f);
                }
                // the last forward pass's placement is the first inverse pass's
                EI::run_db(y[o], lds, lds2, c, ES, t, tws);
            }
            if constexpr (PAR) {
                // first radix-2 step of the inverse y transform, split by the
                // parity s of the output rows y = 2m + s:
                //   U_0 = T[q] + T[q + N/2],  U_1 = W_N^-q (T[q] - T[q + N/2])
                // (the inverse y pass of rows of parity s is the N/2-point
                // inverse transform of U_s), stored in the places of T[q] and
                // T[q + N/2]
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const cx<float> u = y[0][e], v = y[1][e];
                    const cx<float> d = mk(u.x - v.x, u.y - v.y);
                    y[0][e] = mk(u.x + v.x, u.y + v.y);
                    y[1][e] = mk(fmaf(wq.x, d.x, wq.y * d.y), fmaf(wq.x, d.y, -wq.y * d.x));   // conj(W^q) d
                }
            }
#pragma unroll
            for (int o = 0; o < NO; ++o) put(b, o, y[o]);
        }
        };
    if (a.rounds) {
        // whole tiles in rounds: all workgroups sweep the slices together
        // main tiles per row (0: rows do not split into whole tiles, identity order)
        const int npb = (L / 2) % CPW == 0 ? (int)((L / 2) / CPW) : 0;
        constexpr int GP = CPW >= 32 ? 1 : 32 / CPW;
        const int nrow = PAR ? L / 2 : L;
        const int64_t full = a.tiles / a.P * a.P;   // slots of the whole rounds
        for (int64_t slot = w; slot < full; slot += a.P)
            segment(fused_slot_tile(slot, s0.n_wgs, nrow, npb, GP), 0, a.kmax);
        // the tiles of the remaining slots (fewer than P) would leave most
        // workgroups idle for a whole round: their (tile, slice) pairs are
        // split evenly over all workgroups instead. Only a workgroup's first
        // segment can start inside a tile; it goes to the workgroup's part
        // slot, and fused_rest_merge_kernel adds the parts of each tile.
        const int64_t U = (a.tiles - full) * a.kmax;
        int64_t u = (int64_t)w * U / a.P;
        const int64_t ue = (int64_t)(w + 1) * U / a.P;
        while (u < ue) {
            const int64_t i = u / a.kmax;
            const int k0 = (int)(u % a.kmax);
            const int k1 = (int)std::min<int64_t>(a.kmax, k0 + (ue - u));
            u += k1 - k0;
            segment(fused_slot_tile(full + i, s0.n_wgs, nrow, npb, GP), k0, k1);
        }
    } else {
        while (pos < end) {
            const int64_t tile = pos / a.kmax;
            const int k0 = (int)(pos % a.kmax);
            const int k1 = (int)std::min<int64_t>(a.kmax, k0 + (end - pos));
            pos += k1 - k0;
            segment(tile, k0, k1);
        }
    }
}

// Parts of the tiles split by slices after the whole rounds (the rounds
// schedule's remaining slots full .. full + rest - 1): slice unit u of those
// tiles (u = i kmax + k for remaining tile i) belongs to workgroup w with
// w U / P <= u < (w + 1) U / P, U = rest kmax. The workgroup whose range holds
// unit i kmax wrote tile i to the accumulator; every other workgroup whose
// range starts inside tile i left its part in slot NO w + o (output o).
// The parts are added in a fixed order (within each quarter of the range in
// workgroup order, then the quarters in order), so the result does not
// depend on timing.
struct RestMerge {
    cx<float> *acc;
    int64_t acc_stride;
    const cx<float> *part;
    int64_t part_stride;
    int32_t nband, no, cpw, L;
    int64_t full, rest, kmax, P;
    int32_t npb, gp, nrow;
};

// Workgroup: 64 consecutive elements of one (tile, output, band); its four
// waves sum a quarter of the parts each (eight loads in flight at a time)
// and wave 0 adds the four partial sums in wave order.
__global__ __launch_bounds__(256) void fused_rest_merge_kernel(RestMerge m, ColSet s0, ColSet s1) {
    __shared__ cx<float> red[3][64];
    const int64_t per = (int64_t)m.L * m.cpw;
    const int64_t chunks = (per + 63) / 64;
    const int64_t g = blockIdx.x;
    const int64_t ch = g % chunks;
    int64_t r = g / chunks;
    const int b = (int)(r % m.nband);
    r /= m.nband;
    const int o = (int)(r % m.no);
    const int64_t i = r / m.no;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t e = ch * 64 + lane;
    const bool ok_e = e < per;
    const int64_t U = m.rest * m.kmax, lo = i * m.kmax, hi = lo + m.kmax;
    // workgroups whose range starts inside the tile: w U / P in (lo, hi),
    // i.e. w in [ceil((lo + 1) P / U), ceil(hi P / U))
    const int64_t w0 = ((lo + 1) * m.P + U - 1) / U;
    const int64_t w1 = std::min<int64_t>(m.P, (hi * m.P + U - 1) / U);
    const int64_t nq = (w1 - w0 + 3) / 4;
    const int64_t qa = w0 + wv * nq, qb = std::min<int64_t>(w1, qa + nq);
    const cx<float> *src = m.part + (int64_t)b * m.part_stride + o * per + (ok_e ? e : 0);
    cx<float> v = mk(0.f, 0.f);
    for (int64_t w = qa; w < qb; w += 8) {
        cx<float> t[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t ww = w + j;
            const bool on = ok_e && ww < qb && (ww + 1) * U / m.P > ww * U / m.P;   // non-empty range
            t[j] = on ? src[m.no * ww * per] : mk(0.f, 0.f);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) v = v + t[j];
    }
    if (wv > 0) red[wv - 1][lane] = v;
    __syncthreads();
    if (wv > 0 || !ok_e) return;
    v = v + red[0][lane];
    v = v + red[1][lane];
    v = v + red[2][lane];
    const int z = (int)(e / m.cpw), c = (int)(e % m.cpw);
    const int64_t tile = fused_slot_tile(m.full + i, s0.n_wgs, m.nrow, m.npb, m.gp);
    const bool is_main = tile < s0.n_wgs;
    const ColSet &s = is_main ? s0 : s1;
    const int64_t col = (is_main ? tile : tile - s0.n_wgs) * m.cpw + c;
    if (col >= s.n_cols) return;
    const int64_t H = m.L / 2;
    const int64_t obase = is_main ? H * H : H;
    cx<float> *dst = m.acc + (int64_t)b * m.acc_stride + o * obase + col_base(s, col) + (int64_t)z * s.row_stride;
    *dst = *dst + v;
}

// tab[t] = the workgroup holding the second part of tile t, or -1. With
// two outputs per tile (parity layout: pair tiles, main_k of them main),
// the entries go to the tiles of both output rows, as part slots 2 w + o.
__global__ __launch_bounds__(256) void fused_split_kernel(int *__restrict__ tab, int64_t tiles, int64_t kmax,
                                                          int64_t P, int64_t W, int32_t pair, int64_t main_k) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tiles) return;
    const int64_t lo = t * kmax;
    const int64_t wc = ((lo + 1) * P + W - 1) / W;      // first workgroup starting after lo
    int v = -1;
    if (wc < P) {
        const int64_t st = wc * W / P;
        if (st > lo && st < lo + kmax) v = (int)wc;
    }
    if (!pair) {
        tab[t] = v;
        return;
    }
    // standard tiles: main rows q < N/2 keep their index, rows q + N/2 are
    // main_k further; nyq tiles follow the 2 main_k main ones, likewise
    const int64_t nyq_k = tiles - main_k;
    const int64_t t0 = t < main_k ? t : 2 * main_k + (t - main_k);
    const int64_t t1 = t0 + (t < main_k ? main_k : nyq_k);
    tab[t0] = v < 0 ? -1 : 2 * v;
    tab[t1] = v < 0 ? -1 : 2 * v + 1;
}

// Schedule that fixes the tiling of the fused pass for N: the 16-element
// schedule, except at N = 384 and 512, where only the 8-element one keeps
// its per-band compensated sums and prefetch ring in registers.
template <int N> constexpr bool fused_sched8_only() { return N == 384 || N == 512; }
template <int N> using FusedTiling = std::conditional_t<fused_sched8_only<N>(), Sched8<N>, Sched<N>>;

// Column sets of the fused pass; with pair (parity layout) only the columns
// of rows q < N/2, each standing for rows q and q + N/2.
template <int N>
static void fused_sets(ColSet &s0, ColSet &s1, bool pair = false) {
    constexpr int CPW = FusedShape<N, FusedTiling<N>>::CPW;
    const int64_t H = N / 2;
    const int64_t rows = pair ? H : N;
    // main: columns (q, p) flat q*H + p; element (row r) at r*N*H + col
    s0.n_cols = rows * H; s0.W = (int64_t)N * H; s0.plane_stride = 0; s0.col_stride = 1;
    s0.row_stride = (int64_t)N * H; s0.off = 0; s0.rowfast = 0;
    // nyq: columns q; element (row r) at main + r*N + q
    s1.n_cols = rows; s1.W = N; s1.plane_stride = 0; s1.col_stride = 1; s1.row_stride = N;
    s1.off = spec_main(N); s1.rowfast = 0;
    s0.n_wgs = (int32_t)((s0.n_cols + CPW - 1) / CPW);
    s1.n_wgs = (int32_t)((s1.n_cols + CPW - 1) / CPW);
}

// variant 1: eight elements per thread (Sched8), where a schedule exists
template <int N> struct HasSched8 {
    static constexpr bool value = (N == 64 || N == 128 || N == 192 || N == 256 || N == 384 || N == 512);
};

template <int N, int NB, typename S, int PF, int IN>
static int fused_slots() {
    static int cached = 0;
    if (cached) return cached;
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fused_z_kernel<N, NB, S, PF, IN>, FusedShape<N, S>::NT,
                                                     0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    cached = per_cu * prop.multiProcessorCount;
    return cached;
}

// Three or four bands per launch (plain sums, prefetch depth 1): compiled
// at N = 384 and 512, where the slice spectra are the largest and reading
// them once for four bands instead of twice pays most.
template <int N, int PF, int IN> constexpr bool fused_nb4() { return (N == 384 || N == 512) && PF == 1 && IN != 1; }

template <int N, typename S, int PF, int IN>
static hipError_t fused_launch(const FusedArgs &fa, const void *tw, hipStream_t st, ColSet s0, ColSet s1,
                               int64_t tiles, int kmax) {
    static_assert(FusedShape<N, S>::CPW == FusedShape<N, FusedTiling<N>>::CPW, "variants share the tiling");
    constexpr bool PAR = IN == 1;
    int slots = 0;
    if (fa.nband > 2) {
        if constexpr (fused_nb4<N, PF, IN>()) slots = fused_slots<N, 4, S, PF, IN>();
        else return hipErrorInvalidValue;
    } else {
        slots = fa.nband == 2 ? fused_slots<N, 2, S, PF, IN>() : fused_slots<N, 1, S, PF, IN>();
    }
    // (two part slots per workgroup with two outputs per tile)
    const int64_t P = std::min<int64_t>(std::min<int64_t>(slots, tiles), fa.max_parts / (PAR ? 2 : 1));
    FusedDev d;
    d.spec = (const cx<float> *)fa.spec; d.spec_stride = fa.spec_stride;
    d.ghat = (const float *)fa.ghat; d.oct_stride = fa.oct_stride;
    d.B = fa.B; d.band0 = fa.band0; d.nb = fa.nband;
    for (int b = 0; b < 4; ++b) d.Kc[b] = b < fa.nband ? fa.kcount[b] : 0;
    d.acc = (cx<float> *)fa.acc; d.acc_stride = fa.acc_stride;
    d.part = (cx<float> *)fa.part; d.part_stride = fa.part_stride;
    d.zero_dc = fa.zero_dc; d.kahan = fa.kahan;
    d.kmax = kmax; d.P = (int32_t)P; d.W = tiles * kmax;
    d.rounds = fa.rounds; d.tiles = tiles;
    d.sk = fa.sk; d.g0 = fa.g0; d.inv_n3 = fa.inv_n3; d.mu = fa.mu; d.K = fa.K; d.ring = fa.ring; d.frozen = fa.frozen;
    // the split table serves the stream-K mode's merge in the inverse y pass;
    // the rounds mode splits no tile and its inverse pass does not read it
    if (!fa.rounds)
        hipLaunchKernelGGL(fused_split_kernel, dim3((unsigned)((tiles + 255) / 256)), dim3(256), 0, st,
                           (int *)fa.split_tab, tiles, (int64_t)kmax, P, d.W, PAR ? 1 : 0, (int64_t)s0.n_wgs);
    constexpr int NT = FusedShape<N, S>::NT;
    if (fa.nband > 2) {
        if constexpr (fused_nb4<N, PF, IN>())
            hipLaunchKernelGGL((fused_z_kernel<N, 4, S, PF, IN>), dim3((unsigned)P), dim3(NT), 0, st, d, s0, s1,
                               (const cx<float> *)tw);
    } else if (fa.nband == 2)
        hipLaunchKernelGGL((fused_z_kernel<N, 2, S, PF, IN>), dim3((unsigned)P), dim3(NT), 0, st, d, s0, s1,
                           (const cx<float> *)tw);
    else
        hipLaunchKernelGGL((fused_z_kernel<N, 1, S, PF, IN>), dim3((unsigned)P), dim3(NT), 0, st, d, s0, s1,
                           (const cx<float> *)tw);
    const int64_t full = tiles / P * P;
    if (fa.rounds && full < tiles) {
        // parts of the tiles split by slices after the whole rounds
        constexpr int CPW = FusedShape<N, S>::CPW;
        RestMerge m;
        m.acc = (cx<float> *)fa.acc; m.acc_stride = fa.acc_stride;
        m.part = (const cx<float> *)fa.part; m.part_stride = fa.part_stride;
        m.nband = fa.nband; m.no = PAR ? 2 : 1; m.cpw = CPW; m.L = N;
        m.full = full; m.rest = tiles - full; m.kmax = kmax; m.P = P;
        m.npb = (N / 2) % CPW == 0 ? (N / 2) / CPW : 0;
        m.gp = CPW >= 32 ? 1 : 32 / CPW;
        m.nrow = PAR ? N / 2 : N;
        const int64_t wgs = m.rest * m.no * m.nband * (((int64_t)N * CPW + 63) / 64);
        hipLaunchKernelGGL(fused_rest_merge_kernel, dim3((unsigned)wgs), dim3(256), 0, st, m, s0, s1);
    }
    return hipGetLastError();
}

// parity-layout input: compiled where a half-plane xy shape exists (the
// pair tiles need rows that split into whole tiles)
template <int N> constexpr bool fused_par() { return N == 192 || N == 256; }
static_assert((256 / 2) % FusedShape<256, FusedTiling<256>>::CPW == 0, "pair tiles cover whole rows");
static_assert((192 / 2) % FusedShape<192, FusedTiling<192>>::CPW == 0, "pair tiles cover whole rows");

template <int N, int IN>
static hipError_t fused_sched(const FusedArgs &fa, const void *tw, hipStream_t st, ColSet s0, ColSet s1,
                              int64_t tiles, int kmax) {
    // variant = 2 * schedule + (prefetch depth 1 ? 1 : 0); schedule 1 = Sched8
    // (N = 384, 512 compile only the Sched8 pair)
    // (three or four bands per launch: prefetch depth 1 only)
    const int sched = fused_sched8_only<N>() ? 1 : fa.variant / 2, pf = fa.variant % 2 || fa.nband > 2 ? 1 : 2;
    if constexpr (HasSched8<N>::value) {
        if (sched == 1)
            return pf == 1 ? fused_launch<N, Sched8<N>, 1, IN>(fa, tw, st, s0, s1, tiles, kmax)
                           : fused_launch<N, Sched8<N>, 2, IN>(fa, tw, st, s0, s1, tiles, kmax);
    }
    if constexpr (!fused_sched8_only<N>()) {
        return pf == 1 ? fused_launch<N, Sched<N>, 1, IN>(fa, tw, st, s0, s1, tiles, kmax)
                       : fused_launch<N, Sched<N>, 2, IN>(fa, tw, st, s0, s1, tiles, kmax);
    }
    return hipErrorInvalidValue;
}

template <int N>
static hipError_t fused_t(const FusedArgs &fa, const void *tw, hipStream_t st) {
    if (fa.parity && (fa.pre || !fused_par<N>())) return hipErrorInvalidValue;
    ColSet s0, s1;
    fused_sets<N>(s0, s1, fa.parity != 0);
    const int64_t tiles = s0.n_wgs + s1.n_wgs;
    const int64_t std_tiles = fa.parity ? 2 * tiles : tiles;
    int kmax = 0;
    for (int b = 0; b < fa.nband; ++b) kmax = std::max(kmax, fa.kcount[b]);
    if (kmax <= 0) {
        // no slice contributes: the accumulators are zero (and so are the
        // kernels' DC values, hence the means)
        if (fa.mu) {
            hipError_t e = launch_fill_f64(fa.mu + fa.band0, fa.nband, 0.0, st);
            if (e != hipSuccess) return e;
        }
        for (int b = 0; b < fa.nband; ++b) {
            hipError_t e = launch_fill_bytes((char *)fa.acc + (size_t)b * fa.acc_stride * 8,
                                             fa.acc_stride * 8, st);
            if (e != hipSuccess) return e;
        }
        if (!fa.rounds)   // no tile split: every entry -1
            hipLaunchKernelGGL(fused_split_kernel, dim3((unsigned)((std_tiles + 255) / 256)), dim3(256), 0, st,
                               (int *)fa.split_tab, std_tiles, (int64_t)1, (int64_t)1, std_tiles, 0, (int64_t)0);
        return hipGetLastError();
    }
    if constexpr (fused_par<N>()) {
        if (fa.parity) return fused_sched<N, 1>(fa, tw, st, s0, s1, tiles, kmax);
    }
    if (fa.pre) return fused_sched<N, 2>(fa, tw, st, s0, s1, tiles, kmax);
    return fused_sched<N, 0>(fa, tw, st, s0, s1, tiles, kmax);
}

// variants: bit 0 selects a prefetch depth of 1 (else 2) slices (fewer
// registers: the two-band instances need it), bit 1 the eight-element
// schedule where one exists (N = 384, 512: the eight-element schedule only,
// bit 0 alone)
int fused_variants(int n) {
    return (n == 384 || n == 512) ? 2 : (n == 64 || n == 128 || n == 192 || n == 256) ? 4 : 2;
}

bool fused_parity_supported(int n) { return n == 192 || n == 256; }

int fused_max_bands(int n) { return (n == 384 || n == 512) ? 4 : 2; }

// Built-in choice: prefetch depth 2 for one band per launch, 1 for two (the
// two-band instances of depth 2 spill registers).
int fused_default_variant(int n, int nband) {
    if (n == 384) return 1;   // depth 1 is the instance without spills there
    const int s8 = fused_variants(n) > 2 ? 2 : 0;
    return s8 + (nband > 1 ? 1 : 0);
}

hipError_t launch_fused_z(int n, const FusedArgs &a, const void *tw_full, hipStream_t st) {
    if (a.nband < 1 || a.nband > 4) return hipErrorInvalidValue;
    switch (n) {
#define X_(N) case N: return fused_t<N>(a, tw_full, st);
        X_(8) X_(12) X_(16) X_(24) X_(32) X_(48) X_(64) X_(96) X_(128) X_(192) X_(256) X_(384) X_(512)
#undef X_
        default: return hipErrorInvalidValue;
    }
}

int64_t fused_tiles(int n) {
    switch (n) {
#define X_(N) case N: { ColSet s0, s1; fused_sets<N>(s0, s1); return (int64_t)s0.n_wgs + s1.n_wgs; }
        X_(8) X_(12) X_(16) X_(24) X_(32) X_(48) X_(64) X_(96) X_(128) X_(192) X_(256) X_(384) X_(512)
#undef X_
        default: return 0;
    }
}

int fused_cpw(int n) {
    switch (n) {
#define X_(N) case N: return FusedShape<N, FusedTiling<N>>::CPW;
        X_(8) X_(12) X_(16) X_(24) X_(32) X_(48) X_(64) X_(96) X_(128) X_(192) X_(256) X_(384) X_(512)
#undef X_
        default: return 0;
    }
}

// ---------------------------------------------------------------------------
// FP64 mean (DC) of each band: mu_b = sum_k G^_{k,b}(0) S^_k(0) / N^3
// Stage 1: one workgroup per slice sums that slice's per-workgroup FP64
// partials of the forward x pass (fixed order: deterministic).
// Stage 2: one workgroup forms mu_b from the slice sums.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void dc_slice_kernel(const double *__restrict__ dcpart, int W,
                                                       double *__restrict__ sk, int *__restrict__ status,
                                                       int ring, int K) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int w = threadIdx.x; w < W; w += 256) s += dcpart[(int64_t)k * W + w];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sk[k] = red[0];
        // a NaN or infinite source value makes its slice's FP64 sum non-finite
        if (status && !isfinite(red[0])) {
            atomicAdd(&status[0], 1);
            atomicMin(&status[1], k >= ring ? k - ring : k - ring + K);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(64) void spec_dc_kernel(const cx<T> *__restrict__ spec, int64_t stride, int K,
                                                     double *__restrict__ sk, int *__restrict__ status,
                                                     int ring) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const double v = (double)spec[(int64_t)k * stride].x;
    sk[k] = v;
    if (!isfinite(v)) {
        atomicAdd(&status[0], 1);
        atomicMin(&status[1], k >= ring ? k - ring : k - ring + K);
    }
}

hipError_t launch_spec_dc(const void *spec, bool f64, int64_t stride, int K, double *sk, int *status, int ring,
                          hipStream_t st) {
    if (K < 1 || ring < 0 || ring >= K) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((K + 63) / 64));
    if (f64)
        hipLaunchKernelGGL(spec_dc_kernel<double>, grid, dim3(64), 0, st, (const cx<double> *)spec, stride, K, sk,
                           status, ring);
    else
        hipLaunchKernelGGL(spec_dc_kernel<float>, grid, dim3(64), 0, st, (const cx<float> *)spec, stride, K, sk,
                           status, ring);
    return hipGetLastError();
}

hipError_t launch_dc_reduce(const double *dcpart, int K, int W, double *sk, int *status, int ring,
                            hipStream_t st) {
    if (K < 1 || W < 1 || ring < 0 || ring >= K) return hipErrorInvalidValue;
    hipLaunchKernelGGL(dc_slice_kernel, dim3(K), dim3(256), 0, st, dcpart, W, sk, status, ring, K);
    return hipGetLastError();
}

}  // namespace lc
