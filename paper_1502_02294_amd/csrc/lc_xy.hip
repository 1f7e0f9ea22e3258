// Forward x and y passes of the 3D transform of Eq. 12 fused per z-plane,
// for the FP32 form at N in {64, 96, 128, 192, 256}.
//
// One workgroup owns one z-plane of one slice (N x N reals, at N = 256 a
// 256 KiB plane whose half spectrum is 264 KiB): it reads the plane once,
// keeps it in registers between the two transforms and writes the
// y-transformed half spectrum once. Against separate x and y passes this
// removes one full write and one full read of the spectrum per slice.
//
// The half-plane shapes (N = 256) give each workgroup the rows of one parity
// instead, so that two workgroups share a CU and one computes while the
// other waits for memory. Their y transforms have length N/2 and the slice
// spectrum is left in the parity layout (even-row and odd-row transforms in
// the lower and upper halves of every z-plane); the fused z pass applies the
// last radix-2 step of the y transform.
//
//   1. Every row is read (all row batches issued up front) as N/2 complex
//      values z[n] = x[2n] + i x[2n+1] and transformed by the N/2-point
//      register-in/register-out engine, RPB rows at a time.
//   2. The real-to-half-spectrum untangle runs in registers: the partner
//      Z[N/2 - q] of the element at position q is held by lane TX - t of the
//      same row at an element index fixed at compile time (see partner_e),
//      so one lane shuffle per element replaces an LDS round trip:
//        E = (Z[q] + conj Z[L-q]) / 2,  O = (Z[q] - conj Z[L-q]) / (2i),
//        Y[q] = E + W^q O,    W = exp(-2 pi i / N).
//   3. The p = 0 and p = N/2 columns are real for real input; they travel
//      through the y transform packed as one complex column
//      C = Y[.][0] + i Y[.][N/2], so the y pass has exactly N/2 columns, and
//      are separated afterwards:
//        Y^[k][0] = (C^[k] + conj C^[N-k]) / 2,
//        Y^[k][N/2] = (C^[k] - conj C^[N-k]) / (2i).
//   4. Column batch by column batch, the plane is transposed through LDS
//      (layout [row][column], one pad column) and each column of N values is
//      transformed by the N-point engine; lanes walk the columns, so every
//      store instruction writes 64 consecutive complex values of a row.
//
// The FP64 sum of the input plane (the DC mode of Eq. 12, kept in FP64 for
// the FP32 form) is written per plane to dcpart.
#include <algorithm>
#include <type_traits>

#include "lc_fft_device.h"
#include "lc_internal.h"

namespace lc {

// f(integral_constant<int, 0>), ..., f(integral_constant<int, C - 1>): the
// batch index stays a compile-time constant, so register arrays indexed by
// it are never demoted to scratch memory, however large the loop body.
template <int C, int I = 0, typename F> __device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < C) {
        f(std::integral_constant<int, I>{});
        static_for<C, I + 1>(f);
    }
}

// Launch shape: S8 selects the 8-elements-per-thread schedules (smaller
// register working set, one more LDS exchange per line), NB_ the number of
// row batches of the x phase (= column batches of the y phase), NC_ the
// number of column batches that the x phase deposits straight into LDS
// regions of their own (the rest of the plane waits in registers). NR_ is
// the number of rows a workgroup takes (= the y transform length): N for a
// whole plane, N/2 for the rows of one parity (y = 2m + s), whose y
// transform leaves the last radix-2 step of the length-N one to the reader.
template <int N, bool S8, int NB_, int NC_, int NR_ = N> struct XYShape {
    static constexpr int L = N / 2;
    static constexpr int NR = NR_;
    static constexpr int HALVES = N / NR;
    using SX = std::conditional_t<S8, Sched8<L>, Sched<L>>;
    using SY = std::conditional_t<S8, Sched8<NR>, Sched<NR>>;
    static constexpr int TX = SX::TPL, TY = SY::TPL;
    static constexpr int NB = NB_;
    static constexpr int RPB = NR / NB;           // rows per x batch
    static constexpr int CPB = L / NB;            // complex columns per y batch
    static constexpr int NT = TX * RPB;
    static constexpr int SK = 4;                  // x lines: one pad slot every 16 elements
    static constexpr int LSX = L + (L >> SK) + 1;
    static constexpr int ES = CPB + 1;            // y: LDS row stride of the transposed batch
    static constexpr int NC = NC_;
    static constexpr int LDS_X = RPB * LSX;
    static constexpr int RG = NR * ES;                    // one transposed column batch
    static constexpr int XS = LDS_X > RG ? LDS_X : RG;    // x scratch, then y batches >= NC
    static constexpr int LDS = XS + NC * RG;
    static_assert(NC >= 0 && NC <= NB, "column batches held in LDS");
    static_assert(HALVES == 1 || HALVES == 2, "whole planes or rows of one parity");
    static_assert((LDS + 2 * L + 2 * NR) * 8 + NT / 8 <= 160 * 1024, "LDS of one workgroup");
    static_assert(NT == TY * CPB, "x and y phases must use the same thread count");
    static_assert(NT % 64 == 0 && NT <= 1024, "whole waves, one workgroup");
    static_assert(CPB % TX == 0, "column batches must hold whole lane groups of a row");
};

// Value held by lane (TX - t) mod TX of the same TX-lane group (the lane
// of the untangle partner), moved with DPP instead of an LDS permute:
//   TX = 4: quad permutation [0, 3, 2, 1];
//   TX = 8 / 16: mirror within 8 / 16 lanes, then shift right by one lane.
// Lanes t = 0 use their own registers instead and ignore the result (their
// value crosses from the neighbouring group).
template <int TX> __device__ __forceinline__ float partner_val(float v) {
    const int iv = __float_as_int(v);
    if constexpr (TX == 2) {
        return v;   // lane 1 is its own partner
    } else if constexpr (TX == 4) {
        return __int_as_float(__builtin_amdgcn_mov_dpp(iv, 0 | (3 << 2) | (2 << 4) | (1 << 6), 0xF, 0xF, true));
    } else if constexpr (TX == 8) {
        const int m = __builtin_amdgcn_mov_dpp(iv, 0x141, 0xF, 0xF, true);    // row_half_mirror
        return __int_as_float(__builtin_amdgcn_mov_dpp(m, 0x111, 0xF, 0xF, true));  // row_shr:1
    } else {
        static_assert(TX == 16, "untangle lane groups of 2, 4, 8 or 16 lanes");
        const int m = __builtin_amdgcn_mov_dpp(iv, 0x140, 0xF, 0xF, true);    // row_mirror
        return __int_as_float(__builtin_amdgcn_mov_dpp(m, 0x111, 0xF, 0xF, true));  // row_shr:1
    }
}

// Element index, in the same thread or in lane TX - t, holding the partner
// position L - q of the element e of the last x pass. Output positions of the
// last pass are q = t + i*TX + r*M (e = i*RL + r, M = L/RL = BPT*TX).
template <int RL, int BPT>
__device__ __forceinline__ constexpr int partner_e(int e, bool t0) {
    const int i = e / RL, r = e % RL;
    if (!t0) return (BPT - 1 - i) * RL + (RL - 1 - r);
    if (i > 0) return (BPT - i) * RL + (RL - 1 - r);
    return (RL - r) % RL;
}

// Pin a value to the point where it is computed: an empty volatile asm
// statement that claims to modify the registers (no instruction is emitted).
// Without it the compiler sinks the untangle arithmetic and the FP64 input
// sum of every row batch down to their uses in the y phase, which keeps the
// inputs of all batches live together and spills them.
__device__ __forceinline__ void pin(cx<float> &v) { asm volatile("" : "+v"(v.x), "+v"(v.y)); }
__device__ __forceinline__ void pin(double &v) { asm volatile("" : "+v"(v)); }

template <int N, int NR_, typename TIN, bool S8, int NB_, int NC_, bool PER>
__global__ __launch_bounds__((XYShape<N, S8, NB_, NC_, NR_>::NT)) void xy_fwd_kernel(
    SrcTab srcs, cx<float> *__restrict__ spec0, int64_t spec_stride, const cx<float> *__restrict__ tw_half,
    const cx<float> *__restrict__ twist, const cx<float> *__restrict__ tw_full, double *__restrict__ dcpart,
    int64_t dc_stride, int n_planes) {
    using SH = XYShape<N, S8, NB_, NC_, NR_>;
    constexpr int L = SH::L, TX = SH::TX, NB = SH::NB, RPB = SH::RPB, CPB = SH::CPB, NT = SH::NT;
    constexpr int NR = SH::NR, HALVES = SH::HALVES;
    constexpr int SK = SH::SK, LSX = SH::LSX, ES = SH::ES, NC = SH::NC, XS = SH::XS, RG = SH::RG;
    constexpr bool F32IN = std::is_same<TIN, float>::value;
    static_assert(!PER || F32IN, "the persistent form reads FP32 grids");
    // Row batches in flight ahead of their transform. One workgroup per
    // plane: two batches (FP32 input) or one (FP64 input, whose loads are
    // twice as wide). Persistent workgroups: the first half of the next
    // plane is fetched during the last column batches of the current one's
    // y phase, the second half half a plane ahead during its x phase (more
    // would not fit in registers without spills, whose reloads would wait
    // for the loads in flight).
    constexpr int PF = PER ? (NB + 1) / 2 : (F32IN ? (NB < 2 ? NB : 2) : 1);
    using EX = Engine<float, L, true, typename SH::SX, SK>;
    using EY = Engine<float, NR, true, typename SH::SY>;
    constexpr int EXN = EX::E, EYN = EY::E;
    constexpr int RL = EX::RL, BPTL = EX::PLs::BPT, M = L / RL;
    static_assert(BPTL * TX == M, "last x pass layout");

    __shared__ cx<float> lds[SH::LDS];
    __shared__ cx<float> twx[L], twt[L], twy[NR];
    __shared__ cx<float> zb[NR];
    __shared__ double red[NT / 64];

    const int tid = threadIdx.x;
    const int xl = tid / TX, xt = tid % TX;
    const int yc = tid % CPB, yt = tid / CPB;
    const int lane = tid & 63;
    const bool t0 = xt == 0;
    const int stride = gridDim.x;   // persistent form: planes w, w + stride, ... of workgroup w

    // row batch b of plane `pl` (row xl of the batch) into dst[b]; with
    // `late`, the address passes through an empty asm statement so that the
    // loads stay after the preceding barrier instead of being hoisted to
    // where their registers are still taken
    auto load_batch = [&](auto bc, int pl, cx<float>(&dst)[NB][EXN], bool late) {
        constexpr int b = decltype(bc)::value;
        if constexpr (b < NB) {
            // (the offset, not the pointer, goes through the asm: the pointer
            // keeps its global address space, so these stay global loads,
            // which LDS waits do not wait for)
            const int pr = pl % (N * HALVES);   // (z, parity) of plane unit pl
            int64_t off = ((int64_t)(pr / HALVES) * N + HALVES * (b * RPB + xl) + pr % HALVES) * N;
            if (late) asm volatile("" : "+v"(off));
            const TIN *row = (const TIN *)srcs.p[pl / (N * HALVES)] + off;
#pragma unroll
            for (int e = 0; e < EXN; ++e) {
                const cx<TIN> v = *(const cx<TIN> *)(row + 2 * EX::in_pos(xt, e));
                dst[b][e] = mk((float)v.x, (float)v.y);
            }
        }
    };

    int plane = blockIdx.x;
    cx<float> xr[NB][EXN];
    static_for<PF>([&](auto bc) { load_batch(bc, plane, xr, false); });
    // untangle twist as V_q = -i W^q / 2:  Y[q] = (A + conj B) / 2 + V_q (A - conj B)
    for (int i = tid; i < L; i += NT) {
        twx[i] = tw_half[i];
        const cx<float> w = twist[i];
        twt[i] = mk(0.5f * w.y, -0.5f * w.x);
    }
    for (int i = tid; i < NR; i += NT) twy[i] = tw_full[HALVES * i];   // W_NR^i = W_N^(HALVES i)

    auto body = [&](int plane) {
        // plane unit: slice, z-plane and row parity (rows y = HALVES m + par);
        // its y-transformed rows go to rows par*NR .. par*NR + NR-1
        const int slice = plane / (N * HALVES), z = (plane % (N * HALVES)) / HALVES, par = plane % HALVES;
        cx<float> *__restrict__ mainp = spec0 + slice * spec_stride + ((int64_t)z * N + par * NR) * L;
        cx<float> *__restrict__ nyq = spec0 + slice * spec_stride + spec_main(N) + (int64_t)z * N + par * NR;
        const int next = plane + stride;
        const bool has_next = PER && next < n_planes;
        cx<float> xn[NB][EXN];   // the next plane's rows (persistent form)
        double dsum = 0.0;

        // ---- 2. x transforms and untangle, one row batch at a time
        static_for<NB>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            load_batch(std::integral_constant<int, b + PF>{}, plane, xr, true);
            if constexpr (F32IN) {
                // FP32 input converts exactly: sum it here, before the batch is
                // transformed, so the raw values need not stay live
#pragma unroll
                for (int e = 0; e < EXN; ++e) dsum += (double)xr[b][e].x + (double)xr[b][e].y;
                pin(dsum);
            }
            EX::run(xr[b], lds, xl * LSX, 1, xt, twx);
            cx<float> pv[EXN];
#pragma unroll
            for (int e = 0; e < EXN; ++e) {
                const cx<float> sv = xr[b][partner_e<RL, BPTL>(e, false)];
                const cx<float> o = mk(partner_val<TX>(sv.x), partner_val<TX>(sv.y));
                // (component-wise selects of values: a select between two
                // cx lvalues becomes a pointer select, which keeps the whole
                // row array in scratch memory where the partner index is
                // not a power of two)
                const cx<float> own = xr[b][partner_e<RL, BPTL>(e, true)];
                pv[e] = mk(t0 ? own.x : o.x, t0 ? own.y : o.y);
            }
#pragma unroll
            for (int e = 0; e < EXN; ++e) {
                const int q = EX::out_pos(xt, e);
                const cx<float> A = xr[b][e], B = pv[e];
                if (e == 0 && t0) {
                    // q = 0: Y[0] = Re A + Im A and Y[L] = Re A - Im A, both real: packed
                    xr[b][e] = mk(A.x + A.y, A.x - A.y);
                } else {
                    const cx<float> S = mk(A.x + B.x, A.y - B.y), D = mk(A.x - B.x, A.y + B.y);
                    const cx<float> V = twt[q];
                    xr[b][e] = mk(fmaf(0.5f, S.x, V.x * D.x - V.y * D.y), fmaf(0.5f, S.y, V.x * D.y + V.y * D.x));
                }
                pin(xr[b][e]);
            }
            if constexpr (NC > 0) {
                // elements of the first NC column batches go to their LDS regions now
                const int row = b * RPB + xl;
#pragma unroll
                for (int e = 0; e < EXN; ++e) {
                    const int i = e / RL, r = e % RL;
                    const int cb = (r * M + i * TX) / CPB;
                    if (cb < NC) lds[XS + cb * RG + row * ES + (EX::out_pos(xt, e) - cb * CPB)] = xr[b][e];
                }
            }
        });

        // ---- 3. y transforms, one column batch at a time
        static_for<NB>([&](auto cbc) {
            constexpr int cb = decltype(cbc)::value;
            // transposed batch: its own region (filled by the x phase) or the scratch
            cx<float> *reg = cb < NC ? lds + XS + cb * RG : lds;
            if constexpr (cb >= NC) {
                lds_barrier();   // earlier readers of the scratch are done
                static_for<NB>([&](auto bc) {
                    constexpr int b = decltype(bc)::value;
                    const int row = b * RPB + xl;
#pragma unroll
                    for (int e = 0; e < EXN; ++e) {
                        const int i = e / RL, r = e % RL;
                        if ((r * M + i * TX) / CPB == cb) {
                            const int q = EX::out_pos(xt, e);
                            reg[row * ES + (q - cb * CPB)] = xr[b][e];
                        }
                    }
                });
            }
            lds_barrier();
            if constexpr (PER) {
                // registers are freeing up: fetch a row batch of the next plane
                if constexpr (cb >= NB - PF) {
                    if (has_next) load_batch(std::integral_constant<int, cb - (NB - PF)>{}, next, xn, true);
                }
            }
            cx<float> y[EYN];
#pragma unroll
            for (int e = 0; e < EYN; ++e) y[e] = reg[EY::in_pos(yt, e) * ES + yc];
            EY::run(y, reg, yc, ES, yt, twy);
            const int p = cb * CPB + yc;
            if (p != 0) {
#pragma unroll
                for (int e = 0; e < EYN; ++e) mainp[(int64_t)EY::out_pos(yt, e) * L + p] = y[e];
            } else {
#pragma unroll
                for (int e = 0; e < EYN; ++e) zb[EY::out_pos(yt, e)] = y[e];
            }
        });

        // ---- 4. separate the packed p = 0 / p = N/2 column; FP64 plane sum
        if constexpr (!F32IN) {
            // FP64 input: the sum needs the values before rounding; read them again
            const TIN *in = (const TIN *)srcs.p[slice] + (int64_t)z * N * N;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const TIN *row = in + (int64_t)(HALVES * (b * RPB + xl) + par) * N;
                for (int e = 0; e < EXN; ++e) {
                    const cx<TIN> v = *(const cx<TIN> *)(row + 2 * EX::in_pos(xt, e));
                    dsum += (double)v.x + (double)v.y;
                }
            }
        }
        for (int o = 32; o > 0; o >>= 1) dsum += __shfl_down(dsum, o, 64);
        if (lane == 0) red[tid >> 6] = dsum;
        lds_barrier();
        for (int k = tid; k < NR; k += NT) {
            const cx<float> A = zb[k], B = zb[(NR - k) % NR];
            mainp[(int64_t)k * L] = mk((A.x + B.x) * 0.5f, (A.y - B.y) * 0.5f);
            nyq[k] = mk((A.y + B.y) * 0.5f, (B.x - A.x) * 0.5f);
        }
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < NT / 64; ++w) sum += red[w];
            dcpart[slice * dc_stride + z * HALVES + par] = sum;
        }
        if constexpr (PER) {
#pragma unroll
            for (int b = 0; b < PF; ++b)
#pragma unroll
                for (int e = 0; e < EXN; ++e) xr[b][e] = xn[b][e];
        }
    };
    if constexpr (PER) {
        for (; plane < n_planes; plane += stride) body(plane);
    } else {
        body(plane);
    }
}

// Inverse y and x passes and the epilogue of Eq. 12's inverse transform,
// fused per half z-plane, for an FP32 accumulator in the parity layout (the
// fused z pass with parity input leaves, in rows q and N/2 + q of every
// z-plane, U_0 = T[q] + T[q + N/2] and U_1 = W_N^-q (T[q] - T[q + N/2])).
// Output rows y = 2m + s of one z-plane are the N/2-point inverse y
// transform of U_s, so a workgroup takes (z, s), reads its half plane once
// and writes N/2 output rows once:
//   1. column batch by column batch (lanes walk the columns), the N/2-point
//      inverse y transform in registers; the p = 0 and p = N/2 columns, whose
//      inverse transforms are real, travel packed as U_s[.][0] + i U_s[.][N/2];
//   2. row batch by row batch, the rows are transposed through LDS and each
//      goes through the complex-to-real x transform (the retangle
//      Z[p] = E'_p + i O'_p of the half-length trick, then the N/2-point
//      inverse transform), scaled by 1/N^3, plus the FP64 mean, and stored.
// With COMBINE the second parts of tiles that the fused pass split between
// two workgroups (tab, part) are added while loading.
template <int N, typename TOUT, bool S8, int NB_, bool COMBINE>
__global__ __launch_bounds__((XYShape<N, S8, NB_, 0, N / 2>::NT)) void yx_inv_kernel(
    const cx<float> *__restrict__ acc, TOUT *__restrict__ out, const cx<float> *__restrict__ tw_half,
    const cx<float> *__restrict__ twist, const cx<float> *__restrict__ tw_full, double scale,
    const double *__restrict__ mu, const int *__restrict__ tab, const cx<float> *__restrict__ part, int cpw_z,
    int64_t tiles_main) {
    using SH = XYShape<N, S8, NB_, 0, N / 2>;
    constexpr int L = SH::L, NR = SH::NR, TX = SH::TX, TY = SH::TY, NB = SH::NB, RPB = SH::RPB, CPB = SH::CPB;
    constexpr int NT = SH::NT, SK = SH::SK, LSX = SH::LSX;
    using EY = Engine<float, NR, false, typename SH::SY>;
    using EX = Engine<float, L, false, typename SH::SX, SK>;
    constexpr int EYN = EY::E, EXN = EX::E;
    constexpr int RLY = EY::RL, BPTY = EY::PLs::BPT;
    static_assert(RPB % TY == 0, "a y output row's batch is fixed by its element index");
    constexpr int ESY = CPB + 1;                 // y exchange: [row][column of the batch]
    constexpr int LSR = L + 1;                   // transposed row batch: [row][p], p = 0 packed
    constexpr int YREG = NR * ESY, RREG = RPB * LSR, XREG = RPB * LSX;
    constexpr int LDSN = YREG > RREG + XREG ? YREG : RREG + XREG;
    static_assert((LDSN + 2 * L + NR) * 8 <= 80 * 1024, "two workgroups per CU");
    __shared__ cx<float> lds[LDSN];
    __shared__ cx<float> twx[L], twt[L], twy[NR];

    const int tid = threadIdx.x;
    const int yc = tid % CPB, yt = tid / CPB;
    const int xl = tid / TX, xt = tid % TX;
    const int z = blockIdx.x / 2, sp = blockIdx.x % 2;
    const cx<float> *__restrict__ mainp = acc + ((int64_t)z * N + sp * NR) * L;
    const cx<float> *__restrict__ nyq = acc + spec_main(N) + (int64_t)z * N + sp * NR;

    // every column batch of the half plane, loaded up front
    cx<float> yr[NB][EYN];
    auto part_at = [&](int64_t zt, int zc) -> cx<float> {
        const int w = tab[zt];
        return w >= 0 ? part[((int64_t)w * N + z) * cpw_z + zc] : mk(0.f, 0.f);
    };
    static_for<NB>([&](auto cbc) {
        constexpr int cb = decltype(cbc)::value;
        const int p = cb * CPB + yc;
#pragma unroll
        for (int e = 0; e < EYN; ++e) {
            const int r = EY::in_pos(yt, e);
            if (p != 0) {
                cx<float> v = mainp[(int64_t)r * L + p];
                if constexpr (COMBINE) {
                    const int64_t cc = (int64_t)(sp * NR + r) * L + p;
                    v = v + part_at(cc / cpw_z, (int)(cc % cpw_z));
                }
                yr[cb][e] = v;
            } else {
                cx<float> a = mainp[(int64_t)r * L], b = nyq[r];
                if constexpr (COMBINE) {
                    const int64_t cc = (int64_t)(sp * NR + r) * L;
                    a = a + part_at(cc / cpw_z, (int)(cc % cpw_z));
                    const int q = sp * NR + r;
                    b = b + part_at(tiles_main + q / cpw_z, q % cpw_z);
                }
                yr[cb][e] = mk(a.x - b.y, a.y + b.x);   // a + i b
            }
        }
    });
    for (int i = tid; i < L; i += NT) {
        twx[i] = tw_half[i];
        twt[i] = twist[i];
    }
    for (int i = tid; i < NR; i += NT) twy[i] = tw_full[2 * i];   // W_NR^i = W_N^(2i)
    lds_barrier();

    // ---- 1. inverse y transforms, one column batch at a time (in place)
    static_for<NB>([&](auto cbc) {
        constexpr int cb = decltype(cbc)::value;
        EY::run(yr[cb], lds, yc, ESY, yt, twy);
    });

    // ---- 2. per row batch: transpose, C2R x transform, epilogue
    const double m = *mu;
    cx<float> *rreg = lds, *xreg = lds + RREG;
    static_for<NB>([&](auto rbc) {
        constexpr int rb = decltype(rbc)::value;
        lds_barrier();   // earlier readers of the row and exchange regions are done
        static_for<NB>([&](auto cbc) {
            constexpr int cb = decltype(cbc)::value;
#pragma unroll
            for (int e = 0; e < EYN; ++e) {
                // output row of element e: yt + TY (i + r BPT), i = e / RL, r = e % RL
                const int j = e / RLY + (e % RLY) * BPTY;
                if ((TY * j) / RPB == rb) rreg[(EY::out_pos(yt, e) - rb * RPB) * LSR + cb * CPB + yc] = yr[cb][e];
            }
        });
        lds_barrier();
        const cx<float> *row = rreg + xl * LSR;
        cx<float> zx[EXN];
#pragma unroll
        for (int e = 0; e < EXN; ++e) {
            const int q = EX::in_pos(xt, e);
            if (q == 0) {
                const cx<float> pk = row[0];   // (Y[y][0], Y[y][N/2]), both real
                zx[e] = mk(pk.x + pk.y, pk.x - pk.y);
            } else {
                // Z[q] = E'_q + i O'_q,  E'_q = X[q] + conj X[L-q],  O'_q = (X[q] - conj X[L-q]) conj(W^q)
                const cx<float> Xp = row[q], Xm = row[L - q];
                const cx<float> Ep = mk(Xp.x + Xm.x, Xp.y - Xm.y);
                const cx<float> Dp = mk(Xp.x - Xm.x, Xp.y + Xm.y);
                const cx<float> w = twt[q];
                const cx<float> Op = mk(Dp.x * w.x + Dp.y * w.y, Dp.y * w.x - Dp.x * w.y);
                zx[e] = mk(Ep.x - Op.y, Ep.y + Op.x);
            }
        }
        EX::run(zx, xreg, xl * LSX, 1, xt, twx);
        const int y = 2 * (rb * RPB + xl) + sp;
        TOUT *orow = out + ((int64_t)z * N + y) * N;
#pragma unroll
        for (int e = 0; e < EXN; ++e) {
            cx<TOUT> o;
            o.x = (TOUT)((double)zx[e].x * scale + m);
            o.y = (TOUT)((double)zx[e].y * scale + m);
            *(cx<TOUT> *)(orow + 2 * EX::out_pos(xt, e)) = o;
        }
    });
}

bool yx_inv_supported(int n) { return n == 192 || n == 256; }

template <int N>
static hipError_t yx_inv_t(const void *acc, void *out, bool out_f64, const void *tw_half, const void *twist,
                           const void *tw_full, double scale, const double *mu, const int *split_tab,
                           const void *part, hipStream_t st) {
    constexpr bool S8 = false;
    constexpr int NB = 4;
    using SH = XYShape<N, S8, NB, 0, N / 2>;
    const int cpw = fused_cpw(N);
    const int64_t tiles_main = (int64_t)N * (N / 2) / cpw;
    const dim3 grid(2 * N);
#define YI_(TOUT, COMB)                                                                                       \
    hipLaunchKernelGGL((yx_inv_kernel<N, TOUT, S8, NB, COMB>), grid, dim3(SH::NT), 0, st, (const cx<float> *)acc, \
                       (TOUT *)out, (const cx<float> *)tw_half, (const cx<float> *)twist,                       \
                       (const cx<float> *)tw_full, scale, mu, split_tab, (const cx<float> *)part, cpw, tiles_main)
    if (part) {
        if (out_f64) YI_(double, true); else YI_(float, true);
    } else {
        if (out_f64) YI_(double, false); else YI_(float, false);
    }
#undef YI_
    return hipGetLastError();
}

hipError_t launch_yx_inv(int n, const void *acc, void *out, bool out_f64, const void *tw_half, const void *twist,
                         const void *tw_full, double scale, const double *mu, const int *split_tab,
                         const void *part, hipStream_t st) {
    if (!mu) return hipErrorInvalidValue;
    if (n == 256) return yx_inv_t<256>(acc, out, out_f64, tw_half, twist, tw_full, scale, mu, split_tab, part, st);
    if (n == 192) return yx_inv_t<192>(acc, out, out_f64, tw_half, twist, tw_full, scale, mu, split_tab, part, st);
    return hipErrorInvalidValue;
}

// Forward x pass alone, FP32 spectrum, for N = 512 (a z-plane is too large
// for one workgroup, so the y pass stays separate): the x phase of the fused
// xy pass over RB batches of RPB rows per workgroup, two batches in flight
// (one for FP64 input), the untangle done with lane moves, and each row's
// half spectrum stored straight from registers (p = 0 and p = N/2 from the
// packed element). With DC the FP64 sum of the workgroup's input goes to
// dcpart + slice * wgs + workgroup.
template <int N> struct XRowShape {
    static constexpr int L = N / 2;
    using SX = Sched<L>;
    static constexpr int TX = SX::TPL;
    static constexpr int NT = 256;
    static constexpr int RPB = NT / TX;         // rows per batch
    static constexpr int RB = 4;                // batches per workgroup
    static constexpr int ROWS = RB * RPB;
    static constexpr int SK = 4;
    static constexpr int LSX = L + (L >> SK) + 1;
};

template <int N, typename TIN, bool DC>
__global__ __launch_bounds__(XRowShape<N>::NT) void x_rows_kernel(SrcTab srcs, cx<float> *__restrict__ spec0,
                                                                  int64_t spec_stride, int wgs,
                                                                  const cx<float> *__restrict__ tw_half,
                                                                  const cx<float> *__restrict__ twist,
                                                                  double *__restrict__ dcpart0) {
    using SH = XRowShape<N>;
    constexpr int L = SH::L, TX = SH::TX, NT = SH::NT, RPB = SH::RPB, RB = SH::RB, SK = SH::SK, LSX = SH::LSX;
    using EX = Engine<float, L, true, typename SH::SX, SK>;
    constexpr int EXN = EX::E, RL = EX::RL, BPTL = EX::PLs::BPT, M = L / RL;
    static_assert(BPTL * TX == M, "last x pass layout");
    constexpr bool F32IN = std::is_same<TIN, float>::value;
    constexpr int PF = F32IN ? 2 : 1;
    __shared__ cx<float> lds[RPB * LSX];
    __shared__ cx<float> twx[L], twt[L];
    __shared__ double red[NT / 64];

    const int tid = threadIdx.x;
    const int xl = tid / TX, xt = tid % TX;
    const bool t0 = xt == 0;
    const int slice = blockIdx.x / wgs, blk = blockIdx.x % wgs;
    const TIN *__restrict__ in = (const TIN *)srcs.p[slice];
    cx<float> *__restrict__ mainp = spec0 + slice * spec_stride;
    cx<float> *__restrict__ nyq = mainp + spec_main(N);
    const int64_t row0 = (int64_t)blk * SH::ROWS;

    cx<float> xr[RB][EXN];
    auto load_batch = [&](auto bc, bool late) {
        constexpr int b = decltype(bc)::value;
        if constexpr (b < RB) {
            int64_t off = (row0 + b * RPB + xl) * N;
            if (late) asm volatile("" : "+v"(off));   // keep the loads after the preceding barrier
            const TIN *row = in + off;
#pragma unroll
            for (int e = 0; e < EXN; ++e) {
                const cx<TIN> v = *(const cx<TIN> *)(row + 2 * EX::in_pos(xt, e));
                xr[b][e] = mk((float)v.x, (float)v.y);
            }
        }
    };
    static_for<PF>([&](auto bc) { load_batch(bc, false); });
    for (int i = tid; i < L; i += NT) {
        twx[i] = tw_half[i];
        const cx<float> w = twist[i];
        twt[i] = mk(0.5f * w.y, -0.5f * w.x);   // V_q = -i W^q / 2
    }
    double dsum = 0.0;
    static_for<RB>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        load_batch(std::integral_constant<int, b + PF>{}, true);
        if constexpr (DC) {
            if constexpr (F32IN) {
#pragma unroll
                for (int e = 0; e < EXN; ++e) dsum += (double)xr[b][e].x + (double)xr[b][e].y;
            } else {
                // FP64 input: sum the values before rounding (read again)
                const TIN *row = in + (row0 + b * RPB + xl) * N;
#pragma unroll
                for (int e = 0; e < EXN; ++e) {
                    const cx<TIN> v = *(const cx<TIN> *)(row + 2 * EX::in_pos(xt, e));
                    dsum += (double)v.x + (double)v.y;
                }
            }
            pin(dsum);
        }
        EX::run(xr[b], lds, xl * LSX, 1, xt, twx);
        cx<float> pv[EXN];
#pragma unroll
        for (int e = 0; e < EXN; ++e) {
            const cx<float> sv = xr[b][partner_e<RL, BPTL>(e, false)];
            const cx<float> o = mk(partner_val<TX>(sv.x), partner_val<TX>(sv.y));
            const cx<float> own = xr[b][partner_e<RL, BPTL>(e, true)];
            pv[e] = mk(t0 ? own.x : o.x, t0 ? own.y : o.y);
        }
        const int64_t row = row0 + b * RPB + xl;
#pragma unroll
        for (int e = 0; e < EXN; ++e) {
            const int q = EX::out_pos(xt, e);
            const cx<float> A = xr[b][e], B = pv[e];
            if (e == 0 && t0) {
                // q = 0: X[0] = Re A + Im A and X[N/2] = Re A - Im A, both real
                mainp[row * L] = mk(A.x + A.y, 0.f);
                nyq[row] = mk(A.x - A.y, 0.f);
            } else {
                const cx<float> S = mk(A.x + B.x, A.y - B.y), D = mk(A.x - B.x, A.y + B.y);
                const cx<float> V = twt[q];
                mainp[row * L + q] = mk(fmaf(0.5f, S.x, V.x * D.x - V.y * D.y), fmaf(0.5f, S.y, V.x * D.y + V.y * D.x));
            }
        }
    });
    if constexpr (DC) {
        for (int o = 32; o > 0; o >>= 1) dsum += __shfl_down(dsum, o, 64);
        if ((tid & 63) == 0) red[tid >> 6] = dsum;
        lds_barrier();
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < NT / 64; ++w) sum += red[w];
            dcpart0[(int64_t)slice * wgs + blk] = sum;
        }
    }
}

bool x_rows_supported(int n) { return n == 512; }
int x_rows_wgs(int n) { return n == 512 ? (int)((int64_t)512 * 512 / XRowShape<512>::ROWS) : 0; }

hipError_t launch_x_rows_batch(int n, const SrcTab &in, int count, bool in_f64, void *spec, int64_t spec_stride,
                               const void *tw_half, const void *twist, double *dcpart, hipStream_t st) {
    if (n != 512 || count < 1 || count > SrcTab::kMax) return hipErrorInvalidValue;
    constexpr int N = 512;
    using SH = XRowShape<N>;
    const int wgs = x_rows_wgs(N);
    const dim3 grid((unsigned)(wgs * count));
#define XR_(TIN, DCF)                                                                                         \
    hipLaunchKernelGGL((x_rows_kernel<N, TIN, DCF>), grid, dim3(SH::NT), 0, st, in, (cx<float> *)spec, spec_stride, \
                       wgs, (const cx<float> *)tw_half, (const cx<float> *)twist, dcpart)
    if (in_f64) {
        if (dcpart) XR_(double, true); else XR_(double, false);
    } else {
        if (dcpart) XR_(float, true); else XR_(float, false);
    }
#undef XR_
    return hipGetLastError();
}

bool xy_supported(int n) { return n == 64 || n == 96 || n == 128 || n == 192 || n == 256; }

// Launch shapes compiled per N (schedule, batches); the plan picks one.
// At N = 256 shapes 4..6, at N = 192 shapes 2..3, take the rows of one
// parity per workgroup (half a plane: two or more workgroups fit on a CU)
// and leave the spectrum in the parity layout that the fused z pass
// completes.
int xy_variants(int n) { return n == 256 ? 7 : n == 192 ? 4 : n == 128 ? 2 : xy_supported(n) ? 1 : 0; }
static int xy_first_parity(int n) { return n == 256 ? 4 : n == 192 ? 2 : -1; }
bool xy_parity(int n, int variant) {
    const int f = xy_first_parity(n);
    return f >= 0 && variant >= f && variant < xy_variants(n);
}

template <int N, int NR, typename TIN, bool S8, int NB, int NC, bool PER>
static hipError_t xy_t(const SrcTab &in, int count, void *spec, int64_t spec_stride, const void *tw_half,
                       const void *twist, const void *tw_full, double *dcpart, int64_t dc_stride,
                       hipStream_t st) {
    using SH = XYShape<N, S8, NB, NC, NR>;
    const int n_planes = N * (N / NR) * count;
    int grid = n_planes;
    if constexpr (PER) {
        // one resident workgroup per slot; each walks planes w, w + grid, ...
        static int slots = 0;
        if (!slots) {
            int dev = 0, per_cu = 0;
            hipDeviceProp_t prop;
            if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
                return hipErrorInvalidDevice;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, xy_fwd_kernel<N, NR, TIN, S8, NB, NC, PER>,
                                                             SH::NT, 0) != hipSuccess ||
                per_cu < 1)
                per_cu = 1;
            slots = per_cu * prop.multiProcessorCount;
        }
        grid = std::min(grid, slots);
    }
    hipLaunchKernelGGL((xy_fwd_kernel<N, NR, TIN, S8, NB, NC, PER>), dim3((unsigned)grid), dim3(SH::NT), 0, st, in,
                       (cx<float> *)spec, spec_stride, (const cx<float> *)tw_half, (const cx<float> *)twist,
                       (const cx<float> *)tw_full, dcpart, dc_stride, n_planes);
    return hipGetLastError();
}

hipError_t launch_xy_fwd_batch(int n, const SrcTab &in, int count, bool in_f64, void *spec, int64_t spec_stride,
                               const void *tw_half, const void *twist, const void *tw_full, double *dcpart,
                               int64_t dc_stride, int variant, hipStream_t st) {
    if (count < 1 || count > SrcTab::kMax || !dcpart) return hipErrorInvalidValue;
    if (variant < 0 || variant >= xy_variants(n)) return hipErrorInvalidValue;
    // FP64 input takes the first shape of the same spectrum layout (the
    // FP64-input instances of the other shapes spill)
    if (in_f64) variant = xy_parity(n, variant) ? xy_first_parity(n) : 0;
#define XS_(N, NR, S8, NB, NC, PER)                                                                            \
    return in_f64 ? xy_t<N, NR, double, S8, NB, NC, false>(in, count, spec, spec_stride, tw_half, twist,       \
                                                           tw_full, dcpart, dc_stride, st)                        \
                  : xy_t<N, NR, float, S8, NB, NC, PER>(in, count, spec, spec_stride, tw_half, twist, tw_full,    \
                                                        dcpart, dc_stride, st);
#define X_(N, S8, NB, NC, PER) XS_(N, N, S8, NB, NC, PER)
#define XH_(N, S8, NB, NC) XS_(N, N / 2, S8, NB, NC, false)
    switch (n) {
        case 64: X_(64, false, 1, 0, false)
        case 96: X_(96, false, 1, 0, false)
        case 128:
            if (variant == 0) { X_(128, false, 1, 0, false) }
            X_(128, true, 2, 0, false)
        case 192:
            if (variant == 0) { X_(192, false, 4, 3, false) }
            if (variant == 1) { X_(192, false, 4, 0, false) }
            if (variant == 2) { XH_(192, false, 4, 1) }
            XH_(192, false, 2, 1)
        case 256:
            if (variant == 0) { X_(256, true, 8, 3, false) }
            if (variant == 1) { X_(256, false, 4, 1, false) }
            if (variant == 2) { X_(256, true, 4, 1, false) }
            if (variant == 3) { X_(256, true, 8, 3, true) }
            if (variant == 4) { XH_(256, false, 4, 1) }
            if (variant == 5) { XH_(256, true, 8, 1) }
            XH_(256, false, 4, 0)
        default: return hipErrorInvalidValue;
    }
#undef XH_
#undef X_
#undef XS_
}

}  // namespace lc
