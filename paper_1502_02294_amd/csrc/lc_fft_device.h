// Device-side building blocks for the LDS-staged Stockham FFT passes on
// gfx950 (wave64). Shared by every pass kernel of the library.
//
// A transform of length L is done by TPL threads per line; each pass of
// radix R performs L/R butterflies. Inputs of butterfly b are read at
// b + r*(L/R); outputs are written at (b/Ns)*Ns*R + b%Ns + r*Ns, where Ns
// is the product of the radices of the earlier passes (mixed-radix
// Stockham autosort, natural order in and out). Twiddles come from a table
// W_L^j = exp(-2 pi i j/L) generated on the host in FP64; the inverse uses
// their conjugates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lc {

// Workgroup barrier ordering LDS accesses only. __syncthreads() is a
// workgroup-scope release/acquire on all memory, which on this chip family
// waits for every outstanding global load too (one counter tracks them),
// so prefetches issued before a barrier would be drained by it. The
// kernels here share data between threads through LDS only; global data a
// thread loads is consumed by that thread before its next barrier.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T> __device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ cx<T> conj(cx<T> a) { return mk(a.x, -a.y); }
template <typename T> __device__ __forceinline__ cx<T> scal(cx<T> a, T s) { return mk(a.x * s, a.y * s); }

// multiply by the quarter-turn of the transform direction: -i forward, +i inverse
template <bool FWD, typename T> __device__ __forceinline__ cx<T> qturn(cx<T> a) {
    return FWD ? mk(a.y, -a.x) : mk(-a.y, a.x);
}

// multiply by exp(-+ i pi/4): (1 -+ i)/sqrt2
template <bool FWD, typename T> __device__ __forceinline__ cx<T> eighth1(cx<T> a) {
    const T h = (T)0.70710678118654752440;
    return FWD ? mk(h * (a.x + a.y), h * (a.y - a.x)) : mk(h * (a.x - a.y), h * (a.x + a.y));
}
// multiply by exp(-+ 3 i pi/4): (-1 -+ i)/sqrt2
template <bool FWD, typename T> __device__ __forceinline__ cx<T> eighth3(cx<T> a) {
    const T h = (T)0.70710678118654752440;
    return FWD ? mk(h * (a.y - a.x), -h * (a.x + a.y)) : mk(-h * (a.x + a.y), h * (a.x - a.y));
}
// multiply by a constant unit complex (c, s) of the forward direction,
// conjugated for the inverse
template <bool FWD, typename T> __device__ __forceinline__ cx<T> rot(cx<T> a, T c, T s) {
    return FWD ? mk(a.x * c - a.y * s, a.x * s + a.y * c) : mk(a.x * c + a.y * s, a.y * c - a.x * s);
}

// ---- small DFTs, in place, natural order ------------------------------------

template <bool FWD, typename T> __device__ __forceinline__ void dft2(cx<T> *v) {
    cx<T> a = v[0];
    v[0] = a + v[1];
    v[1] = a - v[1];
}

template <bool FWD, typename T> __device__ __forceinline__ void dft3(cx<T> *v) {
    const T half = (T)0.5, s3 = (T)0.86602540378443864676;   // sin(2 pi/3)
    cx<T> t1 = v[1] + v[2], t2 = v[1] - v[2];
    cx<T> m = mk(v[0].x - half * t1.x, v[0].y - half * t1.y);
    // forward: -i*s3*t2 ; inverse: +i*s3*t2
    cx<T> j = FWD ? mk(s3 * t2.y, -s3 * t2.x) : mk(-s3 * t2.y, s3 * t2.x);
    v[0] = v[0] + t1;
    v[1] = m + j;
    v[2] = m - j;
}

template <bool FWD, typename T> __device__ __forceinline__ void dft4(cx<T> *v) {
    cx<T> s02 = v[0] + v[2], d02 = v[0] - v[2];
    cx<T> s13 = v[1] + v[3], d13 = qturn<FWD>(v[1] - v[3]);
    v[0] = s02 + s13;
    v[2] = s02 - s13;
    v[1] = d02 + d13;
    v[3] = d02 - d13;
}

// 8 = 2 (inner, stride 4) x 4 (outer): y[k + 2q] = DFT4_q( W8^{jk} (x_j +- x_{j+4}) )
template <bool FWD, typename T> __device__ __forceinline__ void dft8(cx<T> *v) {
    cx<T> a[4], b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        a[j] = v[j] + v[j + 4];
        b[j] = v[j] - v[j + 4];
    }
    b[1] = eighth1<FWD>(b[1]);
    b[2] = qturn<FWD>(b[2]);
    b[3] = eighth3<FWD>(b[3]);
    dft4<FWD>(a);
    dft4<FWD>(b);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[2 * q] = a[q];
        v[2 * q + 1] = b[q];
    }
}

// 16 = 4 (inner, stride 4) x 4 (outer): y[k + 4q] = DFT4_q( W16^{jk} DFT4_m(x_{j+4m})_k )
template <bool FWD, typename T> __device__ __forceinline__ void dft16(cx<T> *v) {
    const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;  // cos, sin(pi/8)
    cx<T> c[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        cx<T> t[4] = {v[j], v[j + 4], v[j + 8], v[j + 12]};
        dft4<FWD>(t);
#pragma unroll
        for (int k = 0; k < 4; ++k) c[j][k] = t[k];
    }
    // twiddles W16^{jk}, forward W16 = exp(-i pi/8)
    c[1][1] = rot<FWD>(c[1][1], c1, -s1);
    c[1][2] = eighth1<FWD>(c[1][2]);
    c[1][3] = rot<FWD>(c[1][3], s1, -c1);
    c[2][1] = eighth1<FWD>(c[2][1]);
    c[2][2] = qturn<FWD>(c[2][2]);
    c[2][3] = eighth3<FWD>(c[2][3]);
    c[3][1] = rot<FWD>(c[3][1], s1, -c1);
    c[3][2] = eighth3<FWD>(c[3][2]);
    c[3][3] = rot<FWD>(c[3][3], -c1, s1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        cx<T> t[4] = {c[0][k], c[1][k], c[2][k], c[3][k]};
        dft4<FWD>(t);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[k + 4 * q] = t[q];
    }
}

template <int R, bool FWD, typename T> __device__ __forceinline__ void dft(cx<T> *v) {
    if constexpr (R == 2) dft2<FWD>(v);
    else if constexpr (R == 3) dft3<FWD>(v);
    else if constexpr (R == 4) dft4<FWD>(v);
    else if constexpr (R == 8) dft8<FWD>(v);
    else if constexpr (R == 16) dft16<FWD>(v);
    else static_assert(R == 2, "unsupported radix");
}

// ---- radix schedules ----------------------------------------------------------
// Forward passes use r(0..NP-1); the inverse runs them reversed, so the last
// forward pass and the first inverse pass share the same element-to-thread
// placement (used by the fused slice-sum pass). TPL threads work on one line;
// the first and the last pass give every thread whole butterflies, so each
// thread holds E = L / TPL elements in registers before the first pass and
// after the last one (middle passes go through LDS).

template <int L> struct Sched;
#define LC_SCHED(L_, NP_, R0, R1, R2, R3, TPL_)                                           \
    template <> struct Sched<L_> {                                                        \
        static constexpr int NP = NP_;                                                    \
        static constexpr int TPL = TPL_;                                                  \
        static constexpr int r(int i) { return i == 0 ? R0 : i == 1 ? R1 : i == 2 ? R2 : R3; } \
    };
LC_SCHED(4, 1, 4, 0, 0, 0, 1)
LC_SCHED(6, 2, 3, 2, 0, 0, 1)
LC_SCHED(8, 1, 8, 0, 0, 0, 1)
LC_SCHED(12, 2, 4, 3, 0, 0, 1)
LC_SCHED(16, 1, 16, 0, 0, 0, 1)
LC_SCHED(24, 2, 8, 3, 0, 0, 1)
LC_SCHED(32, 2, 8, 4, 0, 0, 2)
LC_SCHED(48, 3, 4, 4, 3, 0, 4)
LC_SCHED(64, 2, 16, 4, 0, 0, 4)
LC_SCHED(96, 3, 4, 8, 3, 0, 8)
LC_SCHED(128, 2, 16, 8, 0, 0, 8)
LC_SCHED(192, 3, 4, 16, 3, 0, 16)
LC_SCHED(256, 2, 16, 16, 0, 0, 16)
LC_SCHED(384, 4, 4, 8, 4, 3, 32)
LC_SCHED(512, 3, 16, 8, 4, 0, 32)
#undef LC_SCHED

// Schedules with 8 elements per thread for the fused slice-sum pass, whose
// per-element accumulators make register space scarce.
template <int L> struct Sched8;
#define LC_SCHED8(L_, NP_, R0, R1, R2, R3, TPL_)                                          \
    template <> struct Sched8<L_> {                                                       \
        static constexpr int NP = NP_;                                                    \
        static constexpr int TPL = TPL_;                                                  \
        static constexpr int r(int i) { return i == 0 ? R0 : i == 1 ? R1 : i == 2 ? R2 : R3; } \
    };
LC_SCHED8(64, 2, 8, 8, 0, 0, 8)
LC_SCHED8(128, 3, 8, 2, 8, 0, 16)
LC_SCHED8(192, 3, 8, 3, 8, 0, 24)
LC_SCHED8(256, 3, 8, 4, 8, 0, 32)
LC_SCHED8(384, 4, 8, 3, 4, 4, 48)
LC_SCHED8(512, 3, 8, 8, 8, 0, 64)
#undef LC_SCHED8

template <int L, bool FWD, typename S = Sched<L>> __device__ __host__ constexpr int pass_radix(int p) {
    return FWD ? S::r(p) : S::r(S::NP - 1 - p);
}

template <int L, bool FWD, typename S = Sched<L>> __device__ __host__ constexpr int ns_before(int p) {
    int ns = 1;
    for (int i = 0; i < p; ++i) ns *= pass_radix<L, FWD, S>(i);
    return ns;
}

// ---- one Stockham pass ----------------------------------------------------------
// Line elements live in LDS at lds[lbase + i*es]; thread t in [0, TPL).

// LDS position of line element p with a skew of one pad slot every 2^SK
// elements (SK = 31: no skew). Line passes whose lines are contiguous in LDS
// use it to spread power-of-two strides over the banks.
template <int SK> __device__ __forceinline__ int lpos(int p) { return p + (p >> SK); }

template <typename T, int L, int R, int NS, int TPL, bool FWD, int SK = 31>
struct Pass {
    static constexpr int NB = L / R;
    static constexpr int BPT = (NB + TPL - 1) / TPL;
    static constexpr bool EVEN = (NB % TPL) == 0;

    __device__ __forceinline__ static void twiddle(cx<T> *v, int b, const cx<T> *tw) {
        if constexpr (NS > 1) {
            const int base = (b % NS) * (L / (NS * R));
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cx<T> w = tw[base * r];
                if (!FWD) w.y = -w.y;
                v[r] = cmul(v[r], w);
            }
        }
    }
    // read, twiddle and transform this thread's butterflies into v
    __device__ __forceinline__ static void read(const cx<T> *lds, int lbase, int es, int t,
                                                const cx<T> *tw, cx<T> (&v)[BPT][R]) {
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            const int b = t + i * TPL;
            if (EVEN || b < NB) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = lds[lbase + lpos<SK>(b + r * NB) * es];
                twiddle(v[i], b, tw);
                dft<R, FWD>(v[i]);
            }
        }
    }
    __device__ __forceinline__ static void write(cx<T> *lds, int lbase, int es, int t,
                                                 const cx<T> (&v)[BPT][R]) {
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            const int b = t + i * TPL;
            if (EVEN || b < NB) {
                const int o = (b / NS) * NS * R + (b % NS);
#pragma unroll
                for (int r = 0; r < R; ++r) lds[lbase + lpos<SK>(o + r * NS) * es] = v[i][r];
            }
        }
    }
    // line position of input r of butterfly i of thread t
    __device__ __forceinline__ static int in_pos(int t, int i, int r) { return t + i * TPL + r * NB; }
    // line position of output r of butterfly i of thread t (after write)
    __device__ __forceinline__ static int out_pos(int t, int i, int r) {
        const int b = t + i * TPL;
        return (b / NS) * NS * R + (b % NS) + r * NS;
    }
};

// Run passes [P, PEND) of the schedule from LDS to LDS (barrier after each).
// Every thread of the workgroup must call this.
template <typename T, int L, bool FWD, int P, int PEND, typename S = Sched<L>, int SK = 31>
__device__ __forceinline__ void run_passes(cx<T> *lds, int lbase, int es, int t, bool active,
                                           const cx<T> *tw) {
    if constexpr (P < PEND) {
        constexpr int R = pass_radix<L, FWD, S>(P);
        constexpr int NS = ns_before<L, FWD, S>(P);
        using PS = Pass<T, L, R, NS, S::TPL, FWD, SK>;
        cx<T> v[PS::BPT][R];
        if (active) PS::read(lds, lbase, es, t, tw, v);
        lds_barrier();
        if (active) PS::write(lds, lbase, es, t, v);
        lds_barrier();
        run_passes<T, L, FWD, P + 1, PEND, S, SK>(lds, lbase, es, t, active, tw);
    }
}

// Passes P .. PEND-1 with the exchanges alternating between two LDS line
// buffers: exchange e (pass e + 1 reads, e = 0 written by the first pass)
// uses buffer e % 2. A buffer written here was last read two exchanges
// earlier, before the barrier that followed the exchange in between, so only
// the barrier after each write (readers wait for writers) remains.
template <typename T, int L, bool FWD, int P, int PEND, typename S, int SK>
__device__ __forceinline__ void run_passes_db(cx<T> *la, cx<T> *lb, int lbase, int es, int t, const cx<T> *tw) {
    if constexpr (P < PEND) {
        constexpr int R = pass_radix<L, FWD, S>(P);
        constexpr int NS = ns_before<L, FWD, S>(P);
        using PS = Pass<T, L, R, NS, S::TPL, FWD, SK>;
        cx<T> v[PS::BPT][R];
        PS::read(((P - 1) & 1) ? lb : la, lbase, es, t, tw, v);
        PS::write((P & 1) ? lb : la, lbase, es, t, v);
        lds_barrier();
        run_passes_db<T, L, FWD, P + 1, PEND, S, SK>(la, lb, lbase, es, t, tw);
    }
}

// The same passes for two lines at once, line i alternating between its own
// buffers la_i and lb_i; one barrier after both lines' writes serves both.
template <typename T, int L, bool FWD, int P, int PEND, typename S, int SK>
__device__ __forceinline__ void run_passes2_db(cx<T> *la0, cx<T> *lb0, cx<T> *la1, cx<T> *lb1, int lbase, int es,
                                               int t, const cx<T> *tw) {
    if constexpr (P < PEND) {
        constexpr int R = pass_radix<L, FWD, S>(P);
        constexpr int NS = ns_before<L, FWD, S>(P);
        using PS = Pass<T, L, R, NS, S::TPL, FWD, SK>;
        {
            cx<T> v[PS::BPT][R];
            PS::read(((P - 1) & 1) ? lb0 : la0, lbase, es, t, tw, v);
            PS::write((P & 1) ? lb0 : la0, lbase, es, t, v);
        }
        {
            cx<T> v[PS::BPT][R];
            PS::read(((P - 1) & 1) ? lb1 : la1, lbase, es, t, tw, v);
            PS::write((P & 1) ? lb1 : la1, lbase, es, t, v);
        }
        lds_barrier();
        run_passes2_db<T, L, FWD, P + 1, PEND, S, SK>(la0, lb0, la1, lb1, lbase, es, t, tw);
    }
}

// Register-in / register-out transform of one line by TPL threads.
// x[e] (e < E) holds, on entry, the first pass's inputs at line positions
// in_pos(t, e) and, on return, the last pass's outputs at out_pos(t, e).
template <typename T, int L, bool FWD, typename S = Sched<L>, int SK = 31>
struct Engine {
    static constexpr int NP = S::NP;
    static constexpr int TPL = S::TPL;
    static constexpr int E = L / TPL;
    static constexpr int R0 = pass_radix<L, FWD, S>(0);
    static constexpr int RL = pass_radix<L, FWD, S>(NP - 1);
    static constexpr int NSL = ns_before<L, FWD, S>(NP - 1);
    using P0 = Pass<T, L, R0, 1, TPL, FWD, SK>;
    using PLs = Pass<T, L, RL, NSL, TPL, FWD, SK>;
    static_assert(P0::EVEN && PLs::EVEN, "first and last passes must give every thread whole butterflies");
    static_assert(P0::BPT * R0 == E && PLs::BPT * RL == E, "element count per thread");

    __device__ __forceinline__ static int in_pos(int t, int e) { return P0::in_pos(t, e / R0, e % R0); }
    __device__ __forceinline__ static int out_pos(int t, int e) { return PLs::out_pos(t, e / RL, e % RL); }

    // first pass in registers; with more than one pass its outputs go to LDS
    // (after a barrier protecting earlier readers of the LDS line buffer)
    __device__ __forceinline__ static void first(cx<T> (&x)[E], cx<T> *lds, int lbase, int es, int t) {
#pragma unroll
        for (int i = 0; i < P0::BPT; ++i) dft<R0, FWD>(x + i * R0);
        if constexpr (NP > 1) {
            lds_barrier();
#pragma unroll
            for (int i = 0; i < P0::BPT; ++i) {
                const int o = (t + i * TPL) * R0;
#pragma unroll
                for (int r = 0; r < R0; ++r) lds[lbase + lpos<SK>(o + r) * es] = x[i * R0 + r];
            }
        }
    }
    // remaining passes; outputs in y (with NP == 1, y = x already transformed)
    __device__ __forceinline__ static void rest(const cx<T> (&x)[E], cx<T> (&y)[E], cx<T> *lds, int lbase,
                                                int es, int t, const cx<T> *tw) {
        if constexpr (NP == 1) {
#pragma unroll
            for (int e = 0; e < E; ++e) y[e] = x[e];
        } else {
            lds_barrier();
            run_passes<T, L, FWD, 1, NP - 1, S, SK>(lds, lbase, es, t, true, tw);
#pragma unroll
            for (int i = 0; i < PLs::BPT; ++i) {
                const int b = t + i * TPL;
#pragma unroll
                for (int r = 0; r < RL; ++r) y[i * RL + r] = lds[lbase + lpos<SK>(b + r * PLs::NB) * es];
                PLs::twiddle(y + i * RL, b, tw);
                dft<RL, FWD>(y + i * RL);
            }
        }
    }
    __device__ __forceinline__ static void run(cx<T> (&x)[E], cx<T> *lds, int lbase, int es, int t,
                                               const cx<T> *tw) {
        first(x, lds, lbase, es, t);
        cx<T> y[E];
        rest(x, y, lds, lbase, es, t, tw);
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = y[e];
    }

    // The same transform with its exchanges alternating between the line
    // buffers la and lb (run_passes_db). For a sequence of such transforms
    // by the same threads (any mix of directions with this pass count) the
    // barrier that protects earlier readers is needed only at the start of a
    // transform whose predecessor's last exchange used la, i.e. when the
    // number of exchanges NP - 1 is odd; the caller keeps other LDS users
    // apart as before.
    __device__ __forceinline__ static void first_db(cx<T> (&x)[E], cx<T> *la, int lbase, int es, int t) {
#pragma unroll
        for (int i = 0; i < P0::BPT; ++i) dft<R0, FWD>(x + i * R0);
        if constexpr (NP > 1) {
            if constexpr ((NP - 1) % 2 == 1) lds_barrier();
#pragma unroll
            for (int i = 0; i < P0::BPT; ++i) {
                const int o = (t + i * TPL) * R0;
#pragma unroll
                for (int r = 0; r < R0; ++r) la[lbase + lpos<SK>(o + r) * es] = x[i * R0 + r];
            }
        }
    }
    __device__ __forceinline__ static void rest_db(const cx<T> (&x)[E], cx<T> (&y)[E], cx<T> *la, cx<T> *lb,
                                                   int lbase, int es, int t, const cx<T> *tw) {
        if constexpr (NP == 1) {
#pragma unroll
            for (int e = 0; e < E; ++e) y[e] = x[e];
        } else {
            lds_barrier();
            run_passes_db<T, L, FWD, 1, NP - 1, S, SK>(la, lb, lbase, es, t, tw);
            const cx<T> *src = ((NP - 2) & 1) ? lb : la;
#pragma unroll
            for (int i = 0; i < PLs::BPT; ++i) {
                const int b = t + i * TPL;
#pragma unroll
                for (int r = 0; r < RL; ++r) y[i * RL + r] = src[lbase + lpos<SK>(b + r * PLs::NB) * es];
                PLs::twiddle(y + i * RL, b, tw);
                dft<RL, FWD>(y + i * RL);
            }
        }
    }
    __device__ __forceinline__ static void run_db(cx<T> (&x)[E], cx<T> *la, cx<T> *lb, int lbase, int es,
                                                  int t, const cx<T> *tw) {
        first_db(x, la, lbase, es, t);
        cx<T> y[E];
        rest_db(x, y, la, lb, lbase, es, t, tw);
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = y[e];
    }

    // Two lines through the transform with their exchanges interleaved: line
    // i alternates between its own buffers la_i and lb_i, and each barrier
    // serves both lines (half the barriers of two run_db calls). first2_db
    // takes the first-pass inputs (x0, x1 are free on return); rest2_db calls
    // mid() right after its first barrier, when every thread has finished
    // the previous rest2_db, and then out(i, y) with the outputs of line i
    // (line 0 first, so that only one line's outputs are live at a time).
    // A sequence of these calls by the same threads needs no other barrier.
    __device__ __forceinline__ static void first2_db(cx<T> (&x0)[E], cx<T> (&x1)[E], cx<T> *la0, cx<T> *la1,
                                                     int lbase, int es, int t) {
        static_assert(NP > 1, "the interleaved form exchanges through LDS");
#pragma unroll
        for (int i = 0; i < P0::BPT; ++i) dft<R0, FWD>(x0 + i * R0);
#pragma unroll
        for (int i = 0; i < P0::BPT; ++i) dft<R0, FWD>(x1 + i * R0);
        if constexpr ((NP - 1) % 2 == 1) lds_barrier();
#pragma unroll
        for (int i = 0; i < P0::BPT; ++i) {
            const int o = (t + i * TPL) * R0;
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                la0[lbase + lpos<SK>(o + r) * es] = x0[i * R0 + r];
                la1[lbase + lpos<SK>(o + r) * es] = x1[i * R0 + r];
            }
        }
    }
    template <typename M, typename F>
    __device__ __forceinline__ static void rest2_db(cx<T> *la0, cx<T> *lb0, cx<T> *la1, cx<T> *lb1, int lbase,
                                                    int es, int t, const cx<T> *tw, M &&mid, F &&out) {
        lds_barrier();
        mid();
        run_passes2_db<T, L, FWD, 1, NP - 1, S, SK>(la0, lb0, la1, lb1, lbase, es, t, tw);
        constexpr bool B = ((NP - 2) & 1) != 0;
#pragma unroll
        for (int li = 0; li < 2; ++li) {
            const cx<T> *src = li == 0 ? (B ? lb0 : la0) : (B ? lb1 : la1);
            cx<T> y[E];
#pragma unroll
            for (int i = 0; i < PLs::BPT; ++i) {
                const int b = t + i * TPL;
#pragma unroll
                for (int r = 0; r < RL; ++r) y[i * RL + r] = src[lbase + lpos<SK>(b + r * PLs::NB) * es];
                PLs::twiddle(y + i * RL, b, tw);
                dft<RL, FWD>(y + i * RL);
            }
            out(li, y);
        }
    }
};

// Column sets: a batch of strided lines. Column c of the set has its element
// at row j at  off + (c / W) * plane_stride + (c % W) * col_stride + j * row_stride.
struct ColSet {
    int64_t n_cols;
    int64_t W;
    int64_t plane_stride;
    int64_t col_stride;
    int64_t row_stride;
    int64_t off;
    int32_t rowfast;   // 1: lanes walk along rows when loading (row_stride == 1)
    int32_t n_wgs;     // workgroups covering this set
};

__device__ __forceinline__ int64_t col_base(const ColSet &s, int64_t c) {
    return s.off + (c / s.W) * s.plane_stride + (c % s.W) * s.col_stride;
}

// Global <-> LDS tile moves for CPW columns starting at col0. LDS layout
// [row][CPW + PAD].
template <typename T, int L, int CPW, int NT, int PAD>
__device__ __forceinline__ void tile_load(cx<T> *lds, const cx<T> *__restrict__ g, const ColSet &s,
                                          int64_t col0) {
    constexpr int ES = CPW + PAD;
    if (!s.rowfast) {
        static_assert(NT % CPW == 0, "NT must be a multiple of CPW");
        const int c = threadIdx.x % CPW;
        const int64_t col = col0 + c;
        if (col < s.n_cols) {
            const int64_t base = col_base(s, col);
            for (int j = threadIdx.x / CPW; j < L; j += NT / CPW)
                lds[j * ES + c] = g[base + j * s.row_stride];
        }
    } else {
        for (int e = threadIdx.x; e < L * CPW; e += NT) {
            const int j = e % L, c = e / L;
            const int64_t col = col0 + c;
            if (col < s.n_cols) lds[j * ES + c] = g[col_base(s, col) + j * s.row_stride];
        }
    }
}

template <typename T, int L, int CPW, int NT, int PAD>
__device__ __forceinline__ void tile_store(cx<T> *__restrict__ g, const cx<T> *lds, const ColSet &s,
                                           int64_t col0) {
    constexpr int ES = CPW + PAD;
    if (!s.rowfast) {
        const int c = threadIdx.x % CPW;
        const int64_t col = col0 + c;
        if (col < s.n_cols) {
            const int64_t base = col_base(s, col);
            for (int j = threadIdx.x / CPW; j < L; j += NT / CPW)
                g[base + j * s.row_stride] = lds[j * ES + c];
        }
    } else {
        for (int e = threadIdx.x; e < L * CPW; e += NT) {
            const int j = e % L, c = e / L;
            const int64_t col = col0 + c;
            if (col < s.n_cols) g[col_base(s, col) + j * s.row_stride] = lds[j * ES + c];
        }
    }
}

// Launch shape of the column passes for a line length L and element type:
// CPW columns per workgroup (16 FP32 / 8 FP64 columns = 128-byte rows when
// the lines are strided), TPL threads per column. FP32 lines of 512 take 32
// columns (256-byte row segments, one 1024-thread workgroup per CU): the
// batched forward y pass of a 512^3 grid runs 8% faster than with 16.
template <typename T, int L> struct ColShape {
    static constexpr int TPL = Sched<L>::TPL;
    static constexpr int CPW0 = sizeof(T) == 4 ? (L == 512 ? 32 : 16) : 8;
    static constexpr int CPW = (CPW0 * TPL >= 64) ? CPW0 : 64 / TPL;   // at least one wave
    static constexpr int NT = CPW * TPL;
    static constexpr int PAD = 1;
};

// Launch shape of the fused slice-sum pass: schedule S, 16 columns per
// workgroup (128-byte rows).
template <int L, typename S> struct FusedShape {
    static constexpr int TPL = S::TPL;
    // 16 columns (a 128-byte row segment), at most 512 threads (so that a
    // thread keeps a 256-register budget; a power of two below that), at
    // least one wave. (8-column tiles at L = 256, two workgroups per CU,
    // measured slower: half-line reads cost more than the overlap gains.)
    static constexpr int CMAX = 512 / TPL < 16 ? 512 / TPL : 16;
    static constexpr int CPW = (16 * TPL >= 64)
                                   ? (CMAX >= 16 ? 16 : CMAX >= 8 ? 8 : CMAX >= 4 ? 4 : CMAX >= 2 ? 2 : 1)
                                   : 64 / TPL;
    static constexpr int NT = CPW * TPL;
    static constexpr int PAD = 1;
    // requested waves per SIMD: bounds the register budget (512 / WPE)
    static constexpr int WPE = (L / TPL <= 8) ? 4 : 2;
};

// Launch shape of the row (x) passes for half-length L = N/2.
template <typename T, int L> struct RowShape {
    static constexpr int TPL = Sched<L>::TPL;
    static constexpr int NT = 256;
    static constexpr int RPW = NT / TPL;
    static constexpr int SK = 4;                          // one pad slot every 16 elements
    static constexpr int LS = L + (L >> 4) + 1;           // line stride in LDS (odd)
};

}  // namespace lc
