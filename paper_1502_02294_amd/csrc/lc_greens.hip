// Periodic retarded-time shell kernel G_k (Eq. 10, algorithm step 2) and the
// folding of its FP64 spectrum (step 3), plus small utility kernels.
//
// Builder: one thread per cell of the non-negative octant c in [0, N/2]^3.
// For every periodic image u whose cell box can reach [r_k, r_{k+1}) it sums
// the m^3 subpoints with exact integer squared distance n (units of the
// half-subcell h = L/(2 m N)) inside [T_k, T_{k+1}), each weighing
// pref * phi(rho) / (4 pi rho^2) / m^3, rho = sqrt(n) h. G is even in every
// axis, so the octant value is written to all of its mirror cells.
#include <algorithm>

#include "lc_fft_device.h"
#include "lc_internal.h"

namespace lc {

__device__ __forceinline__ double phi_eval(int kind, double r, double a, double s, double p,
                                           double c, double cut) {
    if (kind == 0) return 1.0;
    const double v = a * exp(-pow(r / s, p)) - c;
    if (kind == 1) return v > 0.0 ? v : 0.0;
    return r <= cut ? v : 0.0;
}

__global__ __launch_bounds__(256) void greens_build_kernel(BuildArgs a) {
    const int n = a.n, H = n / 2 + 1;
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= (int64_t)H * H * H) return;
    const int ci = (int)(cell / ((int64_t)H * H)), cj = (int)((cell / H) % H), ck = (int)(cell % H);
    const int m = a.m, U = a.images;
    const double l = a.l;
    const double four_pi = 12.566370614359172954;
    const double wm = a.pref / ((double)m * m * m);
    const double margin = 1e-9 * (a.r_hi + l);
    double acc = 0.0;
    for (int u0 = -U; u0 <= U; ++u0) {
        const int64_t x0 = ci + (int64_t)u0 * n;
        const double lo0 = (x0 - 0.5) * l, hi0 = (x0 + 0.5) * l;
        const double nr0 = lo0 > 0 ? lo0 : (hi0 < 0 ? -hi0 : 0.0), fr0 = fmax(fabs(lo0), fabs(hi0));
        for (int u1 = -U; u1 <= U; ++u1) {
            const int64_t x1 = cj + (int64_t)u1 * n;
            const double lo1 = (x1 - 0.5) * l, hi1 = (x1 + 0.5) * l;
            const double nr1 = lo1 > 0 ? lo1 : (hi1 < 0 ? -hi1 : 0.0), fr1 = fmax(fabs(lo1), fabs(hi1));
            for (int u2 = -U; u2 <= U; ++u2) {
                const int64_t x2 = ck + (int64_t)u2 * n;
                const double lo2 = (x2 - 0.5) * l, hi2 = (x2 + 0.5) * l;
                const double nr2 = lo2 > 0 ? lo2 : (hi2 < 0 ? -hi2 : 0.0), fr2 = fmax(fabs(lo2), fabs(hi2));
                const double dmin = sqrt(nr0 * nr0 + nr1 * nr1 + nr2 * nr2);
                const double dmax = sqrt(fr0 * fr0 + fr1 * fr1 + fr2 * fr2);
                if (dmin > a.r_hi + margin || dmax < a.r_lo - margin) continue;
                if (a.self_pair && x0 == 0 && x1 == 0 && x2 == 0) {
                    acc += a.self_val;     // zero unless this is slice 0
                    continue;
                }
                for (int a0 = 0; a0 < m; ++a0) {
                    const int64_t q0 = 2 * m * x0 + (2 * a0 + 1 - m);
                    for (int a1 = 0; a1 < m; ++a1) {
                        const int64_t q1 = 2 * m * x1 + (2 * a1 + 1 - m);
                        const int64_t s01 = q0 * q0 + q1 * q1;
                        for (int a2 = 0; a2 < m; ++a2) {
                            const int64_t q2 = 2 * m * x2 + (2 * a2 + 1 - m);
                            const int64_t nn = s01 + q2 * q2;
                            const double dn = (double)nn;
                            if (dn >= a.t_lo && dn < a.t_hi) {
                                const double rho = sqrt(dn) * a.h;
                                acc += wm * phi_eval(a.kind, rho, a.a, a.s, a.p, a.c, a.cut) /
                                       (four_pi * rho * rho);
                            }
                        }
                    }
                }
            }
        }
    }
    // mirror into the full grid
    const int is[2] = {ci, (n - ci) % n}, js[2] = {cj, (n - cj) % n}, ks[2] = {ck, (n - ck) % n};
    for (int a0 = 0; a0 < 2; ++a0)
        for (int a1 = 0; a1 < 2; ++a1)
            for (int a2 = 0; a2 < 2; ++a2)
                a.grid[((int64_t)is[a0] * n + js[a1]) * n + ks[a2]] = acc;
}

hipError_t launch_greens_build(const BuildArgs &a, hipStream_t st) {
    const int64_t H = a.n / 2 + 1;
    const int64_t cells = H * H * H;
    hipLaunchKernelGGL(greens_build_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fold: FP64 spectrum -> real octant of the plan precision
// ---------------------------------------------------------------------------
template <typename TO>
__global__ __launch_bounds__(256) void greens_fold_kernel(const cx<double> *__restrict__ spec, TO *__restrict__ oct,
                                                          int n, int conserve, double target_over_l3,
                                                          double *__restrict__ dc,
                                                          unsigned long long *__restrict__ maxima) {
    const int H = n / 2, HP = H + 1;
    const int64_t total = (int64_t)HP * HP * HP;
    const int64_t main_n = (int64_t)n * n * H;
    const double g00 = spec[0].x;
    const double f = conserve ? target_over_l3 / g00 : 1.0;
    double mim = 0.0, mre = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / ((int64_t)HP * HP)), q = (int)((e / HP) % HP), p = (int)(e % HP);
        cx<double> v;
        int64_t o;
        if (p < H) {
            v = spec[((int64_t)r * n + q) * H + p];
            o = ((int64_t)r * HP + q) * H + p;
        } else {
            v = spec[main_n + (int64_t)r * n + q];
            o = (int64_t)HP * HP * H + (int64_t)r * HP + q;
        }
        oct[o] = (TO)(v.x * f);
        mim = fmax(mim, fabs(v.y));
        mre = fmax(mre, fabs(v.x));
        if (e == 0) *dc = v.x * f;
    }
    __shared__ double red[2][4];
    for (int o = 32; o > 0; o >>= 1) {
        mim = fmax(mim, __shfl_down(mim, o, 64));
        mre = fmax(mre, __shfl_down(mre, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = mim;
        red[1][threadIdx.x >> 6] = mre;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) {
            mim = fmax(mim, red[0][w]);
            mre = fmax(mre, red[1][w]);
        }
        // non-negative doubles order like their bit patterns
        atomicMax(&maxima[0], (unsigned long long)__double_as_longlong(mim));
        atomicMax(&maxima[1], (unsigned long long)__double_as_longlong(mre));
    }
}

hipError_t launch_greens_fold(int n, const void *spec64, void *oct, bool oct_f64, int conserve,
                              double target_over_l3, double *dc, unsigned long long *maxima,
                              hipStream_t st) {
    const int64_t HP = n / 2 + 1;
    const int64_t total = HP * HP * HP;
    const int wgs = (int)std::min<int64_t>((total + 255) / 256, 1024);
    if (oct_f64)
        hipLaunchKernelGGL(greens_fold_kernel<double>, dim3(wgs), dim3(256), 0, st,
                           (const cx<double> *)spec64, (double *)oct, n, conserve, target_over_l3, dc,
                           maxima);
    else
        hipLaunchKernelGGL(greens_fold_kernel<float>, dim3(wgs), dim3(256), 0, st,
                           (const cx<double> *)spec64, (float *)oct, n, conserve, target_over_l3, dc,
                           maxima);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// near-field (particle-mesh) correction
//
// A source with a position inside its cell (x_s, in length units) is
// deposited to its nearest node c_s = round(x_s / l) mod N. For target nodes
// x = c_s + o, 0 < |o|_inf <= R, its mesh contribution L G_k(o) has a
// primary-image part that the correction replaces by the retarded kernel at
// the exact distance: J(x) += L (F_k(|x l - x_s|) - G^prim_k(o)), with
// F_k(rho) = [r_k <= rho < r_{k+1}] pref phi(rho) / (4 pi rho^2) and
// G^prim_k(o) the m^3-subpoint average of the image u = 0 (the same rule as
// the builder). The source's own node keeps the mesh value. Distances are
// formed without fused multiply-adds so that shell membership is decided
// on the same rounded values as a plain FP64 evaluation.
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)
// index in [0, n) of node coordinate c (a whole number), wrapped periodically
__device__ __forceinline__ int64_t wrap_node(double c, int n) {
    double v = fmod(c, (double)n);
    if (v < 0.0) v += (double)n;
    if (v >= (double)n) v -= (double)n;
    return (int64_t)v;
}

__global__ __launch_bounds__(256) void near_table_kernel(NearArgs a) {
    const int R = a.R, W = R + 1;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)W * W * W) return;
    const int d0 = (int)(e / (W * W)), d1 = (int)((e / W) % W), d2 = (int)(e % W);
    const int m = a.m;
    const double four_pi = 12.566370614359172954;
    const double wm = a.pref / ((double)m * m * m);
    double acc = 0.0;
    if (d0 | d1 | d2) {
        for (int a0 = 0; a0 < m; ++a0) {
            const int64_t q0 = 2 * m * (int64_t)d0 + (2 * a0 + 1 - m);
            for (int a1 = 0; a1 < m; ++a1) {
                const int64_t q1 = 2 * m * (int64_t)d1 + (2 * a1 + 1 - m);
                for (int a2 = 0; a2 < m; ++a2) {
                    const int64_t q2 = 2 * m * (int64_t)d2 + (2 * a2 + 1 - m);
                    const double dn = (double)(q0 * q0 + q1 * q1 + q2 * q2);
                    if (dn >= a.t_lo && dn < a.t_hi) {
                        const double rho = sqrt(dn) * a.h;
                        acc += wm * phi_eval(a.kind, rho, a.a, a.s, a.p, a.c, a.cut) / (four_pi * rho * rho);
                    }
                }
            }
        }
    }
    a.table[e] = acc;
}

template <typename TL>
__global__ __launch_bounds__(256) void near_corr_kernel(NearArgs a, int64_t n_pts, const double *__restrict__ pos,
                                                        const TL *__restrict__ lum) {
    const int R = a.R, D = 2 * R + 1, W = R + 1;
    const int64_t V = (int64_t)D * D * D;
    const int n = a.n;
    const double four_pi = 12.566370614359172954;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_pts * V;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = e / V;
        const int o = (int)(e % V);
        const int o0 = o / (D * D) - R, o1 = (o / D) % D - R, o2 = o % D - R;
        if (!(o0 | o1 | o2)) continue;
        const double p0 = pos[3 * s], p1 = pos[3 * s + 1], p2 = pos[3 * s + 2];
        // a non-finite position has no cell (its slice is flagged by the deposit)
        if (!isfinite(p0) || !isfinite(p1) || !isfinite(p2)) continue;
        const double L = (double)lum[s];
        const double c0 = floor(p0 / a.l + 0.5), c1 = floor(p1 / a.l + 0.5), c2 = floor(p2 / a.l + 0.5);
        const double y0 = (c0 + o0) * a.l - p0, y1 = (c1 + o1) * a.l - p1, y2 = (c2 + o2) * a.l - p2;
        const double rho = sqrt(y0 * y0 + y1 * y1 + y2 * y2);
        double F = 0.0;
        if (rho >= a.r_lo && rho < a.r_hi)
            F = a.pref * phi_eval(a.kind, rho, a.a, a.s, a.p, a.c, a.cut) / (four_pi * rho * rho);
        const int t0 = o0 < 0 ? -o0 : o0, t1 = o1 < 0 ? -o1 : o1, t2 = o2 < 0 ? -o2 : o2;
        const double M = a.table[((int64_t)t0 * W + t1) * W + t2];
        const double dv = L * (F - M);
        if (dv == 0.0) continue;
        const int64_t cell =
            (wrap_node(c0 + o0, n) * n + wrap_node(c1 + o1, n)) * n + wrap_node(c2 + o2, n);
        atomicAdd(&a.corr[cell], dv);
    }
}

// nearest-node deposit of positioned sources (positions in length units,
// wrapped periodically)
template <typename TL>
__global__ __launch_bounds__(256) void deposit_pos_kernel(double *__restrict__ grid, int64_t n_pts,
                                                          const double *__restrict__ pos,
                                                          const TL *__restrict__ lum, int n, double l) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_pts;
         e += (int64_t)gridDim.x * blockDim.x) {
        const double p0 = pos[3 * e], p1 = pos[3 * e + 1], p2 = pos[3 * e + 2];
        if (!isfinite(p0) || !isfinite(p1) || !isfinite(p2)) {
            // no cell: make the slice's sum non-finite so that the check flags it
            atomicAdd(&grid[0], (double)NAN);
            continue;
        }
        const int64_t cell = (wrap_node(floor(p0 / l + 0.5), n) * n + wrap_node(floor(p1 / l + 0.5), n)) * n +
                             wrap_node(floor(p2 / l + 0.5), n);
        atomicAdd(&grid[cell], (double)lum[e]);
    }
}
#pragma clang fp contract(on)

template <typename TO>
__global__ __launch_bounds__(256) void add_grid_kernel(TO *__restrict__ out, const double *__restrict__ corr,
                                                       int64_t count) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        if (corr[e] != 0.0) out[e] = (TO)((double)out[e] + corr[e]);
}

hipError_t launch_near_table(const NearArgs &a, hipStream_t st) {
    const int64_t cells = (int64_t)(a.R + 1) * (a.R + 1) * (a.R + 1);
    hipLaunchKernelGGL(near_table_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_near_corr(const NearArgs &a, int64_t n_pts, const double *pos, const void *lum, bool lum_f64,
                            hipStream_t st) {
    if (n_pts <= 0) return hipSuccess;
    const int64_t D = 2 * a.R + 1;
    const int64_t work = n_pts * D * D * D;
    const int wgs = (int)std::min<int64_t>((work + 255) / 256, 16384);
    if (lum_f64)
        hipLaunchKernelGGL(near_corr_kernel<double>, dim3(wgs), dim3(256), 0, st, a, n_pts, pos,
                           (const double *)lum);
    else
        hipLaunchKernelGGL(near_corr_kernel<float>, dim3(wgs), dim3(256), 0, st, a, n_pts, pos,
                           (const float *)lum);
    return hipGetLastError();
}

hipError_t launch_deposit_pos(double *grid, int64_t n_pts, const double *pos, const void *lum, bool lum_f64, int n,
                              double l, hipStream_t st) {
    if (n_pts <= 0) return hipSuccess;
    const int wgs = (int)std::min<int64_t>((n_pts + 255) / 256, 8192);
    if (lum_f64)
        hipLaunchKernelGGL(deposit_pos_kernel<double>, dim3(wgs), dim3(256), 0, st, grid, n_pts, pos,
                           (const double *)lum, n, l);
    else
        hipLaunchKernelGGL(deposit_pos_kernel<float>, dim3(wgs), dim3(256), 0, st, grid, n_pts, pos,
                           (const float *)lum, n, l);
    return hipGetLastError();
}

hipError_t launch_add_grid(void *out, bool out_f64, const double *corr, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int wgs = (int)std::min<int64_t>((count + 255) / 256, 16384);
    if (out_f64)
        hipLaunchKernelGGL(add_grid_kernel<double>, dim3(wgs), dim3(256), 0, st, (double *)out, corr, count);
    else
        hipLaunchKernelGGL(add_grid_kernel<float>, dim3(wgs), dim3(256), 0, st, (float *)out, corr, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fill_f64_kernel(double *__restrict__ p, int64_t count, double v) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *__restrict__ p, int64_t count) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0u;
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t *__restrict__ p, int64_t count, int32_t v) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int wgs = (int)std::min<int64_t>((count + 255) / 256, 16384);
    hipLaunchKernelGGL(fill_i32_kernel, dim3(wgs), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void fdiff_kernel(const T *__restrict__ j, const T *__restrict__ ji,
                                                    T *__restrict__ out, int64_t count) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        const double a = (double)j[e], b = (double)ji[e];
        out[e] = (T)(a != 0.0 ? (b - a) / a : 0.0);
    }
}

hipError_t launch_fdiff(const void *j, const void *j_inst, void *out, int64_t count, bool f64, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int wgs = (int)std::min<int64_t>((count + 255) / 256, 16384);
    if (f64)
        hipLaunchKernelGGL(fdiff_kernel<double>, dim3(wgs), dim3(256), 0, st, (const double *)j,
                           (const double *)j_inst, (double *)out, count);
    else
        hipLaunchKernelGGL(fdiff_kernel<float>, dim3(wgs), dim3(256), 0, st, (const float *)j,
                           (const float *)j_inst, (float *)out, count);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, int64_t count, double v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int wgs = (int)std::min<int64_t>((count + 255) / 256, 16384);
    hipLaunchKernelGGL(fill_f64_kernel, dim3(wgs), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

hipError_t launch_fill_bytes(void *p, int64_t bytes, hipStream_t st) {
    if (bytes <= 0) return hipSuccess;
    if (bytes % 4) return hipErrorInvalidValue;
    const int64_t count = bytes / 4;
    const int wgs = (int)std::min<int64_t>((count + 255) / 256, 16384);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(wgs), dim3(256), 0, st, (uint32_t *)p, count);
    return hipGetLastError();
}

template <typename TL>
__global__ __launch_bounds__(256) void deposit_kernel(double *__restrict__ grid, int64_t n_pts,
                                                      const int64_t *__restrict__ cell,
                                                      const TL *__restrict__ lum, int64_t n_cells) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_pts;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = cell[e];
        if (c >= 0 && c < n_cells) atomicAdd(&grid[c], (double)lum[e]);
    }
}

hipError_t launch_deposit(double *grid, int64_t n_pts, const int64_t *cell, const void *lum,
                          bool lum_f64, int64_t n_cells, hipStream_t st) {
    if (n_pts <= 0) return hipSuccess;
    const int wgs = (int)std::min<int64_t>((n_pts + 255) / 256, 8192);
    if (lum_f64)
        hipLaunchKernelGGL(deposit_kernel<double>, dim3(wgs), dim3(256), 0, st, grid, n_pts, cell,
                           (const double *)lum, n_cells);
    else
        hipLaunchKernelGGL(deposit_kernel<float>, dim3(wgs), dim3(256), 0, st, grid, n_pts, cell,
                           (const float *)lum, n_cells);
    return hipGetLastError();
}

}  // namespace lc
