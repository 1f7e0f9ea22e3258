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

// ---------------------------------------------------------------------------
// Exact cell average (rule 1)
//
// For an image cell [x0,x1] x [y0,y1] x [z0,z1] of the unit source at the
// origin, cylindrical coordinates about the z axis (radius R) and
// w = asinh(z / R) (so r = R cosh w and dz / r^2 = dw / (R cosh w)) give
//   pref / l^3 int_cell phi(r) / (4 pi r^2) [r_lo <= r < r_sup] d^3x
//     = pref / (4 pi l^3) int Q(R) V(R) dR,
//   Q(R) = angle of the circle of radius R inside [x0,x1] x [y0,y1],
//   V(R) = int phi(R cosh w) / cosh w dw over w in [asinh(z0/R), asinh(z1/R)]
//          with R cosh w in [r_lo, r_sup).
// Q is formed by inclusion-exclusion over the rectangle's corners of the
// arcs {R cos t >= a} and {R sin t >= b}; V is atan(sinh w) at the interval
// ends for phi = 1, else a 16-point rule on pieces of at most 2 in w (|w|
// <= 40: the weight 1 / cosh w is below 1e-17 beyond). The R integral is
// split where Q or V change form (edge and corner distances of the
// rectangle, r_lo, r_sup, sqrt(r^2 - z^2) for the z faces); each piece takes
// the 16-point rule after R = Ra + (Rb - Ra)(1 - cos u) / 2, which smooths the
// square-root behaviour at piece ends, on parts graded towards any such
// point that lies just outside it. In the cell holding the source,
// V(R) ~ V(0) - C R^p near R = 0 (the r^p cusp of phi at r = 0), so the
// piece from R = 0 is split geometrically at Rb 2^-j, j < 50, each part
// with the same substitution.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double arc_overlap(double a, double b, double c, double d) {
    const double lo = fmax(a, c), hi = fmin(b, d);
    return hi > lo ? hi - lo : 0.0;
}

// angle of {t : R cos t >= a and R sin t >= b}: the arc [-al, al] against
// the arc [be, pi - be] (and its copy one turn lower)
__device__ double arc_quarter(double R, double a, double b) {
    const double pi = 3.141592653589793238;
    const double al = acos(fmin(1.0, fmax(-1.0, a / R)));
    const double be = asin(fmin(1.0, fmax(-1.0, b / R)));
    return arc_overlap(-al, al, be, pi - be) + arc_overlap(-al, al, be - 2.0 * pi, -pi - be);
}

__device__ double circle_in_rect(double R, double x0, double x1, double y0, double y1) {
    return arc_quarter(R, x0, y0) - arc_quarter(R, x1, y0) - arc_quarter(R, x0, y1) + arc_quarter(R, x1, y1);
}

__device__ double exact_v(const ExactRule &e, double R, double z0, double z1) {
    if (!(R < e.r_sup)) return 0.0;
    const double wH = acosh(e.r_sup / R), wL = R < e.r_lo ? acosh(e.r_lo / R) : 0.0;
    const double wa = asinh(z0 / R), wb = asinh(z1 / R);
    double acc = 0.0;
    for (int side = 0; side < 2; ++side) {
        double lo = side ? fmax(wa, wL) : fmax(wa, -wH);
        double hi = side ? fmin(wb, wH) : fmin(wb, -wL);
        if (!(hi > lo)) continue;
        if (e.kind == 0) {
            acc += atan(sinh(hi)) - atan(sinh(lo));
            continue;
        }
        lo = fmax(lo, -40.0);
        hi = fmin(hi, 40.0);
        if (!(hi > lo)) continue;
        const int pieces = (int)ceil((hi - lo) * 0.5);
        const double len = (hi - lo) / pieces;
        for (int q = 0; q < pieces; ++q) {
            const double w0 = lo + q * len;
            double sq = 0.0;
            for (int j = 0; j < 16; ++j) {
                const double w = w0 + len * e.gx[j], ch = cosh(w), r = R * ch;
                const double v = e.a * exp(-pow(r / e.s, e.p)) - e.c;
                const double ph = (e.kind == 1 && v < 0.0) ? 0.0 : v;   // (kind 2: r < r_sup <= cut)
                sq += e.gw[j] * ph / ch;
            }
            acc += len * sq;
        }
    }
    return acc;
}

__device__ double cell_exact(const ExactRule &e, double x0, double x1, double y0, double y1, double z0, double z1) {
    if (!(e.r_sup > e.r_lo)) return 0.0;
    const double nx = x0 > 0.0 ? x0 : (x1 < 0.0 ? -x1 : 0.0);
    const double ny = y0 > 0.0 ? y0 : (y1 < 0.0 ? -y1 : 0.0);
    const double Rmin = sqrt(nx * nx + ny * ny);
    const double fx = fmax(fabs(x0), fabs(x1)), fy = fmax(fabs(y0), fabs(y1));
    const double Rmax = fmin(sqrt(fx * fx + fy * fy), e.r_sup);
    if (!(Rmax > Rmin)) return 0.0;
    // every R where Q or V may change form (sing), and those inside the
    // range, sorted by insertion (br)
    double sing[20], br[20];
    int ns = 0, nb = 0;
    auto add = [&](double v) {
        sing[ns++] = v;
        if (!(v > Rmin && v < Rmax)) return;
        int i = nb++;
        while (i > 0 && br[i - 1] > v) { br[i] = br[i - 1]; --i; }
        br[i] = v;
    };
    const double xs[2] = {x0, x1}, ys[2] = {y0, y1}, zs[2] = {z0, z1}, rs[2] = {e.r_lo, e.r_sup};
    for (int i = 0; i < 2; ++i) {
        add(fabs(xs[i]));
        add(fabs(ys[i]));
        for (int j = 0; j < 2; ++j) {
            add(sqrt(xs[i] * xs[i] + ys[j] * ys[j]));
            if (rs[i] > fabs(zs[j])) add(sqrt(rs[i] * rs[i] - zs[j] * zs[j]));
        }
    }
    add(e.r_lo);
    add(e.r_sup);
    add(0.0);
    const bool source_cell = nx == 0.0 && ny == 0.0 && z0 <= 0.0 && z1 >= 0.0;
    // 16-point rule on [lo, hi] after the cosine substitution
    auto piece = [&](double lo, double hi) {
        const double pi = 3.141592653589793238;
        double sq = 0.0;
        for (int j = 0; j < 16; ++j) {
            const double u = pi * e.gx[j];
            const double R = lo + 0.5 * (hi - lo) * (1.0 - cos(u));
            const double jac = pi * 0.5 * (hi - lo) * sin(u);
            sq += e.gw[j] * jac * circle_in_rect(R, x0, x1, y0, y1) * exact_v(e, R, z0, z1);
        }
        return sq;
    };
    double acc = 0.0;
    double Ra = Rmin;
    for (int pc = 0; pc <= nb; ++pc) {
        const double Rb = pc < nb ? br[pc] : Rmax;
        if (!(Rb > Ra)) continue;
        if (Ra == 0.0 && source_cell) {
            // (the top piece keeps the substitution: R = Rb may be a square-root end)
            double hi = Rb;
            for (int g = 0; g < 50; ++g) {
                acc += piece(0.5 * hi, hi);
                hi *= 0.5;
            }
        } else {
            // A change of form just outside the piece, at distance dl < len
            // from Ra (a shell radius close to an edge distance, say), slows
            // the rule's convergence. The piece is then halved, and the half
            // at Ra is cut into parts graded towards it: [Ra, Ra + dl], then
            // parts as long as their distance to Ra (which, being a piece
            // end, may itself be such a point), up to the middle. The same
            // towards Rb with dr.
            double dl = 1e300, dr = 1e300;
            for (int i = 0; i < ns; ++i) {
                if (sing[i] < Ra) dl = fmin(dl, Ra - sing[i]);
                if (sing[i] > Rb) dr = fmin(dr, sing[i] - Rb);
            }
            const double len = Rb - Ra;
            if (dl >= len && dr >= len) {
                acc += piece(Ra, Rb);
            } else {
                const double mid = Ra + 0.5 * len;
                double lo = Ra;
                if (dl < mid - lo) {
                    acc += piece(lo, lo + dl);
                    lo += dl;
                    for (int g = 0; g < 64 && lo - Ra < mid - lo; ++g) {
                        const double d = lo - Ra;
                        acc += piece(lo, lo + d);
                        lo += d;
                    }
                }
                acc += piece(lo, mid);
                double hi = Rb;
                if (dr < hi - mid) {
                    acc += piece(hi - dr, hi);
                    hi -= dr;
                    for (int g = 0; g < 64 && Rb - hi < hi - mid; ++g) {
                        const double d = Rb - hi;
                        acc += piece(hi - d, hi);
                        hi -= d;
                    }
                }
                acc += piece(mid, hi);
            }
        }
        Ra = Rb;
    }
    const double four_pi = 12.566370614359172954;
    return e.pref * acc / (four_pi * e.l * e.l * e.l);
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
                if (a.rule == 1) {
                    acc += cell_exact(a.ex, lo0, hi0, lo1, hi1, lo2, hi2);
                    continue;
                }
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
    if ((d0 | d1 | d2) && a.rule == 1) {
        const double l = a.l;
        acc = cell_exact(a.ex, (d0 - 0.5) * l, (d0 + 0.5) * l, (d1 - 0.5) * l, (d1 + 0.5) * l, (d2 - 0.5) * l,
                         (d2 + 0.5) * l);
    } else if (d0 | d1 | d2) {
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
