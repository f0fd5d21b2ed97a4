// oci_wb.hip -- the structured exact cell solve of one-cell inversion on
// gfx950 (FP64).
//
// Structure used (paper section 2.4: eqs. scatter_mg, fullOCIlhs and the
// remark on the occupancy of the cell matrix).  The cell matrix is
//   A_j = D - U C V^T,
// D = blockdiag over (g, m) of the 4x4 corner blocks L_{c,j,g,m} (eq. Aj),
// V^T x = the moments t_g = sum_m w_m x_{g,m} of the four corner unknowns (the
// scalar flux of x, eq. si_sf), C = (dx/4) Sigma_s (x) I_4 (eq. scatter with
// the weight of the column's angle) and U the copy of a group's source to
// every angle of the group: the scattering coupling has rank 4G.  Then
//   A x = b  <=>  z = D^-1 b,  (I - W C) t = V^T z,  x = z + D^-1 U C t,
// with W = V^T D^-1 U = blockdiag_g W_g, W_g = sum_m w_m L_{c,j,g,m}^-1; t is
// the scalar flux of x itself.  The 4G x 4G capacitance matrix I - W C and
// C (I - W C)^-1 are formed and inverted once per (dt, materials) per cell
// (k_wb_setup); an iteration then costs two 4x4 corner solves per (g, m), the
// moments, and two 4G x 4G products per cell, instead of an n x n product.
//
// Complex form of a corner block.  On the corner pair (L, R) of one time
// level, the blocks of L_c are d I + (mu/2) J0 (streaming + collision) or
// multiples of I (the time terms), with J0 = [[0, 1], [-1, 0]].  These 2x2
// matrices multiply like the complex numbers d + i mu/2 and act on the pair
// (v_L, v_R) as multiplication of v_L - i v_R.  So L_c is the complex 2x2
// matrix [[p, a/2], [-a, p + a]], p = d + i mu/2, d = (|mu| + dx Sigma_t)/2,
// a = dx / (v dt), with inverse
//   (1 / Delta) [[p + a, -a/2], [a, p]],   Delta = p (p + a) + a^2 / 2,
// written below with e2 = (a/2) / Delta, e3 = p / Delta (e1 = e3 + 2 e2).  W_g
// is the complex 2x2 matrix [[o1, -o2], [2 o2, o3]], o_k = sum_m w_m e_k, and
// I - W C is a complex 2G x 2G matrix (rows and columns (g, level)).
//
// The result is the exact OCI iterate (eq. oci) up to rounding, so a step
// stops where the dense solve stops.  Per iteration a thread owns Q of a
// cell's (g, m) pairs; a cell's lanes lie in one wave, so the moments and the
// capacitance products need only wave-local LDS.  Incident edges are read
// from the previous iterate in global memory (only the two outgoing corners
// of each (g, m) are written per iteration), and one grid barrier per
// iteration carries the norm (grid_sync_sum), as in the dense global kernel.
// When the stopping rule holds after iteration l, the workgroups recompute
// iteration l once more from the same inputs (identical arithmetic) and write
// the whole final iterate.
#include "oci_device.hpp"

namespace oci {

namespace {

struct cplx {
    double re, im;
};
__device__ inline cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline cplx cscale(double s, cplx a) { return {s * a.re, s * a.im}; }
__device__ inline double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
__device__ inline cplx crecip(cplx a) {
    const double q = 1.0 / cabs2(a);
    return {a.re * q, -a.im * q};
}

// e2 = (a/2) / Delta and e3 = p / Delta of the corner block with node mu,
// optical width tau = dx Sigma_t and time coefficient a = dx / (v dt).
__device__ inline void corner_inverse(double mu, double tau, double a, cplx &e2, cplx &e3) {
    const double d = 0.5 * (fabs(mu) + tau);
    const double h = 0.5 * mu;
    const cplx delta = {d * (d + a) - h * h + 0.5 * a * a, h * (2.0 * d + a)};
    const cplx r = crecip(delta);
    e2 = cscale(0.5 * a, r);
    e3 = cmul({d, h}, r);
}

// (X_k, X_h) = L_c^-1 (B_k, B_h) in the complex form.
__device__ inline void corner_apply(cplx e2, cplx e3, cplx bk, cplx bh, cplx &xk, cplx &xh) {
    const cplx r = cmul(e2, bk);
    xk = csub(cadd(cmul(e3, bk), cadd(r, r)), cmul(e2, bh));
    xh = cadd(cadd(r, r), cmul(e3, bh));
}

// sum_c row[c] v[c] for c < R: the row's words are loaded four at a time
// before their multiply-adds, so a row costs one memory round trip per four
// words instead of one per word.
__device__ inline cplx row_dot(const cplx *row, const cplx *v, int R) {
    cplx acc{0.0, 0.0};
    for (int c0 = 0; c0 < R; c0 += 4) {
        cplx w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = c0 + k < R ? row[c0 + k] : cplx{0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (c0 + k < R) acc = cadd(acc, cmul(w[k], v[c0 + k]));
    }
    return acc;
}

}  // namespace

constexpr int kWbMaxG = 8;     // capacitance systems up to 2G = 16 complex unknowns
constexpr int kWbMaxN = 128;   // quadrature nodes staged in LDS

// ------------------------------------------------------------------ setup
// One wave per cell: W_g (moments of the corner inverses, ascending m), the
// capacitance matrix M = I - W C, its inverse by Gauss-Jordan elimination with
// row exchanges (largest modulus, lowest row on ties), then the rows of M^-1
// and of C M^-1 into S.wb.  A zero pivot raises the control block's
// `singular` flag.
__global__ __launch_bounds__(64) void k_wb_setup(Slab S, int j0) {
    const int j = j0 + blockIdx.x;
    const int lane = threadIdx.x;
    const int G = S.G, N = S.N, R = 2 * G;
    __shared__ cplx s_om[kWbMaxG][3];
    __shared__ cplx s_m[2 * kWbMaxG][4 * kWbMaxG];
    __shared__ cplx s_f[2 * kWbMaxG];
    __shared__ int s_piv, s_sing;
    const double dx = S.dx[j];
    if (lane < G) {
        const int g = lane;
        const double tau = dx * S.sigma_t[(size_t)j * G + g];
        const double a = dx / (S.speed[g] * S.dt);
        cplx o2{0.0, 0.0}, o3{0.0, 0.0};
        for (int m = 0; m < N; ++m) {
            cplx e2, e3;
            corner_inverse(S.mu[m], tau, a, e2, e3);
            o2 = cadd(o2, cscale(S.w[m], e2));
            o3 = cadd(o3, cscale(S.w[m], e3));
        }
        s_om[g][0] = cadd(o3, cadd(o2, o2));
        s_om[g][1] = o2;
        s_om[g][2] = o3;
    }
    if (lane == 0) s_sing = 0;
    __syncthreads();
    // [M | I]: M[(g, k)][(g', k')] = delta - (dx/4) Sigma_s[g][g'] W_g[k][k']
    for (int e = lane; e < R * 2 * R; e += 64) {
        const int r = e / (2 * R), c = e % (2 * R);
        cplx v{0.0, 0.0};
        if (c < R) {
            const int g = r >> 1, k = r & 1, gp = c >> 1, kp = c & 1;
            const double cs = 0.25 * dx * S.sigma_s[((size_t)j * G + g) * G + gp];
            const cplx o2 = s_om[g][1];
            const cplx wv = k == 0 ? (kp == 0 ? s_om[g][0] : cplx{-o2.re, -o2.im})
                                   : (kp == 0 ? cadd(o2, o2) : s_om[g][2]);
            v = cscale(-cs, wv);
            if (r == c) v.re += 1.0;
            if (j == S.zero_cell) v = cplx{0.0, 0.0};   // test hook: a zero pivot
        } else if (c - R == r) {
            v.re = 1.0;
        }
        s_m[r][c] = v;
    }
    __syncthreads();
    for (int k = 0; k < R; ++k) {
        if (lane == 0) {
            int p = k;
            double best = cabs2(s_m[k][k]);
            for (int r = k + 1; r < R; ++r) {
                const double v = cabs2(s_m[r][k]);
                if (v > best) { best = v; p = r; }
            }
            s_piv = p;
            if (!(best > 0.0)) s_sing = 1;   // zero or not finite
        }
        __syncthreads();
        if (s_sing) break;
        const int p = s_piv;
        if (p != k)
            for (int c = lane; c < 2 * R; c += 64) {
                const cplx t = s_m[k][c];
                s_m[k][c] = s_m[p][c];
                s_m[p][c] = t;
            }
        __syncthreads();
        const cplx ip = crecip(s_m[k][k]);
        __syncthreads();
        for (int c = lane; c < 2 * R; c += 64) s_m[k][c] = cmul(s_m[k][c], ip);
        if (lane < R) s_f[lane] = s_m[lane][k];
        __syncthreads();
        for (int e = lane; e < R * 2 * R; e += 64) {
            const int r = e / (2 * R), c = e % (2 * R);
            if (r != k) s_m[r][c] = csub(s_m[r][c], cmul(s_f[r], s_m[k][c]));
        }
        __syncthreads();
    }
    if (s_sing) {
        if (lane == 0) __hip_atomic_store(&S.ctl->singular, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    cplx *out = reinterpret_cast<cplx *>(S.wb) + (size_t)j * 2 * R * R;
    for (int e = lane; e < R * R; e += 64) {
        const int r = e / R, c = e % R;
        out[e] = s_m[r][R + c];
        const int g = r >> 1, k = r & 1;
        cplx acc{0.0, 0.0};
        for (int gp = 0; gp < G; ++gp)
            acc = cadd(acc, cscale(0.25 * dx * S.sigma_s[((size_t)j * G + g) * G + gp], s_m[2 * gp + k][R + c]));
        out[R * R + e] = acc;
    }
}

hipError_t launch_wb_setup(const Slab &S, hipStream_t st) {
    if (S.G > kWbMaxG) return hipErrorInvalidValue;
    const int chunk = 65535;
    for (int j0 = 0; j0 < S.J; j0 += chunk) {
        const int nb = (S.J - j0) < chunk ? (S.J - j0) : chunk;
        hipLaunchKernelGGL(k_wb_setup, dim3(nb), dim3(64), 0, st, S, j0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------ iteration
// Lanes per cell: the (g, m) pairs of a cell, padded to a power of two, at
// most a wave; Q = pairs per lane (1, or 2 when a cell has more than 64).
struct WbShape {
    int lc, cpw;   // lanes per cell, cells per wave
};
__host__ __device__ inline WbShape wb_shape(int NG) {
    int p = 1;
    while (p < NG) p <<= 1;
    const int lc = p < 64 ? p : 64;
    return WbShape{lc, 64 / lc};
}

// LDS per wave, in complex words: area A holds the weighted corner solutions
// w_m z of the wave's pairs, then the rows' results t and C t (4G per cell);
// area B the moments V^T z (2G per cell).
template <int Q>
struct WbLds {
    static constexpr int kA = 128 * Q;
    static constexpr int kB = 64 * Q;
};

template <int Q, int BS>
__device__ __attribute__((always_inline)) inline void wb_body(const Slab &S, const StepIO &io, int ntiles, int wg,
                                                         unsigned nwg, cplx *lds, double *s_tmp, int *s_flag,
                                                         double *s_ivdt, double *s_mu, double *s_w) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int J = S.J, N = S.N, G = S.G, NG = N * G, nh = N / 2, R = 2 * G;
    const WbShape sh = wb_shape(NG);
    const int cw = lane / sh.lc, li = lane % sh.lc;
    constexpr int W = BS / 64;
    const int cpt = W * sh.cpw;
    cplx *A = lds + (size_t)wave * (WbLds<Q>::kA + WbLds<Q>::kB);
    cplx *B = A + WbLds<Q>::kA;
    cplx *Acell = A + (size_t)cw * sh.lc * Q * 2;       // this cell's w_m z pairs
    cplx *Tcell = A + (size_t)cw * 2 * R;               // ... later its t and C t rows
    cplx *Zcell = B + (size_t)cw * R;                   // its moments
    const int tile0 = (int)(((long)ntiles * wg) / nwg);
    const int tile1 = (int)(((long)ntiles * (wg + 1)) / nwg);
    for (int g = tid; g < G; g += BS) s_ivdt[g] = 1.0 / (S.speed[g] * S.dt);
    for (int m = tid; m < N; m += BS) { s_mu[m] = S.mu[m]; s_w[m] = S.w[m]; }
    __syncthreads();
    // outgoing corners of iteration l go to the compact edge buffer of parity
    // l, through coherent stores (other workgroups read them after the grid
    // barrier); the first iteration reads its upstream corners from the first
    // iterate, written before the launch
    const size_t ehalf = (size_t)J * NG * 2;

    // Red-black ordering (S.ordering = 1): an iteration is two half-sweeps,
    // the even cells from the previous iterate's edges, then, after a grid
    // barrier, the odd cells from the even cells' new edges; tiles then run
    // over the cells of one colour.  With a periodic mesh cell 0 and cell J-1
    // are neighbours.
    const bool rb = S.ordering == 1;
    const int nhalf = rb ? 2 : 1;
    double e_prev = __builtin_nan("");
    const int base = S.ctl->base;
    for (int l = 0;; ++l) {
        const int cur = (base + l) & 1;
        const double *__restrict__ psi_in = S.psi[cur];
        double *__restrict__ psi_out = S.psi[cur ^ 1];
        const double *__restrict__ phi_in = S.phi[cur];
        double *__restrict__ phi_out = S.phi[cur ^ 1];
        double *__restrict__ e_out = S.edge + (size_t)(l & 1) * ehalf;
        const double *__restrict__ e_in = S.edge + (size_t)((l + 1) & 1) * ehalf;
        double dsq = 0.0;   // summed per lane over its tiles in order, reduced once per iteration
        bool fin = false;
        // one pass per iteration; after a stop, one more pass over the same
        // inputs writes the whole final iterate
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1 && !fin) break;
            for (int half = 0; half < nhalf; ++half) {
            // upstream corners: the first iterate (iteration 0, even cells),
            // the previous iteration's, or (odd cells of red-black) the even
            // cells' of this iteration
            const bool from_iterate = l == 0 && half == 0;
            const double *edges = half == 1 ? e_out : e_in;
            for (int tile = tile0; tile < tile1; ++tile) {
                const int cc = tile * cpt + wave * sh.cpw + cw;
                const int j = rb ? 2 * cc + half : cc;
                const bool cell = j < J;
                const double dx = cell ? S.dx[j] : 0.0;
                // this lane's entry of the previous scalar flux (a cell's first
                // R lanes, one (g, level) each: R = 2G <= NG <= lanes per cell),
                // loaded early so that its latency hides behind the solves
                double2 fprev{0.0, 0.0};
                if (cell && pass == 0 && li < R)
                    fprev = *reinterpret_cast<const double2 *>(phi_in + (size_t)j * 4 * G + 2 * li);
                cplx z[Q][2], e2[Q], e3[Q];
                // (1) b = constant part + lagged incident edge (eq. rhs_sg);
                //     z = L_c^-1 b; the weighted z into LDS for the moments
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int i = li + q * sh.lc;
                    z[q][0] = z[q][1] = cplx{0.0, 0.0};
                    e2[q] = e3[q] = cplx{0.0, 0.0};
                    cplx wz0{0.0, 0.0}, wz1{0.0, 0.0};
                    if (cell && i < NG) {
                        const int g = i / N, m = i % N;
                        const double mu = s_mu[m];
                        const size_t row = ((size_t)j * G + g) * N + m;
                        // constant part of b (eq. rhs_sg): dx/4 Q, plus dx/(2 v dt)
                        // psi_{k-1/2} in the level-k rows
                        const double2 pp = *reinterpret_cast<const double2 *>(S.psi_prev + row * 2);
                        const double ht = 0.5 * dx * s_ivdt[g];
                        double b0 = ht * pp.x, b1 = ht * pp.y, b2 = 0.0, b3 = 0.0;
                        if (io.q) {
                            const double *qq = io.q + ((size_t)j * G + g) * 4;
                            const double q4 = 0.25 * dx;
                            b0 += q4 * qq[0];
                            b1 += q4 * qq[1];
                            b2 = q4 * qq[2];
                            b3 = q4 * qq[3];
                        }
                        if (m >= nh) {   // mu > 0: upstream is the right corner of cell j - 1
                            double ek = 0.0, eh = 0.0;
                            if (j > 0 || S.periodic) {
                                const size_t up = j > 0 ? row - (size_t)NG : row + (size_t)(J - 1) * NG;
                                if (from_iterate) {
                                    ek = psi_in[up * 4 + 1];
                                    eh = psi_in[up * 4 + 3];
                                } else {
                                    ek = ld_coherent(edges + up * 2);
                                    eh = ld_coherent(edges + up * 2 + 1);
                                }
                            } else if (io.inc_l) {
                                ek = io.inc_l[(size_t)g * nh + (m - nh)];
                                eh = io.inc_l[((size_t)G + g) * nh + (m - nh)];
                            }
                            b0 += mu * ek;
                            b2 += mu * eh;
                        } else {         // mu < 0: upstream is the left corner of cell j + 1
                            double ek = 0.0, eh = 0.0;
                            if (j < J - 1 || S.periodic) {
                                const size_t up = j < J - 1 ? row + (size_t)NG : row - (size_t)(J - 1) * NG;
                                if (from_iterate) {
                                    ek = psi_in[up * 4 + 0];
                                    eh = psi_in[up * 4 + 2];
                                } else {
                                    ek = ld_coherent(edges + up * 2);
                                    eh = ld_coherent(edges + up * 2 + 1);
                                }
                            } else if (io.inc_r) {
                                ek = io.inc_r[(size_t)g * nh + m];
                                eh = io.inc_r[((size_t)G + g) * nh + m];
                            }
                            b1 -= mu * ek;
                            b3 -= mu * eh;
                        }
                        corner_inverse(mu, dx * S.sigma_t[(size_t)j * G + g], dx * s_ivdt[g], e2[q], e3[q]);
                        corner_apply(e2[q], e3[q], cplx{b0, -b1}, cplx{b2, -b3}, z[q][0], z[q][1]);
                        const double w = s_w[m];
                        wz0 = cscale(w, z[q][0]);
                        wz1 = cscale(w, z[q][1]);
                    }
                    Acell[(size_t)i * 2 + 0] = wz0;
                    Acell[(size_t)i * 2 + 1] = wz1;
                }
                wave_sync();
                // (2) moments V^T z, ascending m, one lane per (g, level)
                for (int o = li; o < R; o += sh.lc) {
                    const int g = o >> 1, k = o & 1;
                    cplx s{0.0, 0.0};
                    for (int m = 0; m < N; ++m) s = cadd(s, Acell[((size_t)g * N + m) * 2 + k]);
                    Zcell[o] = s;
                }
                wave_sync();
                // (3) t = (I - W C)^-1 V^T z and C t: one lane per row of the
                //     cell's [4G][2G] block
                //     (a lane has at most two rows: 4G <= 2 x lanes per cell)
                const int o0 = li, o1 = li + sh.lc;
                cplx r0{0.0, 0.0}, r1{0.0, 0.0};
                if (cell) {
                    const cplx *Mj = reinterpret_cast<const cplx *>(S.wb) + (size_t)j * 2 * R * R;
                    if (o0 < 2 * R) r0 = row_dot(Mj + (size_t)o0 * R, Zcell, R);
                    if (o1 < 2 * R) r1 = row_dot(Mj + (size_t)o1 * R, Zcell, R);
                }
                wave_sync();   // area A's weighted z is no longer needed
                if (cell && o0 < 2 * R) Tcell[o0] = r0;
                if (cell && o1 < 2 * R) Tcell[o1] = r1;
                wave_sync();
                // (4) x = z + L_c^-1 (C t)_g; outgoing corners (every corner
                //     on the final pass)
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int i = li + q * sh.lc;
                    if (cell && i < NG) {
                        const int g = i / N, m = i % N;
                        cplx sk, sh_;
                        corner_apply(e2[q], e3[q], Tcell[R + 2 * g], Tcell[R + 2 * g + 1], sk, sh_);
                        const cplx xk = cadd(z[q][0], sk), xh = cadd(z[q][1], sh_);
                        const size_t row = ((size_t)j * G + g) * N + m;
                        if (pass == 1) {
                            double *p = psi_out + row * 4;
                            *reinterpret_cast<double2 *>(p) = double2{xk.re, -xk.im};
                            *reinterpret_cast<double2 *>(p + 2) = double2{xh.re, -xh.im};
                        } else if (m >= nh) {   // the right corner travels downstream
                            st_coherent(e_out + row * 2, -xk.im);
                            st_coherent(e_out + row * 2 + 1, -xh.im);
                        } else {                // the left corner
                            st_coherent(e_out + row * 2, xk.re);
                            st_coherent(e_out + row * 2 + 1, xh.re);
                        }
                    }
                }
                // (5) the scalar flux is t itself; its change for the norm
                if (cell && pass == 0 && li < R) {
                    const cplx t = Tcell[li];
                    const double n0 = t.re, n1 = -t.im;
                    *reinterpret_cast<double2 *>(phi_out + (size_t)j * 4 * G + 2 * li) = double2{n0, n1};
                    dsq += (n0 - fprev.x) * (n0 - fprev.x) + (n1 - fprev.y) * (n1 - fprev.y);
                }
                wave_sync();   // area A is rewritten by the next tile
            }
            // red-black: the odd cells wait for every even cell's new edges
            // (a grid barrier whose sum is not used)
            if (pass == 0 && rb && half == 0) {
                double unused = 0.0;
                if (!grid_sync_coherent<BS>(S, wg, nwg, 2 * l, 0.0, s_flag, s_tmp, &unused)) return;
            }
            }
            if (pass == 1) break;
            // (6) grid barrier + reduction; every workgroup decides identically
            const double wg_sum = block_sum_t<BS>(dsq, s_tmp);   // valid in thread 0
            double tot = 0.0;
            if (!grid_sync_coherent<BS>(S, wg, nwg, rb ? 2 * l + 1 : l, wg_sum, s_flag, s_tmp, &tot)) return;
            const int iters = l + 1;
            const double e = sqrt(tot);
            const double rho = iters >= 2 ? e / e_prev : __builtin_nan("");
            int done = 0, status = OK;
            if (!isfinite(e)) { done = 1; status = NONFINITE; }
            else if (S.fixed_iters > 0) done = iters >= S.fixed_iters;
            else if (iters >= 2 && (e == 0.0 || e < S.tol * (1.0 - e / e_prev))) done = 1;
            else if (iters >= S.max_iters) { done = 1; status = NOT_CONVERGED; }
            e_prev = e;
            if (S.hist && iters <= S.hist_cap && wg == 0 && tid == 0) S.hist[iters - 1] = e;
            if (done) {
                if (wg == 0 && tid == 0) {
                    Ctl *c = S.ctl;
                    c->iter = iters;
                    c->e_last = e;
                    c->rho = rho;
                    c->e_prev = e;
                    c->status = status;
                    c->done = 1;
                }
                fin = true;
            }
        }
        if (fin) return;
    }
}

template <int Q, int BS>
__global__ __launch_bounds__(BS) void k_oci_wb(Slab S, StepIO io, int ntiles) {
    __shared__ __align__(16) cplx s_lds[(BS / 64) * (WbLds<Q>::kA + WbLds<Q>::kB)];
    __shared__ double s_tmp[BS / 64 + 1];
    __shared__ int s_flag[4];
    __shared__ double s_ivdt[kWbMaxG];
    __shared__ double s_mu[kWbMaxN], s_w[kWbMaxN];
    wb_body<Q, BS>(S, io, ntiles, blockIdx.x, gridDim.x, s_lds, s_tmp, s_flag, s_ivdt, s_mu, s_w);
}

// Many slabs in one persistent launch: slab k owns the workgroups
// [wg0, wg0 + nwg) and runs the structured body on its own control block,
// barrier words and partial sums, so slabs converge independently (the
// structured counterpart of the dense batched kernel).
template <int BS>
__global__ __launch_bounds__(BS) void k_wb_batch(const BatchEntry *tab, int nslab) {
    __shared__ __align__(16) cplx s_lds[(BS / 64) * (WbLds<2>::kA + WbLds<2>::kB)];
    __shared__ double s_tmp[BS / 64 + 1];
    __shared__ int s_flag[4];
    __shared__ double s_ivdt[kWbMaxG];
    __shared__ double s_mu[kWbMaxN], s_w[kWbMaxN];
    __shared__ int s_k;
    if (threadIdx.x == 0) {
        int lo = 0, hi = nslab - 1;     // last entry with wg0 <= blockIdx.x
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tab[mid].wg0 <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
        }
        s_k = lo;
    }
    __syncthreads();
    const BatchEntry &e = tab[__builtin_amdgcn_readfirstlane(s_k)];
    const int lw = (int)blockIdx.x - e.wg0;
    if (lw < 0 || lw >= e.nwg) return;
    if (e.S.N * e.S.G > 64)
        wb_body<2, BS>(e.S, e.io, e.ntiles, lw, e.nwg, s_lds, s_tmp, s_flag, s_ivdt, s_mu, s_w);
    else
        wb_body<1, BS>(e.S, e.io, e.ntiles, lw, e.nwg, s_lds, s_tmp, s_flag, s_ivdt, s_mu, s_w);
}

constexpr int kWbBlock = 256;

hipError_t wb_batch_occupancy(int *blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void *)&k_wb_batch<kWbBlock>, kWbBlock, 0);
}

hipError_t launch_wb_batch(const BatchEntry *tab, int nslab, int nwg, hipStream_t st) {
    hipLaunchKernelGGL((k_wb_batch<kWbBlock>), dim3(nwg), dim3(kWbBlock), 0, st, tab, nslab);
    return hipGetLastError();
}

int wb_cells_per_tile(int N, int G) { return (kWbBlock / 64) * wb_shape(N * G).cpw; }
int wb_block() { return kWbBlock; }

hipError_t wb_occupancy(int N, int G, int *blocks) {
    const void *f = N * G > 64 ? (const void *)&k_oci_wb<2, kWbBlock> : (const void *)&k_oci_wb<1, kWbBlock>;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, f, kWbBlock, 0);
}

hipError_t launch_oci_wb(const Slab &S, const StepIO &io, int nwg, int ntiles, hipStream_t st) {
    if (S.N * S.G > 64)
        hipLaunchKernelGGL((k_oci_wb<2, kWbBlock>), dim3(nwg), dim3(kWbBlock), 0, st, S, io, ntiles);
    else
        hipLaunchKernelGGL((k_oci_wb<1, kWbBlock>), dim3(nwg), dim3(kWbBlock), 0, st, S, io, ntiles);
    return hipGetLastError();
}

}  // namespace oci
