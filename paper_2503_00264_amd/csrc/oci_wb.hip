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
// capacitance products need only the wave (cross-lane sums, wave-local LDS).
// Incident edges are read from the previous iterate in global memory (only
// the two outgoing corners of each (g, m) are written per iteration), and one
// grid barrier per iteration carries the norm (grid_sync_coherent).
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

// corner_inverse with the reciprocal from the hardware estimate refined by
// two Newton steps (r <- r (2 - q r)) instead of the correctly rounded
// division: a relative error of a few units in the last place, no
// division sequence (the staged body recomputes it every iteration).
__device__ inline void corner_inverse_nr(double mu, double tau, double a, cplx &e2, cplx &e3) {
    const double d = 0.5 * (fabs(mu) + tau);
    const double h = 0.5 * mu;
    const cplx delta = {d * (d + a) - h * h + 0.5 * a * a, h * (2.0 * d + a)};
    const double q = cabs2(delta);
    double r = __builtin_amdgcn_rcp(q);
    r = fma(r, fma(-q, r, 1.0), r);
    r = fma(r, fma(-q, r, 1.0), r);
    const cplx inv = {delta.re * r, -delta.im * r};
    e2 = cscale(0.5 * a, inv);
    e3 = cmul({d, h}, inv);
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
// The stopping rule after iteration l (0-based) from the squared norm of the
// scalar-flux change; every workgroup takes the same decision.  Returns true
// when the step ends (thread 0 of workgroup 0 records the outcome).
__device__ inline bool wb_decide(const Slab &S, int wg, int l, double tot, double &e_prev) {
    const int iters = l + 1;
    const double e = sqrt(tot);
    const double rho = iters >= 2 ? e / e_prev : __builtin_nan("");
    int status = OK;
    const int done = stop_rule(S, iters, e, e_prev, &status);
    e_prev = e;
    if (S.hist && iters <= S.hist_cap && wg == 0 && threadIdx.x == 0) S.hist[iters - 1] = e;
    if (done && wg == 0 && threadIdx.x == 0) {
        Ctl *c = S.ctl;
        c->t_end = wall_clock64();
        c->iter = iters;
        c->e_last = e;
        c->rho = rho;
        c->e_prev = e;
        c->status = status;
        c->done = 1;
    }
    return done != 0;
}

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
    if (wg == 0 && tid == 0) S.ctl->t_begin = wall_clock64();
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
            fin = wb_decide(S, wg, l, tot, e_prev);
        }
        if (fin) return;
    }
}

// ------------------------------------------------------ staged iteration
// The same iteration with the inputs of a tile staged into LDS by the memory
// system (global_load_lds: the data lands in LDS without passing through
// registers), one tile ahead of the arithmetic, so a wave keeps a tile's worth
// of loads in flight while it computes the previous tile.  Per tile t a wave
//   waits for the staged data of t: the rows of (I - W C)^-1 of its cells,
//   then psi_{k-1/2}, upstream corners, the cells' sources, scalar flux,
//   cross sections and widths;
//   reads all of it from LDS before using any, and the incident flux at the
//   slab's ends; then issues the staging of t + 1 (the rows into the other of
//   two row buffers, then the inputs);
//   forms b and z = L_c^-1 b and sums the moments over m across the N lanes
//   of each group (DPP and permlane exchanges, no LDS);
//   forms t = (I - W C)^-1 V^T z and C t = (dx/4) (Sigma_s (x) I) t; stores
//   the new scalar flux;
//   forms x = z + L_c^-1 (C t)_g and stores the outgoing corners.
// Vector memory operations complete in issue order, so "the loads of t have
// landed" is "at most k operations are outstanding", k the number issued
// after them: the previous tile's stores, one for the scalar flux and Q for
// the corners (2Q and none on the final pass, which is more).  Every staging
// load and every store is issued by all 64 lanes (addresses of idle lanes
// clamped into the slab, stores of idle lanes sent past the end of a buffer
// resource, which drops them), and after the staging of a wave's first tile
// come 1 + Q one-dword loads into a slot that nothing reads, so one wait with
// a fixed count serves every tile.  (A store that every lane drops is never
// counted on: it need not wait for the memory system to retire.)
// Shapes: N a power of two in [8, 64], G in {1, 2, 4}, at most two pairs per
// lane, a wave's rows of (I - W C)^-1 within 2 KiB and its per-cell data
// within 1 KiB (wb_staged_shape); other shapes take the direct body above.
typedef __attribute__((address_space(3))) void lds_void;
typedef unsigned v4u __attribute__((ext_vector_type(4)));

__host__ __device__ inline bool wb_staged_shape(long J, int N, int G) {
    if (N < 8 || N > 64 || (N & (N - 1))) return false;
    if (G != 1 && G != 2 && G != 4) return false;
    const int NG = N * G;
    if (NG > 128) return false;
    const WbShape sh = wb_shape(NG);
    if (sh.cpw * 4 * G * G > 128) return false;                          // rows: 128 complex words
    if (sh.cpw * G > 8 || sh.cpw > 8) return false;                      // per-cell data: four 64-dword loads
    return J * NG * 32 < (1L << 31);                                     // 32-bit buffer offsets
}

// Byte layout of one wave's LDS area in the staged body.
template <int Q>
struct WbStage {
    static constexpr int kP = 0;               // psi_{k-1/2} of the lanes' pairs: [Q][64] x 16 B
    static constexpr int kE = kP + Q * 1024;   // upstream corners: [Q][64] x 16 B, or [Q][4][64] dwords
    static constexpr int kC = kE + Q * 1024;   // per-cell data: 256 dwords
    static constexpr int kM = kC + 1024;       // rows of (I - W C)^-1: [2][128] complex words
    static constexpr int kB = kM + 4096;       // moments V^T z: 16 complex words
    static constexpr int kT = kB + 256;        // t, then C t: 32 complex words
    static constexpr int kD = kT + 512;        // target of the count-keeping loads: 64 dwords
    static constexpr int kBytes = kD + 256;
};

// s_waitcnt vmcnt(K): at most K of the wave's vector memory operations
// remain outstanding.
template <int K>
__device__ inline void vm_wait() {
    static_assert(K >= 0 && K < 64, "vmcnt is a 6-bit count");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(K) : "memory");
}

// The wave's LDS reads issued so far have returned (before the memory system
// may overwrite what they read); also a compiler barrier for memory accesses.
__device__ inline void lds_reads_done() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// 16 bytes (lane i's at LDS byte address lds + 16 i) or 4 bytes (at lds +
// 4 i) from each lane's address into LDS; lds is wave-uniform; SC1:
// agent-coherent, as ld_coherent.  Written as inline assembly so that the
// compiler, which cannot tell the staging areas apart, does not wait for every
// staging load before each LDS read: the body orders them itself (vm_wait).
// M0 (the LDS base) is saved and restored.
template <bool SC1>
__device__ inline void stage16(const void *src, unsigned base) {
    unsigned saved;
    if (SC1)
        asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off sc1\n\t"
                     "s_mov_b32 m0, %0"
                     : "=&s"(saved) : "v"(src), "s"(base) : "memory");
    else
        asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off\n\t"
                     "s_mov_b32 m0, %0"
                     : "=&s"(saved) : "v"(src), "s"(base) : "memory");
}
__device__ inline void stage4(const void *src, unsigned base) {
    unsigned saved;
    asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dword %1, off\n\t"
                 "s_mov_b32 m0, %0"
                 : "=&s"(saved) : "v"(src), "s"(base) : "memory");
}
// Two doubles loaded and waited for in one block (the rare boundary lanes),
// so the compiler sees no load in flight.
__device__ inline void load2_now(const double *a, const double *b, double &va, double &vb) {
    asm volatile("global_load_dwordx2 %0, %2, off\n\tglobal_load_dwordx2 %1, %3, off\n\ts_waitcnt vmcnt(0)"
                 : "=&v"(va), "=&v"(vb) : "v"(a), "v"(b) : "memory");
}

constexpr unsigned kDropped = 0x80000000u;   // buffer offset past every resource: the store is dropped
__device__ inline __amdgpu_buffer_rsrc_t buffer_of(void *base, long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, 0x00020000);
}
// Two doubles to byte offset `off` of a buffer; AUX = 16: agent-coherent (sc1).
template <int AUX>
__device__ inline void store16(__amdgpu_buffer_rsrc_t r, unsigned off, double a, double b) {
    const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
    const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
    const v4u d = {(unsigned)ua, (unsigned)(ua >> 32), (unsigned)ub, (unsigned)(ub >> 32)};
    __builtin_amdgcn_raw_buffer_store_b128(d, r, off, 0, AUX);
}

__device__ inline int ilog2(int v) { return 31 - __builtin_clz(v); }

// sum_c row[c] v[c] over the R words of a row, every word loaded before the
// first multiply-add (one LDS round trip)
template <int R>
__device__ inline cplx row_dot_r(const cplx *row, const cplx *v) {
    cplx w[R], x[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
        w[c] = row[c];
        x[c] = v[c];
    }
    cplx acc{0.0, 0.0};
#pragma unroll
    for (int c = 0; c < R; ++c) acc = cadd(acc, cmul(w[c], x[c]));
    return acc;
}

// Cross-lane sums without LDS.  Lane partners across bit B of the lane index:
// B = 5 and 4 by the permlane swaps (lanes i and i ^ 32, i and i ^ 16), B = 3
// and 2 by the DPP row mirrors (i and i ^ 15, i and i ^ 7 within rows of 16
// lanes), B = 1 and 0 by DPP quad permutations (i ^ 2, i ^ 1).  The mirrors
// flip lower bits as well, but taken from the highest bit down the flips (32,
// 16, 15, 7, 2, 1) are independent, so each level adds two disjoint partial
// sums and a lane ends with the sum over its whole group.  Every lane of the
// wave takes part.
template <int B>
struct LaneXor {
    static constexpr int kDpp = B == 3 ? 0x140 : B == 2 ? 0x141 : B == 1 ? 0x4E : 0xB1;
};
template <int B>
__device__ inline double dpp_partner(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)v, LaneXor<B>::kDpp, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), LaneXor<B>::kDpp, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// Permlane swap of (a, b): lanes whose bit B is 0 get a and the partner's a,
// the others b and the partner's b; returned as (first, second) summed.
template <int B>
__device__ inline double swap_sum(double a, double b) {
    const long long va = __double_as_longlong(a), vb = __double_as_longlong(b);
    unsigned lo0, lo1, hi0, hi1;
    if constexpr (B == 5) {
        const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)va, (unsigned)vb, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(va >> 32), (unsigned)(vb >> 32), false, false);
        lo0 = lo[0]; lo1 = lo[1]; hi0 = hi[0]; hi1 = hi[1];
    } else {
        const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)va, (unsigned)vb, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(va >> 32), (unsigned)(vb >> 32), false, false);
        lo0 = lo[0]; lo1 = lo[1]; hi0 = hi[0]; hi1 = hi[1];
    }
    return __hiloint2double((int)hi0, (int)lo0) + __hiloint2double((int)hi1, (int)lo1);
}
// One reduce-scatter level across bit B: a lane whose bit B is 0 keeps a plus
// the partner's a, the other keeps b plus the partner's b.
template <int B>
__device__ inline double rs_level(double a, double b, bool bit) {
    if constexpr (B >= 4) {
        return swap_sum<B>(a, b);
    } else {
        const double send = bit ? a : b, keep = bit ? b : a;
        return keep + dpp_partner<B>(send);
    }
}
// One full level across bit B: x plus the partner's x.
template <int B>
__device__ inline double full_level(double x) {
    if constexpr (B >= 4) return swap_sum<B>(x, x);
    else return x + dpp_partner<B>(x);
}
// Sums over each group of 2^LGN consecutive lanes of the two complex values
// m[0], m[1] of every lane.  Two reduce-scatter levels over the group's two
// highest lane bits, then full levels over the rest: the lane whose bits
// LGN-1, LGN-2 are (h, p) holds part p (0: real, 1: imaginary) of the group
// sum of m[h].
template <int LGN>
__device__ inline double group_sum2c(const cplx m[2], int lane) {
    const bool b1 = (lane >> (LGN - 1)) & 1, b2 = (lane >> (LGN - 2)) & 1;
    const double re = rs_level<LGN - 1>(m[0].re, m[1].re, b1);
    const double im = rs_level<LGN - 1>(m[0].im, m[1].im, b1);
    double x = rs_level<LGN - 2>(re, im, b2);
    if constexpr (LGN >= 6) x = full_level<3>(x);
    if constexpr (LGN >= 5) x = full_level<2>(x);
    if constexpr (LGN >= 4) x = full_level<1>(x);
    return full_level<0>(x);
}
__device__ inline double group_sum2c(const cplx m[2], int lane, int lgN) {
    switch (lgN) {
        case 3: return group_sum2c<3>(m, lane);
        case 4: return group_sum2c<4>(m, lane);
        case 5: return group_sum2c<5>(m, lane);
        default: return group_sum2c<6>(m, lane);
    }
}

template <int Q, int BS>
__device__ __attribute__((always_inline)) inline void wb_body_staged(const Slab &S, const StepIO &io, int ntiles,
                                                                int wg, unsigned nwg, unsigned char *lds,
                                                                double *s_tmp, int *s_flag, double *s_ivdt,
                                                                double *s_mu, double *s_w) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int J = S.J, N = S.N, G = S.G, NG = N * G, nh = N / 2, R = 2 * G;
    const WbShape sh = wb_shape(NG);
    const int lc = sh.lc, cpw = sh.cpw;
    const int cw = lane / lc, li = lane % lc;
    constexpr int W = BS / 64;
    const int cpt = W * cpw;
    const int lgN = ilog2(N), lgG = ilog2(G);
    unsigned char *A = lds + (size_t)wave * WbStage<Q>::kBytes;
    // the wave's area as an LDS byte address (wave-uniform) for the staging loads
    const unsigned a_lds = __builtin_amdgcn_readfirstlane((unsigned)(size_t)(lds_void *)A);
    const int lglc = ilog2(lc);
    const double2 *Pv = reinterpret_cast<const double2 *>(A + WbStage<Q>::kP);
    const double2 *Ev = reinterpret_cast<const double2 *>(A + WbStage<Q>::kE);
    const unsigned *Ed = reinterpret_cast<const unsigned *>(A + WbStage<Q>::kE);
    const double *Cd = reinterpret_cast<const double *>(A + WbStage<Q>::kC);
    const cplx *Mv = reinterpret_cast<const cplx *>(A + WbStage<Q>::kM);
    cplx *Zcell = reinterpret_cast<cplx *>(A + WbStage<Q>::kB) + (size_t)cw * R;
    cplx *Tcell = reinterpret_cast<cplx *>(A + WbStage<Q>::kT) + (size_t)cw * 2 * R;
    // per-cell data, one 64-dword staging load each, in doubles: q
    // [cpw][G][4] at 0, phi [cpw][G][4] at 32, Sigma_s [cpw][G][G] at 64,
    // Sigma_t [cpw][G] at 96, dx [cpw] at 112 (cpw G <= 8, cpw <= 8)
    constexpr int c_phi = 32, c_ss = 64, c_st = 96, c_dx = 112;
    // this lane's pair q (any pair of the cell for padding lanes)
    auto pair_of = [&](int q) { return li + q * lc < NG ? li + q * lc : 0; };
    const int m_words = cpw * 4 * G * G;       // 16-byte words of the wave's rows
    const int nM = (m_words + 63) >> 6;        // 1 or 2
    const int lgM = 2 + 2 * lgG;               // log2(4 G^2)
    const int tile0 = (int)(((long)ntiles * wg) / nwg);
    const int tile1 = (int)(((long)ntiles * (wg + 1)) / nwg);
    for (int g = tid; g < G; g += BS) s_ivdt[g] = 1.0 / (S.speed[g] * S.dt);
    for (int m = tid; m < N; m += BS) { s_mu[m] = S.mu[m]; s_w[m] = S.w[m]; }
    if (wg == 0 && tid == 0) S.ctl->t_begin = wall_clock64();
    __syncthreads();
    // this lane's node, weight and 1/(v dt) of each pair, fixed for the launch
    double mu_q[Q], w_q[Q], ivdt_q[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = li + q * lc < NG ? li + q * lc : 0;
        mu_q[q] = s_mu[i & (N - 1)];
        w_q[q] = li + q * lc < NG ? s_w[i & (N - 1)] : 0.0;
        ivdt_q[q] = s_ivdt[i >> lgN];
    }
    const size_t ehalf = (size_t)J * NG * 2;
    const bool rb = S.ordering == 1;
    const int nhalf = rb ? 2 : 1;
    double e_prev = __builtin_nan("");
    const int base = S.ctl->base;
    const cplx *Wb = reinterpret_cast<const cplx *>(S.wb);
    // flags the tile loop tests, held in registers for the launch (a reload of
    // a scalar field waits for every LDS read in flight)
    int periodic = __builtin_amdgcn_readfirstlane(S.periodic);
    int has_q = __builtin_amdgcn_readfirstlane(io.q != nullptr ? 1 : 0);
    asm volatile("" : "+s"(periodic), "+s"(has_q));
    for (int l = 0;; ++l) {
        const int cur = (base + l) & 1;
        const double *psi_in = S.psi[cur];
        const double *phi_in = S.phi[cur];
        double *e_out = S.edge + (size_t)(l & 1) * ehalf;
        const double *e_in = S.edge + (size_t)((l + 1) & 1) * ehalf;
        const __amdgpu_buffer_rsrc_t r_edge = buffer_of(e_out, (long)ehalf * 8);
        const __amdgpu_buffer_rsrc_t r_phi = buffer_of(S.phi[cur ^ 1], (long)J * G * 32);
        const __amdgpu_buffer_rsrc_t r_psi = buffer_of(S.psi[cur ^ 1], (long)J * NG * 32);
        const double *qsrc = io.q ? io.q : phi_in;   // any [J][G][4] array when there is no source
        double dsq = 0.0;
        bool fin = false;
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1 && !fin) break;
            for (int half = 0; half < nhalf; ++half) {
                const bool from_iterate = l == 0 && half == 0;
                const double *edges = half == 1 ? e_out : e_in;
                auto cell_of = [&](int tile, int c) {
                    const int cc = tile * cpt + wave * cpw + c;
                    return rb ? 2 * cc + half : cc;
                };
                // stage psi_{k-1/2}, the upstream corners and the per-cell data of a tile
                auto stage_inputs = [&](int tile) {
                    // lane-dependent offsets recomputed here rather than kept
                    // live across the tile loop (register pressure)
                    int ln = lane;
                    asm volatile("" : "+v"(ln));
                    const int lcw = ln >> lglc, lli = ln & (lc - 1);
                    const int jc = cell_of(tile, lcw);
                    const int jj = jc < J ? jc : J - 1;
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const int i = lli + q * lc < NG ? lli + q * lc : 0;
                        const int row = jj * NG + i;   // (j, g, m) with i = g N + m; J NG < 2^26
                        stage16<false>(S.psi_prev + (size_t)row * 2, a_lds + WbStage<Q>::kP + q * 1024);
                        const bool right = (i & (N - 1)) >= nh;
                        int up = row;   // no upstream cell: any address in the slab
                        if (right) {
                            if (jj > 0) up = row - NG;
                            else if (periodic) up = row + (J - 1) * NG;
                        } else {
                            if (jj < J - 1) up = row + NG;
                            else if (periodic) up = row - (J - 1) * NG;
                        }
                        if (!from_iterate) {
                            stage16<true>(edges + (size_t)up * 2, a_lds + WbStage<Q>::kE + q * 1024);
                        } else {   // the corner of the first iterate: dwords of psi[up][c], psi[up][c + 2]
                            const unsigned *pc = reinterpret_cast<const unsigned *>(psi_in + (size_t)up * 4 + (right ? 1 : 0));
                            const unsigned e = a_lds + WbStage<Q>::kE + q * 1024;
                            stage4(pc, e);
                            stage4(pc + 1, e + 256);
                            stage4(pc + 4, e + 512);
                            stage4(pc + 5, e + 768);
                        }
                    }
                    auto clampj = [&](int c) {
                        const int jx = cell_of(tile, c);
                        return jx < J ? jx : J - 1;
                    };
                    const unsigned C = a_lds + WbStage<Q>::kC;
                    // this lane's dword of each per-cell load: (cell of the
                    // wave, dword in the cell's record)
                    const int cq = ln >> (3 + lgG), oq = ln & (8 * G - 1);
                    const int cs = ln >> (1 + 2 * lgG), os = ln & (2 * G * G - 1);
                    const bool dxl = ln >= 32;
                    const int ct = dxl ? (ln & 31) >> 1 : (ln & 31) >> (1 + lgG);
                    const int ot = dxl ? ln & 1 : ln & (2 * G - 1);
                    stage4(reinterpret_cast<const unsigned *>(qsrc) + clampj(cq) * 8 * G + oq, C);
                    stage4(reinterpret_cast<const unsigned *>(phi_in) + clampj(cq) * 8 * G + oq, C + 256);
                    stage4(reinterpret_cast<const unsigned *>(S.sigma_s) + clampj(cs) * 2 * G * G + os, C + 512);
                    const int jt = clampj(ct);
                    const unsigned *pt = dxl ? reinterpret_cast<const unsigned *>(S.dx) + jt * 2 + ot
                                             : reinterpret_cast<const unsigned *>(S.sigma_t) + jt * 2 * G + ot;
                    stage4(pt, C + 768);
                };
                // stage the rows of (I - W C)^-1 of a tile's cells, into row
                // buffer tile & 1
                auto stage_rows = [&](int tile) {
                    for (int k = 0; k < nM; ++k) {
                        const int d = k * 64 + lane;
                        const cplx *src = Wb;
                        if (d < m_words) {
                            const int j = cell_of(tile, d >> lgM);
                            src = Wb + (size_t)(j < J ? j : J - 1) * 2 * R * R + (d & ((1 << lgM) - 1));
                        }
                        stage16<false>(src, a_lds + WbStage<Q>::kM + (tile & 1) * 2048 + k * 1024);
                    }
                };
                if (tile0 < tile1) {
                    stage_rows(tile0);
                    stage_inputs(tile0);
#pragma unroll
                    for (int k = 0; k < 1 + Q; ++k) stage4(S.dx, a_lds + WbStage<Q>::kD);
                }
                for (int tile = tile0; tile < tile1; ++tile) {
                    const bool more = tile + 1 < tile1;
                    const int j = cell_of(tile, cw);
                    const bool cell = j < J;
                    // (1) the staged rows and inputs of this tile have landed:
                    //     after them came at least 1 + Q operations (the
                    //     previous tile's stores, or the count-keeping loads)
                    vm_wait<1 + Q>();
                    // every LDS read of the tile's inputs, before any use
                    const double dx = Cd[c_dx + cw];
                    double2 pp[Q], ev[Q], qa[Q], qb[Q];
                    double st[Q];
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const int g = pair_of(q) >> lgN;
                        pp[q] = Pv[q * 64 + lane];
                        if (!from_iterate) {
                            ev[q] = Ev[q * 64 + lane];
                        } else {
                            const unsigned *e = Ed + q * 256 + lane;
                            ev[q] = double2{__hiloint2double((int)e[64], (int)e[0]),
                                            __hiloint2double((int)e[192], (int)e[128])};
                        }
                        const double2 *qq = reinterpret_cast<const double2 *>(Cd + (cw * G + g) * 4);
                        qa[q] = qq[0];
                        qb[q] = qq[1];
                        st[q] = Cd[c_st + cw * G + g];
                    }
                    // the previous scalar flux of this lane's (g, level), for the
                    // norm, and its row of Sigma_s (lanes li < R; the others read
                    // in-range words and drop them)
                    const int lr = li < R ? li : 0;
                    const double2 fp = *reinterpret_cast<const double2 *>(Cd + c_phi + cw * 4 * G + 2 * lr);
                    const double *ss = Cd + c_ss + (cw * G + (lr >> 1)) * G;
                    double ssr[4];
#pragma unroll
                    for (int gp = 0; gp < 4; ++gp) {
                        const double v = ss[gp < G ? gp : 0];
                        ssr[gp] = li < R && gp < G ? v : 0.0;
                    }
                    const double2 fprev = li < R && pass == 0 ? fp : double2{0.0, 0.0};
                    // the slab's boundary: the incident flux, or vacuum (before
                    // the restaging, whose loads the wait here would include)
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const int g = pair_of(q) >> lgN, m = pair_of(q) & (N - 1);
                        const bool up_in = m >= nh ? (j > 0 || periodic) : (j < J - 1 || periodic);
                        if (!up_in) {
                            const double *inc = m >= nh ? io.inc_l : io.inc_r;
                            const int mi = m >= nh ? m - nh : m;
                            double ek = 0.0, eh = 0.0;
                            if (cell && li + q * lc < NG && inc)
                                load2_now(inc + (size_t)g * nh + mi, inc + ((size_t)G + g) * nh + mi, ek, eh);
                            ev[q] = double2{ek, eh};
                        }
                    }
                    lds_reads_done();
                    // (2) the staged inputs are consumed, and the rows of the
                    //     previous tile: stage the next tile's
                    if (more) {
                        stage_rows(tile + 1);
                        stage_inputs(tile + 1);
                    }
                    cplx z[Q][2], e2[Q], e3[Q];
                    cplx mom[Q][2];
                    const double q4 = has_q ? 0.25 * dx : 0.0;   // no source: the staged words are unused
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const int m = pair_of(q) & (N - 1);
                        const double mu = mu_q[q];
                        const double ek = ev[q].x, eh = ev[q].y;
                        const double ivdt = ivdt_q[q];
                        const double ht = 0.5 * dx * ivdt;
                        double b0 = ht * pp[q].x + q4 * qa[q].x, b1 = ht * pp[q].y + q4 * qa[q].y;
                        double b2 = q4 * qb[q].x, b3 = q4 * qb[q].y;
                        if (m >= nh) {
                            b0 += mu * ek;
                            b2 += mu * eh;
                        } else {
                            b1 -= mu * ek;
                            b3 -= mu * eh;
                        }
                        corner_inverse_nr(mu, dx * st[q], dx * ivdt, e2[q], e3[q]);
                        corner_apply(e2[q], e3[q], cplx{b0, -b1}, cplx{b2, -b3}, z[q][0], z[q][1]);
                        const double w = cell ? w_q[q] : 0.0;
                        mom[q][0] = cscale(w, z[q][0]);
                        mom[q][1] = cscale(w, z[q][1]);
                    }
                    // (3) moments: sums over the N lanes of each group across
                    //     lanes (a group's lanes are N consecutive lanes of the
                    //     wave, so lane bits below log2 N are bits of m); four
                    //     lanes of a group hold one real part each
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const double v = group_sum2c(mom[q], lane, lgN);
                        const int i = li + q * lc, m = i & (N - 1);
                        if (cell && i < NG && (m & ((N >> 2) - 1)) == 0) {
                            const int g = i >> lgN, h = (m >> (lgN - 1)) & 1, part = (m >> (lgN - 2)) & 1;
                            reinterpret_cast<double *>(Zcell)[(2 * g + h) * 2 + part] = v;
                        }
                    }
                    wave_sync();
                    // (4) t = (I - W C)^-1 V^T z from the staged rows
                    //     (a lane pair per row, each lane half of its words; the
                    //     halves summed across the pair)
                    {
                        cplx tp{0.0, 0.0};
                        if (cell && li < 2 * R) {
                            const int hw = (li & 1) * G;   // R / 2 = G words per lane
                            const cplx *row =
                                Mv + ((size_t)(tile & 1) << 7) + ((size_t)cw << lgM) + (size_t)(li >> 1) * R + hw;
                            tp = G == 4 ? row_dot_r<4>(row, Zcell + hw)
                                        : G == 2 ? row_dot_r<2>(row, Zcell + hw) : row_dot_r<1>(row, Zcell + hw);
                        }
                        tp.re += dpp_partner<0>(tp.re);
                        tp.im += dpp_partner<0>(tp.im);
                        if (cell && li < 2 * R && (li & 1) == 0) Tcell[li >> 1] = tp;
                    }
                    wave_sync();
                    // (5) C t = (dx/4) sum_g' Sigma_s[g][g'] t_g' on each level;
                    //     the scalar flux is t itself
                    unsigned phi_off = kDropped;
                    double n0 = 0.0, n1 = 0.0;
                    if (cell && li < R) {
                        const int g = li >> 1, kk = li & 1;
                        cplx ct{0.0, 0.0};
#pragma unroll
                        for (int gp = 0; gp < 4; ++gp)   // ssr[gp] = 0 for gp >= G
                            ct = cadd(ct, cscale(ssr[gp], Tcell[(gp < G ? 2 * gp : 0) + kk]));
                        const cplx t = Tcell[li];
                        Tcell[R + li] = cscale(0.25 * dx, ct);
                        n0 = t.re;
                        n1 = -t.im;
                        if (pass == 0) {
                            phi_off = (unsigned)(((j * G + g) * 4 + 2 * kk) * 8);
                            dsq += (n0 - fprev.x) * (n0 - fprev.x) + (n1 - fprev.y) * (n1 - fprev.y);
                        }
                    }
                    if (pass == 0) store16<0>(r_phi, phi_off, n0, n1);
                    wave_sync();
                    // (6) x = z + L_c^-1 (C t)_g; the outgoing corners (the
                    //     whole iterate after a stop)
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const bool act = cell && li + q * lc < NG;
                        const int g = pair_of(q) >> lgN, m = pair_of(q) & (N - 1);
                        cplx sk, sh_;
                        corner_apply(e2[q], e3[q], Tcell[R + 2 * g], Tcell[R + 2 * g + 1], sk, sh_);
                        const cplx xk = cadd(z[q][0], sk), xh = cadd(z[q][1], sh_);
                        const unsigned row = (unsigned)(j * NG + pair_of(q));
                        if (pass == 1) {
                            const unsigned o = act ? row * 32 : kDropped;
                            store16<0>(r_psi, o, xk.re, -xk.im);
                            store16<0>(r_psi, act ? o + 16 : kDropped, xh.re, -xh.im);
                        } else {
                            // the right corner travels downstream (mu > 0), else the left
                            const unsigned o = act ? row * 16 : kDropped;
                            const bool right = m >= nh;
                            store16<16>(r_edge, o, right ? -xk.im : xk.re, right ? -xh.im : xh.re);
                        }
                    }
                    wave_sync();   // T is rewritten by the next tile
                }
                // red-black: the odd cells wait for every even cell's new edges
                if (pass == 0 && rb && half == 0) {
                    double unused = 0.0;
                    if (!grid_sync_coherent<BS>(S, wg, nwg, 2 * l, 0.0, s_flag, s_tmp, &unused)) return;
                }
            }
            if (pass == 1) break;
            const double wg_sum = block_sum_t<BS>(dsq, s_tmp);   // valid in thread 0
            double tot = 0.0;
            if (!grid_sync_coherent<BS>(S, wg, nwg, rb ? 2 * l + 1 : l, wg_sum, s_flag, s_tmp, &tot)) return;
            fin = wb_decide(S, wg, l, tot, e_prev);
        }
        if (fin) return;
    }
}

// Waves per SIMD asked of the compiler: four for one pair per lane, three
// for two (the register budgets 128 and 168 the bodies fit without spills).
template <int Q, int BS, bool STAGED>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(Q == 1 ? 4 : 3))) void k_oci_wb(Slab S, StepIO io,
                                                                                                int ntiles) {
    __shared__ double s_tmp[BS / 64 + 1];
    __shared__ int s_flag[4];
    __shared__ double s_ivdt[kWbMaxG];
    __shared__ double s_mu[kWbMaxN], s_w[kWbMaxN];
    if constexpr (STAGED) {
        __shared__ __align__(16) unsigned char s_lds[(BS / 64) * WbStage<Q>::kBytes];
        wb_body_staged<Q, BS>(S, io, ntiles, blockIdx.x, gridDim.x, s_lds, s_tmp, s_flag, s_ivdt, s_mu, s_w);
    } else {
        __shared__ __align__(16) cplx s_lds[(BS / 64) * (WbLds<Q>::kA + WbLds<Q>::kB)];
        wb_body<Q, BS>(S, io, ntiles, blockIdx.x, gridDim.x, s_lds, s_tmp, s_flag, s_ivdt, s_mu, s_w);
    }
}

// Many slabs in one persistent launch: slab k owns the workgroups
// [wg0, wg0 + nwg) and runs the structured body on its own control block,
// barrier words and partial sums, so slabs converge independently (the
// structured counterpart of the dense batched kernel).  STAGED: every slab
// has a staged shape.
// Three waves per SIMD (168 registers; the one- and two-pair bodies share the
// kernel, at the price of a few spilled registers).
template <int BS, bool STAGED>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(3))) void k_wb_batch(
    const BatchEntry *__restrict__ tab, int nslab) {
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
    // the table is read-only for the kernel (restrict): its fields are read
    // with scalar loads wherever the body needs them, not with vector loads
    const BatchEntry &e = tab[__builtin_amdgcn_readfirstlane(s_k)];
    const Slab &S = e.S;
    const StepIO &io = e.io;
    const int ntiles = e.ntiles, nwg = e.nwg;
    const int lw = (int)blockIdx.x - e.wg0;
    if (lw < 0 || lw >= nwg) return;
    if constexpr (STAGED) {
        __shared__ __align__(16) unsigned char s_lds[(BS / 64) * WbStage<2>::kBytes];
        if (S.N * S.G > 64)
            wb_body_staged<2, BS>(S, io, ntiles, lw, nwg, s_lds, s_tmp, s_flag, s_ivdt, s_mu, s_w);
        else
            wb_body_staged<1, BS>(S, io, ntiles, lw, nwg, s_lds, s_tmp, s_flag, s_ivdt, s_mu, s_w);
    } else {
        __shared__ __align__(16) cplx s_lds[(BS / 64) * (WbLds<2>::kA + WbLds<2>::kB)];
        if (S.N * S.G > 64)
            wb_body<2, BS>(S, io, ntiles, lw, nwg, s_lds, s_tmp, s_flag, s_ivdt, s_mu, s_w);
        else
            wb_body<1, BS>(S, io, ntiles, lw, nwg, s_lds, s_tmp, s_flag, s_ivdt, s_mu, s_w);
    }
}

constexpr int kWbBlock = 256;

bool wb_staged(long J, int N, int G) { return wb_staged_shape(J, N, G); }

hipError_t wb_batch_occupancy(bool staged, int *blocks) {
    const void *f = staged ? (const void *)&k_wb_batch<kWbBlock, true> : (const void *)&k_wb_batch<kWbBlock, false>;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, f, kWbBlock, 0);
}

hipError_t launch_wb_batch(const BatchEntry *tab, int nslab, int nwg, bool staged, hipStream_t st) {
    if (staged)
        hipLaunchKernelGGL((k_wb_batch<kWbBlock, true>), dim3(nwg), dim3(kWbBlock), 0, st, tab, nslab);
    else
        hipLaunchKernelGGL((k_wb_batch<kWbBlock, false>), dim3(nwg), dim3(kWbBlock), 0, st, tab, nslab);
    return hipGetLastError();
}

int wb_cells_per_tile(int N, int G) { return (kWbBlock / 64) * wb_shape(N * G).cpw; }
int wb_block() { return kWbBlock; }

hipError_t wb_occupancy(int N, int G, bool staged, int *blocks) {
    const bool two = N * G > 64;
    const void *f = staged ? (two ? (const void *)&k_oci_wb<2, kWbBlock, true> : (const void *)&k_oci_wb<1, kWbBlock, true>)
                           : (two ? (const void *)&k_oci_wb<2, kWbBlock, false> : (const void *)&k_oci_wb<1, kWbBlock, false>);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, f, kWbBlock, 0);
}

hipError_t launch_oci_wb(const Slab &S, const StepIO &io, int nwg, int ntiles, bool staged, hipStream_t st) {
    const bool two = S.N * S.G > 64;
    if (staged && two)
        hipLaunchKernelGGL((k_oci_wb<2, kWbBlock, true>), dim3(nwg), dim3(kWbBlock), 0, st, S, io, ntiles);
    else if (staged)
        hipLaunchKernelGGL((k_oci_wb<1, kWbBlock, true>), dim3(nwg), dim3(kWbBlock), 0, st, S, io, ntiles);
    else if (two)
        hipLaunchKernelGGL((k_oci_wb<2, kWbBlock, false>), dim3(nwg), dim3(kWbBlock), 0, st, S, io, ntiles);
    else
        hipLaunchKernelGGL((k_oci_wb<1, kWbBlock, false>), dim3(nwg), dim3(kWbBlock), 0, st, S, io, ntiles);
    return hipGetLastError();
}

}  // namespace oci
