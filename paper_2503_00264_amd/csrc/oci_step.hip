// oci_step.hip -- the per-iteration hot path of one-cell inversion and of
// source iteration on gfx950.
//
// OCI (paper eq. oci, Algorithm 2): one persistent kernel runs every
// iteration of a time step.  Each thread owns one row i = (g*N + m)*4 + u of
// one cell system.  Per iteration it
//   1. gathers the lagged incident edge flux of its row from the neighbour
//      cell (upstream closure) and forms b_i (eq. rhs_sg);
//   2. FP64 path: stores b_i for the solve.  Refined path: forms the FP64
//      residual r_i = b_i - (A_j Psi^(l))_i matrix-free from the 4x4 corner
//      block and the scalar flux of the iterate, scales the cell's residual
//      by a power of two and rounds it to FP32;
//   3. applies the cell's inverse (one row per thread; factors streamed as
//      coalesced 16-byte words, or held in registers for the whole step when
//      they fit);
//   4. writes Psi^(l+1), the scalar flux phi = sum_m w_m psi_m (eq. si_sf) and
//      its squared change into a per-workgroup partial sum;
//   5. takes the stopping decision on the device from the per-workgroup
//      partials, summed in a fixed order by every workgroup, so it repeats
//      bit for bit: after a grid barrier (global-memory kernels), or, in the
//      workgroup-local kernel, from partials tagged with their iteration
//      while the next iteration's solve is already under way.
// SI (Appendix A, Algorithm 1): one kernel sweeps all (group, angle) chains
// cell by cell with the lagged scattering source, a second forms phi and the
// norm and takes the decision (last-block reduction).
#include "oci_device.hpp"

namespace oci {

// Stopping rule of section 2.1 / Algorithms 1-2 applied to the new change e.
__device__ inline void decide(const Slab &S, double e) {
    Ctl *c = S.ctl;
    const int iters = c->iter + 1;
    const double e_prev = c->e_prev;
    int status = OK;
    const int done = stop_rule(S, iters, e, e_prev, &status);
    c->iter = iters;
    c->e_last = e;
    c->rho = iters >= 2 ? e / e_prev : __builtin_nan("");
    c->e_prev = e;
    c->status = status;
    c->done = done;
}

// ------------------------------------------------------- step bookkeeping
// Before a step: the first iterate is where the previous step ended.
__device__ inline void begin_one(const Slab &S) {
    Ctl *c = S.ctl;
    c->base = (c->base + c->iter) & 1;
    c->iter = 0;
    c->done = 0;
    c->status = OK;
    c->err = 0;
    c->bar_count = 0;
    c->bar_gen = 0;
    S.bar[0] = 0;
    S.bar[kBarStride] = 0;
    for (int k = 0; k < S.bar_groups; ++k) S.bar[(size_t)(2 + k) * kBarStride] = 0;
    c->e_prev = __builtin_nan("");
    c->e_last = __builtin_nan("");
    c->rho = __builtin_nan("");
}
__global__ void k_begin_step(Slab S) { begin_one(S); }

// phi of the first iterate: one thread per (j, g, u), m summed in order.
__device__ inline void phi0_at(const Slab &S, size_t t, int b) {
    const int u = t & 3;
    const size_t jg = t >> 2;
    const double *p = S.psi[b] + jg * S.N * 4 + u;
    double s = 0.0;
    for (int m = 0; m < S.N; ++m) s += S.w[m] * p[m * 4];
    S.phi[b][t] = s;
}
__device__ inline void phi0_elem(const Slab &S, size_t t) { phi0_at(S, t, S.ctl->base); }
// Also empties the hand-off slots of a workgroup-local launch of nwg
// workgroups that follows (nwg = 0: none).
__global__ __launch_bounds__(kBlock) void k_phi0(Slab S, int nwg) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < (size_t)S.J * S.G * 4) phi0_elem(S, t);
    const size_t nex = (size_t)8 * nwg * S.N * S.G;
    if (t < nex) reinterpret_cast<uint64_t *>(S.exch)[t] = kSlotEmpty;
    if (t < (size_t)kPartSlots * nwg) reinterpret_cast<uint64_t *>(S.partials)[t] = kSlotEmpty;
}

__device__ inline void const_rhs_elem(const Slab &S, const StepIO &io, size_t t);

// Opens a time step of a workgroup-local kernel in one launch when no state
// broadcast is needed: the constant part of b, phi of the first iterate (the
// last iterate of the previous step, in buffer (base + iter) & 1) and the
// empty hand-off slots of a launch of nwg workgroups.  The control block is
// left as the previous step left it: the local kernels take the first
// iterate's buffer from it the same way and rewrite it when they stop, and
// k_end_step clears its error flag once reported.
__global__ __launch_bounds__(kBlock) void k_step_open(Slab S, StepIO io, int nwg) {
    const Ctl *c = S.ctl;
    const int nb = (c->base + c->iter) & 1;
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < (size_t)S.J * S.n) const_rhs_elem(S, io, t);
    if (t < (size_t)S.J * S.G * 4) phi0_at(S, t, nb);
    if (t < (size_t)8 * nwg * S.N * S.G) reinterpret_cast<uint64_t *>(S.exch)[t] = kSlotEmpty;
    if (t < (size_t)kPartSlots * nwg) reinterpret_cast<uint64_t *>(S.partials)[t] = kSlotEmpty;
}

// psi of the first iterate from the state (both time levels).
__device__ inline void broadcast_elem(const Slab &S, size_t t) {
    S.psi[S.ctl->base][t] = S.psi_prev[(t >> 2) * 2 + (t & 1)];
}
// from_flag: only when the control block's broadcast flag is set (steps
// captured in a graph learn on the device whether the state was replaced).
__global__ __launch_bounds__(kBlock) void k_broadcast_state(Slab S, int from_flag) {
    if (from_flag && !S.ctl->bcast) return;
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < (size_t)S.J * S.G * S.N * 4) broadcast_elem(S, t);
}
__global__ void k_clear_bcast(Slab S) { S.ctl->bcast = 0; }

// Checkpoints: the first iterate of the next step lives in buffer
// (base + iter) & 1 of the control block (or is psi_prev on both levels when
// the host still has to broadcast it).
__global__ __launch_bounds__(kBlock) void k_checkpoint_get(Slab S, double *iter_out, int from_state) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (size_t)S.J * S.n) return;
    const Ctl *c = S.ctl;
    iter_out[t] = from_state ? S.psi_prev[(t >> 2) * 2 + (t & 1)] : S.psi[(c->base + c->iter) & 1][t];
}
__global__ __launch_bounds__(kBlock) void k_checkpoint_set(Slab S, const double *iter_in) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (size_t)S.J * S.n) return;
    const Ctl *c = S.ctl;
    S.psi[(c->base + c->iter) & 1][t] = iter_in[t];
}
hipError_t launch_checkpoint(const Slab &S, double *out, const double *in, bool from_state, hipStream_t st) {
    const size_t tot = (size_t)S.J * S.n;
    const dim3 grid((unsigned)((tot + kBlock - 1) / kBlock));
    if (out) hipLaunchKernelGGL(k_checkpoint_get, grid, dim3(kBlock), 0, st, S, out, from_state ? 1 : 0);
    else hipLaunchKernelGGL(k_checkpoint_set, grid, dim3(kBlock), 0, st, S, in);
    return hipGetLastError();
}

// After a step: time update psi_{k-1/2} <- psi_{k+1/2} and the outputs.
// Elements: one per (j, g, m) row quad and per phi entry.
__device__ inline void end_elem(const Slab &S, const StepIO &io, size_t t) {
    const Ctl *c = S.ctl;
    const int fin = (c->base + c->iter) & 1;
    const size_t nrow = (size_t)S.J * S.G * S.N;
    if (t < nrow) {
        const double *p = S.psi[fin] + t * 4;
        S.psi_prev[t * 2 + 0] = p[2];
        S.psi_prev[t * 2 + 1] = p[3];
        if (io.psi_out) {
            io.psi_out[t * 4 + 0] = p[0];
            io.psi_out[t * 4 + 1] = p[1];
            io.psi_out[t * 4 + 2] = p[2];
            io.psi_out[t * 4 + 3] = p[3];
        }
    }
    if (t < (size_t)S.J * S.G * 4) io.phi_out[t] = S.phi[fin][t];
    if (t == 0) {
        int32_t *ip = reinterpret_cast<int32_t *>(io.info);
        double *dp = reinterpret_cast<double *>(io.info);
        ip[0] = c->iter;
        ip[1] = c->err ? -6 : c->status;
        dp[1] = c->e_last;
        dp[2] = c->rho;
        const_cast<Ctl *>(c)->err = 0;   // reported; the next step starts clean
    }
}
__device__ inline size_t end_elems(const Slab &S) {
    const size_t a = (size_t)S.J * S.G * S.N, b = (size_t)S.J * S.G * 4;
    return a > b ? a : b;
}
__global__ __launch_bounds__(kBlock) void k_end_step(Slab S, StepIO io) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < end_elems(S)) end_elem(S, io, t);
}

// -------------------------------------------------------------- OCI kernel
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 type; };
template <> struct Vec16<double> { typedef double2 type; };

__device__ inline float dot16(const float4 &a, const float4 &b) {
    return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
}
__device__ inline double dot16(const double2 &a, const double2 &b) { return a.x * b.x + a.y * b.y; }
// acc + a . b as a chain of fused multiply-adds
__device__ inline float fma_dot16(const float4 &a, const float4 &b, float acc) {
    return fmaf(a.w, b.w, fmaf(a.z, b.z, fmaf(a.y, b.y, fmaf(a.x, b.x, acc))));
}
__device__ inline double fma_dot16(const double2 &a, const double2 &b, double acc) {
    return fma(a.y, b.y, fma(a.x, b.x, acc));
}

// The streamed inverse-row product acc[r] += X[t + r TPC, :] . vec over the
// cell's tiled NP x NP block, in the same order as one word at a time, with
// B 16-byte words of every row loaded together before any is used: each
// thread keeps B x RPT loads in flight instead of waiting on each one.  Used
// by the workgroup-local kernel; in the batched kernel, which holds the
// bodies of all cell sizes, the same batching measured 45 % slower, and its
// body keeps the plain loop.
constexpr int kStreamWords = 8;
template <typename T, int NP, int RPT, int TPC, int B>
__device__ inline void stream_rows(const T *Xc, int t, const T *vec, T (&acc)[RPT]) {
    typedef typename Vec16<T>::type VT;
    constexpr int V = 16 / sizeof(T), NV = NP / V;
    constexpr int BB = (B / RPT < NV ? B / RPT : NV) > 0 ? (B / RPT < NV ? B / RPT : NV) : 1;
    static_assert(NV % BB == 0, "whole batches");
    for (int kv0 = 0; kv0 < NV; kv0 += BB) {
        VT xv[BB][RPT];
#pragma unroll
        for (int u = 0; u < BB; ++u)
#pragma unroll
            for (int r = 0; r < RPT; ++r)
                xv[u][r] = *reinterpret_cast<const VT *>(Xc + ((size_t)(kv0 + u) * NP + t + r * TPC) * V);
#pragma unroll
        for (int u = 0; u < BB; ++u) {
            const VT bv = *reinterpret_cast<const VT *>(vec + (kv0 + u) * V);
#pragma unroll
            for (int r = 0; r < RPT; ++r) acc[r] += dot16(xv[u][r], bv);
        }
    }
}

// Coefficients of row u of the 4x4 corner block L_{c,j,g,m} (eq. Aj) acting
// on (psi_kL, psi_kR, psi_hL, psi_hR) of the same (g, m).
__device__ inline void lc_row(const Slab &S, int j, int g, double mu, int u, double c[4]) {
    const double dx = S.dx[j];
    const double a = dx / (S.speed[g] * S.dt);
    const double d = 0.5 * (fabs(mu) + dx * S.sigma_t[(size_t)j * S.G + g]);
    const double h = 0.5 * mu;
    if (u == 0) { c[0] = d; c[1] = h; c[2] = 0.5 * a; c[3] = 0.0; }
    else if (u == 1) { c[0] = -h; c[1] = d; c[2] = 0.0; c[3] = 0.5 * a; }
    else if (u == 2) { c[0] = -a; c[1] = 0.0; c[2] = a + d; c[3] = h; }
    else { c[0] = 0.0; c[1] = -a; c[2] = -h; c[3] = a + d; }
}

// The persistent OCI kernel.  T = float: refined path (FP32 inverse applied
// to the power-of-two scaled FP64 residual); T = double: plain FP64 path.
// NP: padded cell size (power of two >= n); RES: each thread keeps its row of
// the inverse in registers, and the row's constants in LDS, for the whole
// step (one tile per workgroup); BS: threads per workgroup.  At most 128
// VGPRs (4 waves per SIMD).
// LDS of one workgroup of the global iteration body.  A kernel provides it as
// raw bytes, so that kernels holding several bodies (one per cell size) can
// overlay them.
template <typename T, int NP, bool RES, int BS>
struct GlobalLds {
    static constexpr bool REF = sizeof(T) == 4;
    static constexpr int RPT = NP > BS ? NP / BS : 1;
    static constexpr int CPT = BS / (NP / RPT);
    static constexpr bool CACHE = RES && REF;
    __align__(16) T vec[CPT][NP];
    double psi[REF ? CPT : 1][REF ? NP : 1];
    double wx[CPT][NP];
    double phi[REF ? CPT : 1][REF ? NP / 2 : 1];
    double coef[CACHE ? CPT : 1][CACHE ? NP : 1][4];
    double crow[CACHE ? CPT : 1][CACHE ? NP : 1];
    double scat[CACHE ? CPT : 1][CACHE ? NP / 8 * NP / 8 : 1];
    double mu[NP / 4], w[NP / 4];
    double tmp[BS / 64 + 1];
    double mx[BS / 64];
    int flag[4];
};

template <typename T, int NP, bool RES, int BS>
__device__ __attribute__((always_inline)) inline void oci_global_body(const Slab &S, const StepIO &io, int ntiles, int wg,
                                                                 unsigned nwg, unsigned char *lds_raw) {
    constexpr bool REF = sizeof(T) == 4;
    constexpr int RPT = NP > BS ? NP / BS : 1;   // rows per thread
    constexpr int TPC = NP / RPT;                 // threads per cell
    constexpr int CPT = BS / TPC;                 // cells per tile
    constexpr int V = 16 / sizeof(T);
    constexpr int NV = NP / V;
    constexpr bool CACHE = RES && REF;            // row constants cached in LDS
    typedef typename Vec16<T>::type VT;

    typedef GlobalLds<T, NP, RES, BS> Lds;
    Lds &lds = *reinterpret_cast<Lds *>(lds_raw);
    auto &s_vec = lds.vec;
    auto &s_psi = lds.psi;
    auto &s_wx = lds.wx;
    auto &s_phi = lds.phi;
    auto &s_coef = lds.coef;
    auto &s_crow = lds.crow;
    auto &s_scat = lds.scat;
    auto &s_mu = lds.mu;
    auto &s_w = lds.w;
    auto &s_tmp = lds.tmp;
    auto &s_max = lds.mx;
    auto &s_flag = lds.flag;

    const int tid = threadIdx.x;
    const int cl = tid / TPC;
    const int t = tid % TPC;
    const int J = S.J, N = S.N, G = S.G, n = S.n;
    const int tile0 = (int)(((long)ntiles * wg) / nwg);
    const int tile1 = (int)(((long)ntiles * (wg + 1)) / nwg);

    for (int m = tid; m < N; m += BS) { s_mu[m] = S.mu[m]; s_w[m] = S.w[m]; }

    const T *Xall = reinterpret_cast<const T *>(S.X);
    VT xr[RES ? NV : 1];
    if constexpr (RES) {
        const int j = tile0 * CPT + cl;
        if (tile0 < tile1 && j < J) {
            const T *Xc = Xall + (size_t)j * NP * NP;
#pragma unroll
            for (int kv = 0; kv < NV; ++kv) xr[kv] = *reinterpret_cast<const VT *>(Xc + ((size_t)kv * NP + t) * V);
        }
    }
    __syncthreads();
    if constexpr (CACHE) {
        const int j = tile0 * CPT + cl;
        const int i = t;
        if (tile0 < tile1 && j < J && i < n) {
            const int g = i / (4 * N), m = (i >> 2) % N, u = i & 3;
            lc_row(S, j, g, s_mu[m], u, s_coef[cl][i]);
            s_crow[cl][i] = S.crhs[(size_t)j * n + i];
        }
        if (tile0 < tile1 && j < J && t < G * G)
            s_scat[cl][t] = 0.25 * S.dx[j] * S.sigma_s[(size_t)j * G * G + t];
        __syncthreads();
    }

    double e_prev = __builtin_nan("");
    const int base = S.ctl->base;
    for (int l = 0;; ++l) {
        const int cur = (base + l) & 1;
        const double *__restrict__ psi_in = S.psi[cur];
        double *__restrict__ psi_out = S.psi[cur ^ 1];
        const double *__restrict__ phi_in = S.phi[cur];
        double *__restrict__ phi_out = S.phi[cur ^ 1];
        double wg_sum = 0.0;

        for (int tile = tile0; tile < tile1; ++tile) {
            const int j = tile * CPT + cl;
            const bool live = j < J;
            double xold[RPT];
            int expo = 0;

            // (1) b = constant part (per step) + lagged incident edge (eq. rhs_sg)
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = t + r * TPC;
                double b = 0.0;
                xold[r] = 0.0;
                if (live && i < n) {
                    const int g = i / (4 * N), m = (i >> 2) % N, u = i & 3;
                    const double mu = s_mu[m];
                    xold[r] = psi_in[(size_t)j * n + i];
                    b = CACHE ? s_crow[cl][i] : S.crhs[(size_t)j * n + i];
                    if (mu > 0.0 && !(u & 1)) {
                        const double e = j > 0 ? psi_in[(((size_t)(j - 1) * G + g) * N + m) * 4 + u + 1]
                                               : (io.inc_l ? io.inc_l[((size_t)(u >> 1) * G + g) * (N / 2) + (m - N / 2)] : 0.0);
                        b += mu * e;
                    } else if (mu < 0.0 && (u & 1)) {
                        const double e = j < J - 1 ? psi_in[(((size_t)(j + 1) * G + g) * N + m) * 4 + u - 1]
                                                   : (io.inc_r ? io.inc_r[((size_t)(u >> 1) * G + g) * (N / 2) + m] : 0.0);
                        b -= mu * e;
                    }
                }
                if constexpr (REF) {
                    s_psi[cl][i] = xold[r];
                    s_wx[cl][i] = b;          // b parked until the residual is formed
                } else {
                    s_vec[cl][i] = b;
                }
            }
            if constexpr (REF) {
                if (live && t < 4 * G) s_phi[cl][t] = phi_in[(size_t)j * 4 * G + t];
                __syncthreads();
                // (2) FP64 residual r = b - A_j Psi^(l), matrix-free:
                //     L_c rows on the corner quad, scattering through phi
                double rr[RPT];
                double mx = 0.0;
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int i = t + r * TPC;
                    double res = 0.0;
                    if (live && i < n) {
                        const int g = i / (4 * N), u = i & 3;
                        double cf[4];
                        if constexpr (CACHE) {
                            cf[0] = s_coef[cl][i][0]; cf[1] = s_coef[cl][i][1];
                            cf[2] = s_coef[cl][i][2]; cf[3] = s_coef[cl][i][3];
                        } else {
                            lc_row(S, j, g, s_mu[(i >> 2) % N], u, cf);
                        }
                        const double *p = &s_psi[cl][i & ~3];
                        const double lp = cf[0] * p[0] + cf[1] * p[1] + cf[2] * p[2] + cf[3] * p[3];
                        double sc = 0.0;
                        if constexpr (CACHE) {
                            for (int gp = 0; gp < G; ++gp) sc += s_scat[cl][g * G + gp] * s_phi[cl][gp * 4 + u];
                        } else {
                            const double *ss = S.sigma_s + ((size_t)j * G + g) * G;
                            for (int gp = 0; gp < G; ++gp) sc += ss[gp] * s_phi[cl][gp * 4 + u];
                            sc *= 0.25 * S.dx[j];
                        }
                        res = s_wx[cl][i] - lp + sc;
                    }
                    rr[r] = res;
                    mx = fmax(mx, fabs(res));
                }
                // cell maximum -> power-of-two scale
                if constexpr (TPC <= 64) {
#pragma unroll
                    for (int off = TPC / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
                } else {
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
                    if ((tid & 63) == 0) s_max[tid >> 6] = mx;
                    __syncthreads();
                    mx = 0.0;
                    for (int w = cl * (TPC / 64); w < (cl + 1) * (TPC / 64); ++w) mx = fmax(mx, s_max[w]);
                }
                if (mx > 0.0 && isfinite(mx)) frexp(mx, &expo);
#pragma unroll
                for (int r = 0; r < RPT; ++r) s_vec[cl][t + r * TPC] = (T)ldexp(rr[r], -expo);
            }
            __syncthreads();

            // (3) apply the inverse, one row per thread
            T acc[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) acc[r] = T(0);
            if (live) {
                if constexpr (RES) {
#pragma unroll
                    for (int kv = 0; kv < NV; ++kv) {
                        const VT bv = *reinterpret_cast<const VT *>(&s_vec[cl][kv * V]);
                        acc[0] += dot16(xr[kv], bv);
                    }
                } else {
                    const T *Xc = Xall + (size_t)j * NP * NP;
#pragma unroll 8
                    for (int kv = 0; kv < NV; ++kv) {
                        const VT bv = *reinterpret_cast<const VT *>(&s_vec[cl][kv * V]);
#pragma unroll
                        for (int r = 0; r < RPT; ++r) {
                            const VT xv = *reinterpret_cast<const VT *>(Xc + ((size_t)kv * NP + t + r * TPC) * V);
                            acc[r] += dot16(xv, bv);
                        }
                    }
                }
            }

            // (4) new iterate, scalar flux and its change
            double dsq = 0.0;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = t + r * TPC;
                double x = REF ? xold[r] + ldexp((double)acc[r], expo) : (double)acc[r];
                if (live && i < n) {
                    psi_out[(size_t)j * n + i] = x;
                    if (S.norm == 1) dsq += (x - xold[r]) * (x - xold[r]);
                } else {
                    x = 0.0;
                }
                s_wx[cl][i] = (i < n ? s_w[(i >> 2) % N] : 0.0) * x;
            }
            __syncthreads();
            if (live && t < 4 * G) {
                const int g = t >> 2, u = t & 3;
                double f = 0.0;
                for (int m = 0; m < N; ++m) f += s_wx[cl][(g * N + m) * 4 + u];
                const size_t o = (size_t)j * 4 * G + t;
                const double f0 = phi_in[o];
                phi_out[o] = f;
                if (S.norm == 0) dsq += (f - f0) * (f - f0);
            }
            const double part = block_sum_t<BS>(dsq, s_tmp);
            if (tid == 0) wg_sum += part;
        }

        // (5) grid barrier + reduction; every workgroup decides identically
        double tot = 0.0;
        const bool ok = grid_sync_sum<BS>(S, wg, nwg, l, wg_sum, s_flag, s_tmp, &tot);
        if (!ok) break;
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
            break;
        }
    }
}

template <typename T, int NP, bool RES, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4)))
void k_oci_step(Slab S, StepIO io, int ntiles) {
    __shared__ __align__(16) unsigned char s_lds[sizeof(GlobalLds<T, NP, RES, BS>)];
    oci_global_body<T, NP, RES, BS>(S, io, ntiles, blockIdx.x, gridDim.x, s_lds);
}

// Relaxed agent-scope accesses: coherent across the XCDs without any L2
// writeback or invalidate.  Only the data that crosses workgroups inside a
// launch (boundary edges and partial sums) goes through them.
__device__ inline uint64_t ld_bits(const uint64_t *p) {
    return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_bits(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Edge hand-off between neighbouring workgroups: the producer stores each
// 32-bit half of the value beside the tag of the iteration that will read it,
// as two single-copy-atomic 64-bit words; the consumer waits until both words
// carry its own iteration.  The slots are double-buffered by iteration parity,
// so a stale word carries the tag of two iterations earlier; no slot is ever
// reset inside a launch.  The wait is bounded: on expiry *bad is raised and
// the value is NaN.
__device__ inline void put_edge(uint64_t *slot, double v, int tag) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t t = (uint64_t)(uint32_t)tag << 32;
    st_bits(slot, t | (b & 0xFFFFFFFFull));
    st_bits(slot + 1, t | (b >> 32));
}
__device__ inline double take_edge(const uint64_t *slot, int tag, int *bad) {
    const uint32_t want = (uint32_t)tag;
    uint64_t lo = ld_bits(slot), hi = ld_bits(slot + 1);
    long spins = 0;
#pragma clang loop unroll(disable)
    while ((uint32_t)(lo >> 32) != want || (uint32_t)(hi >> 32) != want) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) { *bad = 1; return __builtin_nan(""); }
        lo = ld_bits(slot);
        hi = ld_bits(slot + 1);
    }
    return __longlong_as_double((long long)((hi << 32) | (lo & 0xFFFFFFFFull)));
}

// Partial sums carry the iteration that produced them in their lowest
// mantissa bits, so a reader recognises the value it waits for by its tag
// alone (no counter).  Clearing those bits on the way out keeps an exact zero
// exactly zero.
constexpr uint64_t kTagMask = (1ull << kPartTagBits) - 1;
__device__ inline uint64_t part_encode(double v, int l) {
    const uint64_t b = (uint64_t)__double_as_longlong(fabs(v));
    return (b & ~kTagMask) | ((uint64_t)l & kTagMask);
}
__device__ inline bool part_ready(uint64_t b, int l) {
    return (b >> 63) == 0 && (b & kTagMask) == ((uint64_t)l & kTagMask);
}
__device__ inline double part_value(uint64_t b) { return __longlong_as_double((long long)(b & ~kTagMask)); }

// Cross-lane moves inside a row of 16 lanes (DPP: no LDS round trip), for the
// wave-level reductions of the workgroup-local kernel.  Called with every lane
// of the wave active.
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <- 7 - i within 8
constexpr int kDppMirror = 0x140;      // lane i <- 15 - i within 16
constexpr int kDppRor4 = 0x124;        // rotate the row by 4 lanes
constexpr int kDppRor8 = 0x128;        // rotate the row by 8 lanes
// Every lane reads a lane of its own row, so no lane keeps an old value: a lane
// whose source is disabled reads zero (bound_ctrl), and the destination needs
// no initialisation.
template <int CTRL>
__device__ inline int dpp_i32(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const int lo = dpp_i32<CTRL>(__double2loint(v));
    const int hi = dpp_i32<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ inline double readlane_f64(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}
// Across rows: lanes i and i ^ 16 (B = 4) or i and i ^ 32 (B = 5) exchange
// their values by a permlane swap (one instruction per dword, no LDS).  The
// swap of (v, v) leaves the lower-half lanes their own value in the first
// result and the partner's in the second, the upper-half lanes the reverse;
// either way a lane holds both values.
template <int B>
__device__ inline double xor_add_f64(double v) {
    static_assert(B == 4 || B == 5, "row pairs or wave halves");
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    unsigned l0, l1, h0, h1;
    if constexpr (B == 5) {
        const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        l0 = a[0]; l1 = a[1]; h0 = b[0]; h1 = b[1];
    } else {
        const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        l0 = a[0]; l1 = a[1]; h0 = b[0]; h1 = b[1];
    }
    return __hiloint2double((int)h0, (int)l0) + __hiloint2double((int)h1, (int)l1);
}
template <int B>
__device__ inline int xor_max_i32(int v) {
    static_assert(B == 4 || B == 5, "row pairs or wave halves");
    if constexpr (B == 5) {
        const auto a = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
        return max((int)a[0], (int)a[1]);
    } else {
        const auto a = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
        return max((int)a[0], (int)a[1]);
    }
}
// Sum over the 64 lanes of the wave in a fixed order, (r0 + r1) + (r2 + r3)
// over the four row sums; every lane gets the same value (each step adds two
// equal-order partial sums, and floating-point addition is commutative).
__device__ inline double wave_sum_dpp(double v) {
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    v += dpp_f64<kDppHalfMirror>(v);
    v += dpp_f64<kDppMirror>(v);
    return xor_add_f64<5>(xor_add_f64<4>(v));
}
// Maximum over aligned groups of TPC lanes (TPC = 8 .. 64).
template <int TPC>
__device__ inline int seg_max_i32(int v) {
    v = max(v, dpp_i32<kDppXor1>(v));
    v = max(v, dpp_i32<kDppXor2>(v));
    v = max(v, dpp_i32<kDppHalfMirror>(v));
    if constexpr (TPC >= 16) v = max(v, dpp_i32<kDppMirror>(v));
    if constexpr (TPC >= 32) v = xor_max_i32<4>(v);
    if constexpr (TPC == 64) v = xor_max_i32<5>(v);
    return v;
}


// Workgroup-local persistent OCI kernel with streamed inverse rows.  Each
// workgroup owns the contiguous cells [c0, c1) (one or more tiles) for the
// whole step and keeps their iterate Psi and scalar flux phi in LDS (dynamic
// shared memory: [cells][n] Psi, [cells][4G] phi, then per internal tile
// boundary a snapshot of the 2NG edge values that cross it).  Only the edges
// at the two ends of the range cross workgroups, handed to the neighbour
// through tagged slots (put_edge / take_edge); iterate 0's neighbour edges
// come from global memory (written by earlier launches).  There is no grid
// barrier: a workgroup waits only for its two neighbours' edges, and for the
// tagged partial sums it needs for the stopping decision.  An edge slot is
// written again two iterations later, and the writer cannot get there before
// the reader has taken the old value: the writer's next iteration needs the
// reader's edges, which the reader only publishes after that read.  A
// partial-sum slot (kPartSlots of them, by iteration) is written again
// kPartSlots iterations later, after its writer has taken a decision that
// needs every workgroup's partial of an iteration whose end follows that
// workgroup's last read of the slot.  No store has to complete before
// another is issued.  At the end the final Psi and phi are written to global
// memory.  T = float: refined path; T = double: plain FP64 path.  NP: padded
// cell size; BS: threads per workgroup.
template <typename T, int NP, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4)))
void k_oci_local(Slab S, StepIO io, int ntiles) {
    constexpr bool REF = sizeof(T) == 4;
    constexpr int RPT = NP > BS ? NP / BS : 1;
    constexpr int TPC = NP / RPT;
    constexpr int CPT = BS / TPC;
    constexpr int V = 16 / sizeof(T);
    constexpr int NV = NP / V;
    constexpr int PV = 4;               // partial sums per lane loaded ahead of the decision
    constexpr bool WAVE_CELL = TPC <= 64;   // a cell's rows lie in one wave (then RPT = 1)
    static_assert(BS <= 1024, "wave sums are added within one row of 16 lanes");
    typedef typename Vec16<T>::type VT;

    extern __shared__ __align__(16) double s_dyn[];
    __shared__ __align__(16) T s_vec[CPT][NP];
    __shared__ double s_w[NP / 4];
    __shared__ double s_max[BS / 64];
    __shared__ double s_part[2][BS / 64];   // per-wave partial sums, by iteration parity
    __shared__ double s_dec[2][4];          // decision (done, status, e, rho), by iteration parity

    const int tid = threadIdx.x;
    const int dec_wave = (BS / 64) / 2;   // the wave that takes the stopping decision
    const int J = S.J, N = S.N, G = S.G, n = S.n, nh = S.N / 2, NG = S.N * S.G;
    const unsigned nwg = gridDim.x;
    const int wg = blockIdx.x;
    const int tile0 = (int)(((long)ntiles * wg) / nwg);
    const int tile1 = (int)(((long)ntiles * (wg + 1)) / nwg);
    const int ntw = tile1 - tile0;
    const int c0 = tile0 * CPT;
    const int c1 = min(tile1 * CPT, J);
    const int ncell = ntw * CPT;
    double *L_psi = s_dyn;                                   // [ncell][n]
    double *L_phi = L_psi + (size_t)ncell * n;               // [ncell][4G]
    double *L_snap = L_phi + (size_t)ncell * 4 * G;          // [ntw - 1][2][NG]: R-going, L-going
    double *L_wx = L_snap + (size_t)(ntw > 1 ? ntw - 1 : 0) * 2 * NG;   // [CPT][NP] w_m psi, only without tree_phi
    // exchange buffer [2 parity][nwg][2 side][2 lev][G][nh] slots of two
    // words; side 0: my first cell's L corners of mu<0 angles, side 1: my
    // last cell's R corners of mu>0
    uint64_t *exch_bits = reinterpret_cast<uint64_t *>(S.exch);
    auto exq = [&](int par, int w, int side, int lev, int g, int mm) -> uint64_t * {
        return exch_bits + 2 * ((((size_t)par * nwg + w) * 2 + side) * NG + ((size_t)lev * G + g) * nh + mm);
    };

    for (int m = tid; m < N; m += BS) s_w[m] = S.w[m];

    const T *Xall = reinterpret_cast<const T *>(S.X);
    // the iterate and its scalar flux into LDS
    // the first iterate is the last one of the previous step (a step opened
    // by k_step_open leaves the control block as that step left it)
    const int base = (S.ctl->base + S.ctl->iter) & 1;
    const double *__restrict__ psi_g = S.psi[base];   // the iterate in global memory: only read at l = 0
    {
        const double *pin = psi_g + (size_t)c0 * n;
        const int tot = (c1 - c0) * n;
        for (int k = tid; k < tot; k += BS) L_psi[k] = pin[k];
        const double *fin = S.phi[base] + (size_t)c0 * 4 * G;
        const int totf = (c1 - c0) * 4 * G;
        for (int k = tid; k < totf; k += BS) L_phi[k] = fin[k];
    }
    __syncthreads();

    // phi by lane moves within the wave: the N angles of a (g, u) pair lie in
    // 4N consecutive rows, a power of two that divides 64, so they share a
    // wave even when the cell spans several
    const bool tree_phi = RPT == 1 && (N & (N - 1)) == 0 && N <= 16;
    uint64_t *part_bits = reinterpret_cast<uint64_t *>(S.partials);
    double e_prev = __builtin_nan("");
    uint64_t pv[PV];   // the decision wave's partial sums, loaded at the end of the previous iteration
#pragma unroll
    for (int r = 0; r < PV; ++r) pv[r] = kSlotEmpty;
    // Iteration l forms Psi^(l+1).  At its start one wave decides, while the
    // others wait for the neighbours' edges, on e_l (the partials of
    // iteration l - 1); the outcome reaches every wave through the barrier
    // that precedes the solve, before anything in LDS is overwritten, so LDS
    // still holds the final iterate Psi^(l) when the decision stops the step.
    for (int l = 0;; ++l) {
        // lane indices are re-derived every iteration from an opaque copy, so
        // the compiler does not keep per-lane addresses live across the loop
        int tid_o = tid;
        asm volatile("" : "+v"(tid_o));
        const int cl = tid_o / TPC;
        const int t = tid_o % TPC;
        const int lp = l - 1;                            // iteration whose partials are decided on
        const uint64_t *part_prev = part_bits + (size_t)(lp & (kPartSlots - 1)) * nwg;
        const int par = (l + 1) & 1;                     // exchange parity this iteration publishes
        const bool dec = (tid_o >> 6) == dec_wave && lp >= 0;   // this wave decides (wave-uniform)
        double dsq_acc = 0.0;
        int bad = 0;

        // Stopping rule (section 2.1) on e_(lp+1), the change made by
        // iteration lp, in the decision wave: every workgroup's decision wave
        // sums the same tagged partials in the same order (lane k holds k,
        // k + 64, ...) and takes the same decision, left in s_dec.
        if (dec) {
            const int lane = tid_o & 63;
            auto wait_part = [&](uint64_t x, int k) -> double {
                long spins = 0;
#pragma clang loop unroll(disable)
                while (!part_ready(x, lp)) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > kSpinLimit) { bad = 1; break; }
                    x = ld_bits(part_prev + k);
                }
                return part_value(x);
            };
            double v = 0.0;
#pragma unroll
            for (int r = 0; r < PV; ++r)
                if (lane + 64 * r < (int)nwg) v += wait_part(pv[r], lane + 64 * r);
            for (int k = lane + 64 * PV; k < (int)nwg; k += 64) v += wait_part(ld_bits(part_prev + k), k);
            if (bad) {
                __hip_atomic_store(&S.ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                v = __builtin_nan("");
            }
            const double tot = wave_sum_dpp(v);
            const int iters = lp + 1;
            const double e = sqrt(tot);
            const double rho = iters >= 2 ? e / e_prev : __builtin_nan("");
            int done = 0, status = OK;
            if (!isfinite(e)) { done = 1; status = NONFINITE; }
            else if (S.fixed_iters > 0) done = iters >= S.fixed_iters;
            else if (iters >= 2 && (e == 0.0 || e < S.tol * (1.0 - rho))) done = 1;
            else if (iters >= S.max_iters) { done = 1; status = NOT_CONVERGED; }
            e_prev = e;
            if (S.hist && iters <= S.hist_cap && wg == 0 && lane == 0) S.hist[iters - 1] = e;
            if (lane == 0) {
                s_dec[l & 1][0] = done;
                s_dec[l & 1][1] = status;
                s_dec[l & 1][2] = e;
                s_dec[l & 1][3] = rho;
            }
        }

        // edges crossing internal tile boundaries, before any tile updates
        if (ntw > 1) {
            for (int k = tid_o; k < (ntw - 1) * 2 * NG; k += BS) {
                const int tt = 1 + k / (2 * NG), r = k % (2 * NG);   // the boundary before tile tt
                const int side = r / NG, q = r % NG;           // side 0: R-going, 1: L-going
                const int lev = q / (G * nh), g = (q / nh) % G, mm = q % nh;
                const int jb = (tile0 + tt) * CPT;             // first cell of tile tt
                double v;
                if (side == 0) v = L_psi[(size_t)(jb - 1 - c0) * n + (g * N + nh + mm) * 4 + 2 * lev + 1];
                else v = L_psi[(size_t)(jb - c0) * n + (g * N + mm) * 4 + 2 * lev];
                L_snap[(size_t)(tt - 1) * 2 * NG + r] = v;
            }
            __syncthreads();
        }

        for (int tile = tile0; tile < tile1; ++tile) {
            const int tt = tile - tile0;
            const int j = tile * CPT + cl;
            const bool live = j < J;
            double *Lp = L_psi + (size_t)(j - c0) * n;          // this cell's iterate
            double *Lf = L_phi + (size_t)(j - c0) * 4 * G;
            double xold[RPT], bb[RPT];
            int expo = 0;

            // (1) b = constant part + lagged incident edge
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = t + r * TPC;
                double b = 0.0;
                xold[r] = 0.0;
                if (live && i < n) {
                    const int g = i / (4 * N), m = (i >> 2) % N, u = i & 3;
                    const double mu = S.mu[m];
                    xold[r] = Lp[i];
                    b = S.crhs[(size_t)j * n + i];
                    const int lev = u >> 1;
                    if (mu > 0.0 && !(u & 1)) {
                        double e;
                        if (j == 0)
                            e = io.inc_l ? io.inc_l[((size_t)lev * G + g) * nh + (m - nh)] : 0.0;
                        else if (j % CPT != 0)
                            e = Lp[i - n + 1];                                   // same tile
                        else if (j - 1 >= c0)
                            e = L_snap[(size_t)(tt - 1) * 2 * NG + (lev * G + g) * nh + (m - nh)];
                        else if (l == 0)
                            e = psi_g[(size_t)(j - 1) * n + i + 1];
                        else
                            e = take_edge(exq(l & 1, wg - 1, 1, lev, g, m - nh), l, &bad);
                        b += mu * e;
                    } else if (mu < 0.0 && (u & 1)) {
                        double e;
                        if (j == J - 1)
                            e = io.inc_r ? io.inc_r[((size_t)lev * G + g) * nh + m] : 0.0;
                        else if ((j + 1) % CPT != 0)
                            e = Lp[i + n - 1];                                   // same tile
                        else if (j + 1 < c1)
                            e = L_snap[(size_t)tt * 2 * NG + NG + (lev * G + g) * nh + m];
                        else if (l == 0)
                            e = psi_g[(size_t)(j + 1) * n + i - 1];
                        else
                            e = take_edge(exq(l & 1, wg + 1, 0, lev, g, m), l, &bad);
                        b -= mu * e;
                    }
                }
                bb[r] = b;
                if constexpr (!REF) s_vec[cl][i] = b;
            }
            if (bad) __hip_atomic_store(&S.ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if constexpr (REF) {
                // (2) FP64 residual r = b - A_j Psi^(l), matrix-free
                double rr[RPT];
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int i = t + r * TPC;
                    double res = 0.0;
                    if (live && i < n) {
                        const int g = i / (4 * N), u = i & 3;
                        double cf[4];
                        lc_row(S, j, g, S.mu[(i >> 2) % N], u, cf);
                        const double *p = Lp + (i & ~3);
                        const double lp4 = cf[0] * p[0] + cf[1] * p[1] + cf[2] * p[2] + cf[3] * p[3];
                        double sc = 0.0;
                        const double *ss = S.sigma_s + ((size_t)j * G + g) * G;
                        for (int gp = 0; gp < G; ++gp) sc += ss[gp] * Lf[gp * 4 + u];
                        sc *= 0.25 * S.dx[j];
                        res = bb[r] - lp4 + sc;
                    }
                    rr[r] = res;
                }
                if constexpr (WAVE_CELL) {
                    // biased exponent of the largest |r| (0x7FF: not finite)
                    int ex = (int)(((uint64_t)__double_as_longlong(rr[0]) >> 52) & 0x7FF);
                    ex = seg_max_i32<TPC>(ex);
                    if (ex > 0 && ex < 0x7FF) expo = ex - 1022;
                } else {
                    double mx = 0.0;
#pragma unroll
                    for (int r = 0; r < RPT; ++r) mx = fmax(mx, fabs(rr[r]));
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
                    if ((tid_o & 63) == 0) s_max[tid_o >> 6] = mx;
                    __syncthreads();
                    mx = 0.0;
                    for (int w = cl * (TPC / 64); w < (cl + 1) * (TPC / 64); ++w) mx = fmax(mx, s_max[w]);
                    if (mx > 0.0 && isfinite(mx)) frexp(mx, &expo);
                }
#pragma unroll
                for (int r = 0; r < RPT; ++r) s_vec[cl][t + r * TPC] = (T)ldexp(rr[r], -expo);
            }
            __syncthreads();   // s_vec and the decision complete; every read of this tile's Psi^(l) is done
            if (tile == tile0 && lp >= 0 && s_dec[l & 1][0] != 0.0) {
                // the final iterate Psi^(l) and its flux leave LDS
                const int iters = lp + 1;
                const int fin = (base + iters) & 1;
                double *pout = S.psi[fin] + (size_t)c0 * n;
                const int totp = (c1 - c0) * n;
                for (int k = tid_o; k < totp; k += BS) pout[k] = L_psi[k];
                double *fout = S.phi[fin] + (size_t)c0 * 4 * G;
                const int totf = (c1 - c0) * 4 * G;
                for (int k = tid_o; k < totf; k += BS) fout[k] = L_phi[k];
                if (wg == 0 && tid_o == 0) {
                    Ctl *c = S.ctl;
                    c->base = base;
                    c->iter = iters;
                    c->e_last = s_dec[l & 1][2];
                    c->rho = s_dec[l & 1][3];
                    c->e_prev = s_dec[l & 1][2];
                    c->status = (int)s_dec[l & 1][1];
                    c->done = 1;
                }
                return;
            }

            // (3) apply the inverse, one row per thread, factors streamed as
            // coalesced 16-byte words
            T acc[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) acc[r] = T(0);
            if (live) stream_rows<T, NP, RPT, TPC, kStreamWords>(Xall + (size_t)j * NP * NP, t, &s_vec[cl][0], acc);

            // (4) new iterate (the range's two end edges also go to the
            // neighbours), scalar flux and its change
            double dsq = 0.0;
            double xs[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = t + r * TPC;
                double x = REF ? xold[r] + ldexp((double)acc[r], expo) : (double)acc[r];
                if (live && i < n) {
                    Lp[i] = x;
                    if (S.norm == 1) dsq += (x - xold[r]) * (x - xold[r]);
                    const int g = i / (4 * N), m = (i >> 2) % N, u = i & 3;
                    if (j == c0 && wg > 0 && m < nh && !(u & 1))
                        put_edge(exq(par, wg, 0, u >> 1, g, m), x, l + 1);
                    if (j == c1 - 1 && wg + 1 < (int)nwg && m >= nh && (u & 1))
                        put_edge(exq(par, wg, 1, u >> 1, g, m - nh), x, l + 1);
                } else {
                    x = 0.0;
                }
                xs[r] = x;
            }
            if (tree_phi) {
                // phi_(g,u) = sum_m w_m psi_(g,m,u): the m index occupies lane
                // bits 2 .. 1 + log2 N; rows of 16 lanes first (DPP), then
                // across rows
                double wx = (t < n) ? s_w[(t >> 2) % N] * xs[0] : 0.0;
                int off = 4;
                if (N >= 4) {
                    wx += dpp_f64<kDppRor4>(wx);
                    wx += dpp_f64<kDppRor8>(wx);
                    off = 16;
                }
                if (off == 16 && N >= 8) { wx = xor_add_f64<4>(wx); off = 32; }
                if (off == 32 && N >= 16) { wx = xor_add_f64<5>(wx); off = 64; }
                for (; off <= 2 * N; off <<= 1) wx += __shfl_xor(wx, off, 64);
                if (live && t < n && (t >> 2) % N == 0) {
                    const int fi = (t / (4 * N)) * 4 + (t & 3);
                    const double f0 = Lf[fi];
                    Lf[fi] = wx;
                    if (S.norm == 0) dsq += (wx - f0) * (wx - f0);
                }
            } else {
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int i = t + r * TPC;
                    L_wx[cl * NP + i] = (i < n ? s_w[(i >> 2) % N] : 0.0) * xs[r];
                }
                __syncthreads();
                if (live && t < 4 * G) {
                    const int g = t >> 2, u = t & 3;
                    double f = 0.0;
                    for (int m = 0; m < N; ++m) f += L_wx[cl * NP + (g * N + m) * 4 + u];
                    const double f0 = Lf[t];
                    Lf[t] = f;
                    if (S.norm == 0) dsq += (f - f0) * (f - f0);
                }
            }
            dsq_acc += dsq;
            if (tile + 1 < tile1) __syncthreads();   // s_vec / L_wx are reused by the next tile
        }

        // (5) the partial of iteration l (the edges just published need not
        // have completed: their readers wait on the slots themselves)
        {
            const double v = wave_sum_dpp(dsq_acc);
            if ((tid_o & 63) == 0) s_part[l & 1][tid_o >> 6] = v;
        }
        __syncthreads();
        if (tid_o < 64) {
            // wave 0 adds the wave sums (lanes 0 .. BS/64 - 1, a DPP row sum)
            double s = (tid_o < BS / 64) ? s_part[l & 1][tid_o] : 0.0;
            s += dpp_f64<kDppXor1>(s);
            s += dpp_f64<kDppXor2>(s);
            s += dpp_f64<kDppHalfMirror>(s);
            s += dpp_f64<kDppMirror>(s);
            if (tid_o == 0) st_bits(part_bits + (size_t)(l & (kPartSlots - 1)) * nwg + wg, part_encode(s, l));
        }
        // the decision wave loads the partials it decides on next time
        {
            const bool dq = (tid_o >> 6) == dec_wave;
            const uint64_t *pq = part_bits + (size_t)(l & (kPartSlots - 1)) * nwg;
#pragma unroll
            for (int r = 0; r < PV; ++r) {
                const int k = (tid_o & 63) + 64 * r;
                pv[r] = (dq && k < (int)nwg) ? ld_bits(pq + k) : kSlotEmpty;
            }
        }
    }
}

// Register-resident OCI kernel (FP32 n <= 64, FP64 n <= 32): one tile of
// CPT cells per workgroup (launched with nwg = ntiles), one cell per wave or
// less, each thread holding its row of the cell's inverse in VGPRs for the
// whole step.  The step is bound by instruction issue (four waves share a
// SIMD), so everything that does not change between iterations is prepared
// once: each lane's row coordinates and roles packed in one register, the
// constant part of b with the boundary sources folded in, the 4x4 corner
// coefficients and the scattering block (LDS).  Per iteration a wave runs its
// cells on its own (steps 1-4, ordered within the wave only), then all waves
// meet once at a workgroup barrier.  Edges cross workgroups through the tagged
// slots; the stopping decision works as in k_oci_local with three copies of
// the iterate's predecessors in LDS (kResidentCopies in all): every wave other
// than the two end ones adds a share of the partials of iteration l - LAG
// before the barrier, one wave applies the rule after it, and the outcome
// takes effect at the next barrier.  With io.nsteps > 1 one launch runs that
// many time steps: each stop but the last turns the iterate over to the next
// step inside the kernel (res_next_step), so the rows are loaded once.
namespace res {
enum : int {
    LIVE = 1 << 18,    // a row of a live cell (t < n, j < J)
    INL = 1 << 19,     // receives an edge from the left (mu > 0, u even)
    INR = 1 << 20,     // receives an edge from the right (mu < 0, u odd)
    BND = 1 << 21,     // ... from the slab boundary (folded into the constant part of b)
    EXT = 1 << 22,     // ... from a neighbour workgroup
    OUTL = 1 << 23,    // its new value goes to the left neighbour workgroup
    OUTR = 1 << 24,    // ... to the right neighbour workgroup
    PHI = 1 << 25,     // writes phi_(g,u) (m = 0)
    CELL = 1 << 26,    // the lane's cell is live (j < J)
};
}

// End of an inner time step of a multi-step launch of k_oci_res: the step's
// outputs (phi and its report), the next step's first iterate (the final
// one, in D, copied to the LDS copy Q of iteration nl0, with its phi summed
// as k_step_open sums it), the constant part of b after the time update
// psi_(k-1/2) <- psi_(k+1/2) (eq. rhs_sg, with the boundary sources as in the
// prologue), and the range's end edges of that iterate tagged nl0.
// psi_(k-1/2) itself is written by the launch's last step only.  Every thread
// of the workgroup calls it (two workgroup barriers).
template <int BS>
__device__ __attribute__((always_inline)) inline void res_next_step(const Slab &S, const StepIO &io, int step, int iters, int nl0,
                                                        int ri, int cl, int t, const double *D_psi,
                                                        const double *D_phi, double *Q_psi, double *Q_phi,
                                                        double *crow, int ldc, const double *mu_tab,
                                                        const double *dec, int c0, int c1, int wg, unsigned nwg) {
    const int tid = threadIdx.x;
    const int J = S.J, G = S.G, n = S.n, nh = S.N / 2, NG = S.N * S.G;
    const int totf = (c1 - c0) * 4 * G, totp = (c1 - c0) * n;
    double *fo = io.phi_out + ((size_t)step * J + c0) * 4 * G;
    for (int k = tid; k < totf; k += BS) fo[k] = D_phi[k];
    if (wg == 0 && tid == 0) {
        char *rec = reinterpret_cast<char *>(io.info) + (size_t)step * 24;   // oci_step_info
        const int err = __hip_atomic_load(&S.ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        reinterpret_cast<int32_t *>(rec)[0] = iters;
        reinterpret_cast<int32_t *>(rec)[1] = err ? -6 : (int)dec[1];
        reinterpret_cast<double *>(rec)[1] = dec[2];
        reinterpret_cast<double *>(rec)[2] = dec[3];
    }
    for (int k = tid; k < totp; k += BS) Q_psi[k] = D_psi[k];
    // phi of the first iterate summed over m in order, as a step opened by
    // k_step_open has it
    for (int k = tid; k < totf; k += BS) {
        const int u = k & 3, cg = k >> 2;   // cg = cell * G + g
        const double *p = D_psi + (size_t)cg * S.N * 4 + u;
        double f = 0.0;
        for (int m = 0; m < S.N; ++m) f += S.w[m] * p[m * 4];
        Q_phi[k] = f;
    }
    __syncthreads();
    if (ri & res::LIVE) {
        const int m = ri & 0xFF, g = (ri >> 8) & 0xFF, u = (ri >> 16) & 3, lev = u >> 1;
        const int j = c0 + cl;
        const double mu = mu_tab[m], dx = S.dx[j];
        const size_t jg = (size_t)j * G + g;
        // the next step's sources (per-step arrays when the strides are set)
        const double *q = io.q ? io.q + (size_t)(step + 1) * io.q_stride : nullptr;
        const double *il = io.inc_l ? io.inc_l + (size_t)(step + 1) * io.inc_stride : nullptr;
        const double *ir = io.inc_r ? io.inc_r + (size_t)(step + 1) * io.inc_stride : nullptr;
        double c = q ? 0.25 * dx * q[jg * 4 + u] : 0.0;
        if (u < 2) c += dx / (2.0 * S.speed[g] * S.dt) * Q_psi[(size_t)cl * n + t + 2];
        if ((ri & res::INL) && (ri & res::BND) && il) c += mu * il[((size_t)lev * G + g) * nh + (m - nh)];
        if ((ri & res::INR) && (ri & res::BND) && ir) c -= mu * ir[((size_t)lev * G + g) * nh + m];
        crow[(size_t)cl * ldc + t] = c;
        const double x = Q_psi[(size_t)cl * n + t];
        uint64_t *ex = reinterpret_cast<uint64_t *>(S.exch);
        auto slot = [&](int side, int mm) -> uint64_t * {
            return ex + 2 * ((((size_t)(nl0 & 1) * nwg + wg) * 2 + side) * NG + ((size_t)lev * G + g) * nh + mm);
        };
        if (ri & res::OUTL) put_edge(slot(0, m), x, nl0);
        if (ri & res::OUTR) put_edge(slot(1, m - nh), x, nl0);
    }
    __syncthreads();
}

template <typename T, int NP, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4)))
void k_oci_res(Slab S, StepIO io, int ntiles) {
    constexpr bool REF = sizeof(T) == 4;
    static_assert(NP <= 64 && NP >= 8, "one cell per wave or less");
    static_assert(BS <= 1024, "wave sums are added within one row of 16 lanes");
    constexpr int TPC = NP;
    constexpr int LOGT = NP == 8 ? 3 : NP == 16 ? 4 : NP == 32 ? 5 : 6;
    constexpr int CPT = BS / TPC;
    constexpr int W = BS / 64;
    constexpr int V = 16 / sizeof(T);
    constexpr int NV = NP / V;
    constexpr int LAG = kResidentLag;
    constexpr int NCOPY = kResidentCopies;
    typedef typename Vec16<T>::type VT;
    (void)ntiles;

    extern __shared__ __align__(16) double s_dyn[];
    __shared__ __align__(16) T s_vec[CPT][NP];
    __shared__ __align__(16) double s_coef[REF ? CPT : 1][REF ? NP : 1][4];
    __shared__ double s_crow[CPT][NP];
    __shared__ double s_scat[REF ? CPT : 1][REF ? NP * NP / 64 : 1];   // G*G <= NP*NP/64
    __shared__ double s_wx[CPT][NP];
    __shared__ double s_mu[NP / 4], s_w[NP / 4];
    __shared__ double s_part[2][W], s_psum[2][W], s_dec[2][4], s_eprev[2];

    const int tid = threadIdx.x;
    const int J = S.J, N = S.N, G = S.G, n = S.n, nh = S.N / 2, NG = S.N * S.G;
    const unsigned nwg = gridDim.x;
    const int wg = blockIdx.x;
    const int c0 = wg * CPT;
    const int c1 = min(c0 + CPT, J);
    double *L_psi0 = s_dyn;                                  // [NCOPY][CPT][n]
    double *L_phi0 = L_psi0 + (size_t)NCOPY * CPT * n;       // [NCOPY][CPT][4G]
    uint64_t *exch_bits = reinterpret_cast<uint64_t *>(S.exch);
    auto exq = [&](int par, int w, int side, int lev, int g, int mm) -> uint64_t * {
        return exch_bits + 2 * ((((size_t)par * nwg + w) * 2 + side) * NG + ((size_t)lev * G + g) * nh + mm);
    };

    for (int m = tid; m < N; m += BS) { s_mu[m] = S.mu[m]; s_w[m] = S.w[m]; }
    __syncthreads();

    // per-lane row coordinates and roles
    int rinfo = 0;
    {
        const int cl = tid >> LOGT, t = tid & (TPC - 1), j = c0 + cl;
        if (j < J) rinfo |= res::CELL;
        if (j < J && t < n) {
            const int g = t / (4 * N), m = (t >> 2) % N, u = t & 3;
            rinfo |= m | (g << 8) | (u << 16) | res::LIVE;
            if (m == 0) rinfo |= res::PHI;
            if (m >= nh && !(u & 1)) {
                rinfo |= res::INL;
                if (j == 0) rinfo |= res::BND;
                else if (j == c0) rinfo |= res::EXT;
            }
            if (m < nh && (u & 1)) {
                rinfo |= res::INR;
                if (j == J - 1) rinfo |= res::BND;
                else if (j == c1 - 1) rinfo |= res::EXT;
            }
            if (j == c0 && wg > 0 && m < nh && !(u & 1)) rinfo |= res::OUTL;
            if (j == c1 - 1 && c1 < J && m >= nh && (u & 1)) rinfo |= res::OUTR;
        }
    }

    // the inverse rows into registers; the iterate, its flux and the step's
    // constants into LDS
    const T *Xall = reinterpret_cast<const T *>(S.X);
    VT xr[NV];
    {
        const int cl = tid >> LOGT, t = tid & (TPC - 1), j = c0 + cl;
#pragma unroll
        for (int kv = 0; kv < NV; ++kv) xr[kv] = VT{};
        if (rinfo & res::CELL) {
            const T *Xc = Xall + (size_t)j * NP * NP;
#pragma unroll
            for (int kv = 0; kv < NV; ++kv) xr[kv] = *reinterpret_cast<const VT *>(Xc + ((size_t)kv * NP + t) * V);
        }
        if (rinfo & res::LIVE) {
            const int m = rinfo & 0xFF, g = (rinfo >> 8) & 0xFF, u = (rinfo >> 16) & 3, lev = u >> 1;
            const double mu = s_mu[m];
            double b = S.crhs[(size_t)j * n + t];
            if ((rinfo & res::INL) && (rinfo & res::BND) && io.inc_l)
                b += mu * io.inc_l[((size_t)lev * G + g) * nh + (m - nh)];
            if ((rinfo & res::INR) && (rinfo & res::BND) && io.inc_r)
                b -= mu * io.inc_r[((size_t)lev * G + g) * nh + m];
            s_crow[cl][t] = b;
            if constexpr (REF) lc_row(S, j, g, mu, u, s_coef[cl][t]);
        }
        if constexpr (REF)
            if ((rinfo & res::CELL) && t < G * G) s_scat[cl][t] = 0.25 * S.dx[j] * S.sigma_s[(size_t)j * G * G + t];
    }
    // the first iterate is the last one of the previous step (a step opened
    // by k_step_open leaves the control block as that step left it)
    const int base = (S.ctl->base + S.ctl->iter) & 1;
    const double *__restrict__ psi_g = S.psi[base];   // the iterate in global memory: only read at l = 0
    {
        const double *pin = psi_g + (size_t)c0 * n;
        const int tot = (c1 - c0) * n;
        for (int k = tid; k < tot; k += BS) L_psi0[k] = pin[k];
        const double *fin = S.phi[base] + (size_t)c0 * 4 * G;
        const int totf = (c1 - c0) * 4 * G;
        for (int k = tid; k < totf; k += BS) L_phi0[k] = fin[k];
    }
    __syncthreads();

    const bool tree_phi = (N & (N - 1)) == 0;
    uint64_t *part_bits = reinterpret_cast<uint64_t *>(S.partials);
    // shares of the partial sums: waves WS0 .. WS0 + WSN - 1 (not the two end
    // waves, which carry the range's end cells, when there are four or more)
    constexpr int WS0 = W >= 4 ? 1 : 0;
    constexpr int WSN = W >= 4 ? W - 2 : W;
    const int Sw = ((int)nwg + WSN - 1) / WSN;
    const int dec_wave = W / 2;
    // Several time steps in one launch (io.nsteps): iterations are numbered
    // across the launch (the tags of edges and partials never repeat), and
    // the current step starts at iteration l0 from the iterate its
    // predecessor stopped at.
    __shared__ int s_step;   // steps finished in this launch (read at a stop only)
    if (tid == 0) s_step = 0;
    int l0 = 0;

    for (int l = 0;; ++l) {
        // re-derived every iteration from opaque copies, so the compiler keeps
        // no per-lane addresses live across the loop (registers)
        int ri = rinfo, tq = tid;
        asm volatile("" : "+v"(ri), "+v"(tq));
        const int cl = tq >> LOGT, t = tq & (TPC - 1);
        const int m = ri & 0xFF, g = (ri >> 8) & 0xFF, u = (ri >> 16) & 3;
        const unsigned cb = (unsigned)l % NCOPY, nb = ((unsigned)l + 1) % NCOPY;
        // per-lane offsets by 24-bit multiplies (full rate; cl < CPT, n and 4G
        // at most NP), the copy's base in scalar registers
        const unsigned cln = __umul24((unsigned)cl, (unsigned)n), clf = __umul24((unsigned)cl, 4u * G);
        const double *Lp = L_psi0 + (size_t)cb * CPT * n + cln;      // this cell's Psi^(l)
        const double *Lf = L_phi0 + (size_t)cb * CPT * 4 * G + clf;
        double *Np = L_psi0 + (size_t)nb * CPT * n + cln;            // ... and Psi^(l+1)
        double *Nf = L_phi0 + (size_t)nb * CPT * 4 * G + clf;
        const int lp = l - LAG;                                   // iteration whose partials this one adds
        const bool lpv = lp >= l0;                                // ... one of this step
        const uint64_t *part_prev = part_bits + (size_t)(lp & (kPartSlots - 1)) * nwg;
        int bad = 0;

        // this wave's share of the partials of iteration lp, loaded now and
        // added before the barrier
        const int sh = (tq >> 6) - WS0;
        const int q0 = __mul24(sh, Sw) + (tq & 63);   // |sh| <= W, Sw <= the grid size
        const bool qon = lpv && sh >= 0 && sh < WSN && (tq & 63) < Sw && q0 < (int)nwg;
        const uint64_t qv = qon ? ld_bits(part_prev + q0) : kSlotEmpty;

        // (1) b = constant part + lagged incident edge from a cell
        double xold = 0.0, b = 0.0;
        if (ri & res::LIVE) {
            xold = Lp[t];
            b = s_crow[cl][t];
            if ((ri & (res::INL | res::INR)) && !(ri & res::BND)) {
                const double mu = s_mu[m];
                const int lev = u >> 1;
                double e;
                // upwind incident term: + mu psi_(j-1,R) for mu > 0, - mu psi_(j+1,L) for mu < 0
                if (ri & res::INL) {
                    if (!(ri & res::EXT)) e = Lp[t - n + 1];
                    else if (l == 0) e = psi_g[(size_t)(c0 - 1) * n + t + 1];
                    else e = take_edge(exq(l & 1, wg - 1, 1, lev, g, m - nh), l, &bad);
                    b += mu * e;
                } else {
                    if (!(ri & res::EXT)) e = Lp[t + n - 1];
                    else if (l == 0) e = psi_g[(size_t)c1 * n + t - 1];
                    else e = take_edge(exq(l & 1, wg + 1, 0, lev, g, m), l, &bad);
                    b -= mu * e;
                }
            }
        }
        if (bad) __hip_atomic_store(&S.ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

        int expo = 0;
        if constexpr (REF) {
            // (2) FP64 residual r = b - A_j Psi^(l), matrix-free, scaled by
            // the power of two of its largest entry in the cell
            double r = 0.0;
            if (ri & res::LIVE) {
                const double2 ca = *reinterpret_cast<const double2 *>(&s_coef[cl][t][0]);
                const double2 cc = *reinterpret_cast<const double2 *>(&s_coef[cl][t][2]);
                const double2 pa = *reinterpret_cast<const double2 *>(Lp + (t & ~3));
                const double2 pc = *reinterpret_cast<const double2 *>(Lp + (t & ~3) + 2);
                double sc = 0.0;
                const double *sg = &s_scat[cl][__umul24((unsigned)g, (unsigned)G)];
                for (int gp = 0; gp < G; ++gp) sc += sg[gp] * Lf[gp * 4 + u];
                r = b - (ca.x * pa.x + ca.y * pa.y + cc.x * pc.x + cc.y * pc.y) + sc;
            }
            int ex = (int)(((uint64_t)__double_as_longlong(r) >> 52) & 0x7FF);
            ex = seg_max_i32<TPC>(ex);
            if (ex > 0 && ex < 0x7FF) expo = ex - 1022;
            s_vec[cl][t] = (T)ldexp(r, -expo);
        } else {
            s_vec[cl][t] = (T)b;
        }
        wave_sync();   // the cell's s_vec is complete (the cell is this wave's)

        // (3) apply the inverse: four FMA chains over the row, a quarter as
        // long as one
        T a4[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int kv = 0; kv < NV; ++kv) {
            const VT bv = *reinterpret_cast<const VT *>(&s_vec[cl][kv * V]);
            a4[kv & 3] = fma_dot16(xr[kv], bv, a4[kv & 3]);
        }
        const T acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);

        // (4) new iterate (the range's two end edges also go to the
        // neighbours), scalar flux and its change
        const double x = REF ? xold + ldexp((double)acc, expo) : (double)acc;
        double dsq = 0.0;
        if (ri & res::LIVE) {
            Np[t] = x;
            if (S.norm == 1) dsq = (x - xold) * (x - xold);
            const int par = (l + 1) & 1;
            if (ri & res::OUTL) put_edge(exq(par, wg, 0, u >> 1, g, m), x, l + 1);
            if (ri & res::OUTR) put_edge(exq(par, wg, 1, u >> 1, g, m - nh), x, l + 1);
        }
        if (tree_phi) {
            // phi_(g,u) = sum_m w_m psi_(g,m,u): m occupies lane bits 2 ..
            // 1 + log2 N; rows of 16 lanes first (DPP), then across rows
            double wx = (ri & res::LIVE) ? s_w[m] * x : 0.0;
            int off = 4;
            if (N >= 4) {
                wx += dpp_f64<kDppRor4>(wx);
                wx += dpp_f64<kDppRor8>(wx);
                off = 16;
            }
            if (off == 16 && N >= 8) { wx = xor_add_f64<4>(wx); off = 32; }
            if (off == 32 && N >= 16) { wx = xor_add_f64<5>(wx); off = 64; }
            for (; off <= 2 * N; off <<= 1) wx += __shfl_xor(wx, off, 64);
            if (ri & res::PHI) {
                const int fi = g * 4 + u;
                const double f0 = Lf[fi];
                Nf[fi] = wx;
                if (S.norm == 0) dsq += (wx - f0) * (wx - f0);
            }
        } else {
            s_wx[cl][t] = (ri & res::LIVE) ? s_w[m] * x : 0.0;
            wave_sync();
            if ((ri & res::CELL) && t < 4 * G) {
                const int gg = t >> 2, uu = t & 3;
                double f = 0.0;
                for (int mm = 0; mm < N; ++mm) f += s_wx[cl][(gg * N + mm) * 4 + uu];
                const double f0 = Lf[t];
                Nf[t] = f;
                if (S.norm == 0) dsq += (f - f0) * (f - f0);
            }
        }

        // (5) this wave's sum of squared changes and its share of the
        // partials of iteration lp, then the barrier
        {
            double v;
            if (S.norm == 0 && G == 1 && tree_phi) {
                // the changes sit in lanes 0 .. 3 of each cell (m = 0, g = 0)
                double q = dsq;
                q += dpp_f64<kDppXor1>(q);
                q += dpp_f64<kDppXor2>(q);
                v = 0.0;
#pragma unroll
                for (int c = 0; c < 64 / TPC; ++c) v += readlane_f64(q, c * TPC);
            } else {
                v = wave_sum_dpp(dsq);
            }
            if ((tid & 63) == 0) s_part[l & 1][tid >> 6] = v;
        }
        if (lpv) {
            double v = 0.0;
            if (qon) {
                auto wait_part = [&](uint64_t xq, int k) -> double {
                    long spins = 0;
#pragma clang loop unroll(disable)
                    while (!part_ready(xq, lp)) {
                        __builtin_amdgcn_s_sleep(1);
                        if (++spins > kSpinLimit) { bad = 1; break; }
                        xq = ld_bits(part_prev + k);
                    }
                    return part_value(xq);
                };
                const int b0 = q0 - (tid & 63);
                v = wait_part(qv, q0);
                for (int k = (tid & 63) + 64; k < Sw && b0 + k < (int)nwg; k += 64)
                    v += wait_part(ld_bits(part_prev + b0 + k), b0 + k);
            }
            if (bad) {
                __hip_atomic_store(&S.ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                v = __builtin_nan("");
            }
            v = wave_sum_dpp(v);
            if ((tid & 63) == 0) s_psum[l & 1][tid >> 6] = v;
        }
        __syncthreads();

        // the decision taken after the previous barrier applies now; on a
        // stop the iterate it concerns, Psi^(l-LAG), is intact in its copy
        if (l - 1 - LAG >= l0 && s_dec[(l + 1) & 1][0] != 0.0) {
            const int fl = l - LAG;             // the final iterate (launch numbering)
            const int iters = fl - l0;          // iterations of this step
            const double *D_psi = L_psi0 + (size_t)((unsigned)fl % NCOPY) * CPT * n;
            const double *D_phi = L_phi0 + (size_t)((unsigned)fl % NCOPY) * CPT * 4 * G;
            const int step = s_step;
            if (step + 1 < io.nsteps) {
                // iterations l + 1 and l + 2 are skipped: the edge slots of
                // parity l + 1 hold iterate l + 1's edges, which nobody reads,
                // while those of parity l may still be waited for
                const int nl0 = l + 3;
                // iterations l .. l + 2 publish no partials, so their slots
                // would still hold those of l - 8 .. l - 6, whose tags are
                // the ones l + 8 .. l + 10 will carry: empty them (every
                // reader of l - 8 .. l - 6 is done, since every workgroup has
                // published its partial of l - 2).  Thread 0 also writes the
                // later partials, so the stores reach each slot in order.
                if (tid == 0)
                    for (int x = l; x < nl0; ++x)
                        st_bits(part_bits + (size_t)(x & (kPartSlots - 1)) * nwg + wg, kSlotEmpty);
                res_next_step<BS>(S, io, step, iters, nl0, ri, cl, t, D_psi, D_phi,
                                  L_psi0 + (size_t)((unsigned)nl0 % NCOPY) * CPT * n,
                                  L_phi0 + (size_t)((unsigned)nl0 % NCOPY) * CPT * 4 * G, &s_crow[0][0], NP, s_mu,
                                  &s_dec[(l + 1) & 1][0], c0, c1, wg, nwg);
                if (tid == 0) s_step = step + 1;   // read again only after the next step's barriers
                l0 = nl0;
                l = nl0 - 1;
                continue;
            }
            const int fin = (base + iters) & 1;
            double *pout = S.psi[fin] + (size_t)c0 * n;
            const int totp = (c1 - c0) * n;
            for (int k = tid; k < totp; k += BS) pout[k] = D_psi[k];
            double *fout = S.phi[fin] + (size_t)c0 * 4 * G;
            const int totf = (c1 - c0) * 4 * G;
            for (int k = tid; k < totf; k += BS) fout[k] = D_phi[k];
            if (wg == 0 && tid == 0) {
                Ctl *c = S.ctl;
                c->base = base;
                c->iter = iters;
                c->e_last = s_dec[(l + 1) & 1][2];
                c->rho = s_dec[(l + 1) & 1][3];
                c->e_prev = s_dec[(l + 1) & 1][2];
                c->status = (int)s_dec[(l + 1) & 1][1];
                c->done = 1;
            }
            return;
        }
        if (lpv && (tid >> 6) == dec_wave) {
            // the stopping rule (section 2.1) on e_(lp+1), from the shares
            // (every workgroup's decision wave adds the same values in the
            // same order)
            double tot = 0.0;
#pragma unroll
            for (int w = 0; w < W; ++w) tot += s_psum[l & 1][w];
            const int iters = lp + 1 - l0;
            const double e = sqrt(tot);
            const double rho = iters >= 2 ? e / s_eprev[(l + 1) & 1] : __builtin_nan("");
            int done = 0, status = OK;
            if (!isfinite(e)) { done = 1; status = NONFINITE; }
            else if (S.fixed_iters > 0) done = iters >= S.fixed_iters;
            else if (iters >= 2 && (e == 0.0 || e < S.tol * (1.0 - rho))) done = 1;
            else if (iters >= S.max_iters) { done = 1; status = NOT_CONVERGED; }
            if (S.hist && iters <= S.hist_cap && wg == 0 && (tid & 63) == 0) S.hist[iters - 1] = e;
            if ((tid & 63) == 0) {
                s_eprev[l & 1] = e;
                s_dec[l & 1][0] = done;
                s_dec[l & 1][1] = status;
                s_dec[l & 1][2] = e;
                s_dec[l & 1][3] = rho;
            }
        }
        if (tid < 64) {
            // wave 0 publishes the workgroup's partial of iteration l (the
            // W wave sums added in a DPP row)
            double s = (tid < W) ? s_part[l & 1][tid] : 0.0;
            s += dpp_f64<kDppXor1>(s);
            s += dpp_f64<kDppXor2>(s);
            s += dpp_f64<kDppHalfMirror>(s);
            s += dpp_f64<kDppMirror>(s);
            if (tid == 0) st_bits(part_bits + (size_t)(l & (kPartSlots - 1)) * nwg + wg, part_encode(s, l));
        }
    }
}

// Constant part of b for the current step (eq. rhs_sg without the incident
// terms): dx/4 Q_u, plus dx/(2 v dt) psi_{k-1/2} in the level-k rows.  One
// thread per row of every cell; used by every iteration of OCI and SI.
__device__ inline void const_rhs_elem(const Slab &S, const StepIO &io, size_t t) {
    const int u = t & 3;
    const size_t jgm = t >> 2;
    const size_t jg = jgm / S.N;
    const int g = jg % S.G;
    const int j = jg / S.G;
    const double dx = S.dx[j];
    double c = io.q ? 0.25 * dx * io.q[jg * 4 + u] : 0.0;
    if (u < 2) c += dx / (2.0 * S.speed[g] * S.dt) * S.psi_prev[jgm * 2 + u];
    S.crhs[t] = c;
}
__global__ __launch_bounds__(kBlock) void k_const_rhs(Slab S, StepIO io) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < (size_t)S.J * S.n) const_rhs_elem(S, io, t);
}

// --------------------------------------------------------------- SI kernels
// Source iteration (Appendix A, Algorithm 1) with the scattering source of
// the previous iterate.  Each (group, angle) chain is swept cell by cell, as
// in the paper, but the work that does not depend on the incoming edge runs
// in parallel around the serial part:
//   pre    every (cell, group, angle): d = constant RHS + dx/4 sum_g' Ss
//          phi^(l), the uncoupled solution base = L_c^-1 d and its outgoing
//          edges;
//   sweep  one workgroup: the chains run e_out = alpha + M e_in cell by cell
//          (M: the 2x2 edge-to-edge map of the cell), reading alpha and M
//          from an LDS ring that the other waves fill ahead of them; the
//          incident edge met at every cell is recorded;
//   flux   every (cell, group, corner/level): psi = base + response x
//          incident edge, phi = sum_m w_m psi, its change; then the norm and
//          the decision.
// The whole iteration loop of a step runs in one persistent launch
// (k_si_loop: the decision never leaves the device), on one workgroup for
// small problems (phases separated by workgroup barriers) or on many (grid
// barriers with agent-scope release/acquire between the phases).  The
// per-phase kernels (k_si_pre, k_si_sweep, k_si_flux) remain as the launch
// sequence that a host loop can drive.

// One (cell, group, angle) row of the pre pass.
__device__ inline void si_pre_row(const Slab &S, size_t t, int cur) {
    const int N = S.N, G = S.G;
    const unsigned tu = (unsigned)t, jg32 = tu / (unsigned)N;   // J G N < 2^31: 32-bit division
    const int m = tu - jg32 * N, g = jg32 % (unsigned)G, j = jg32 / (unsigned)G;
    const size_t jg = (size_t)j * G + g;
    const double *phi_in = S.phi[cur];
    const double *cr = S.crhs + t * 4;
    const double dx4 = 0.25 * S.dx[j];
    double d[4];
    for (int u = 0; u < 4; ++u) {
        double sc = 0.0;
        for (int gp = 0; gp < G; ++gp) sc += S.sigma_s[jg * G + gp] * phi_in[((size_t)j * G + gp) * 4 + u];
        d[u] = cr[u] + dx4 * sc;
    }
    const double *Li = S.si_linv + t * 16;
    double x[4];
    for (int r = 0; r < 4; ++r) x[r] = Li[r * 4 + 0] * d[0] + Li[r * 4 + 1] * d[1] + Li[r * 4 + 2] * d[2] + Li[r * 4 + 3] * d[3];
    double *o = S.psi[cur ^ 1] + t * 4;
    o[0] = x[0]; o[1] = x[1]; o[2] = x[2]; o[3] = x[3];
    const bool pos = S.mu[m] > 0.0;
    const int step = pos ? j : S.J - 1 - j;
    double *al = S.si_alpha + ((size_t)step * N * G + g * N + m) * 2;
    al[0] = pos ? x[1] : x[0];
    al[1] = pos ? x[3] : x[2];
}

constexpr int kSweepBlock = 1024;

// The chain sweep, run by all kSweepBlock threads of one workgroup.  LDS
// ring: [2][C][NG][6] doubles (alpha0, alpha1, M00, M01, M10, M11 per chain
// and sweep step).  Waves at or after the first wave without chains fill
// buffer (c+1) & 1 while the chain lanes consume c & 1.
__device__ inline void si_sweep_body(const Slab &S, const StepIO &io, int C, double *s_ring) {
    const int N = S.N, G = S.G, J = S.J, NG = N * G, nh = N / 2;
    const int tid = threadIdx.x;
    const int chain_waves = (NG + 63) / 64;
    const int prod0 = chain_waves * 64;                  // first producer thread
    const int nprod = kSweepBlock - prod0;
    const size_t per_step = (size_t)NG * 6;
    const int nchunks = (J + C - 1) / C;
    auto fill = [&](int chunk, int buf, int first, int stride) {
        double *dst = s_ring + (size_t)buf * C * per_step;
        const int s0 = chunk * C;
        const int ns = min(C, J - s0);
        const size_t tot = (size_t)ns * per_step;
        for (size_t idx = first; idx < tot; idx += stride) {
            const int sl = idx / per_step;
            const int r = idx % per_step;
            const int k = r / 6, q = r % 6;
            const size_t st = (size_t)(s0 + sl) * NG + k;
            dst[idx] = q < 2 ? S.si_alpha[st * 2 + q] : S.si_msw[st * 4 + (q - 2)];
        }
    };
    double e0 = 0.0, e1 = 0.0;
    if (tid < NG) {
        const int g = tid / N, m = tid % N;
        if (S.mu[m] > 0.0) {
            if (io.inc_l) { e0 = io.inc_l[(size_t)g * nh + (m - nh)]; e1 = io.inc_l[((size_t)G + g) * nh + (m - nh)]; }
        } else {
            if (io.inc_r) { e0 = io.inc_r[(size_t)g * nh + m]; e1 = io.inc_r[((size_t)G + g) * nh + m]; }
        }
    }
    fill(0, 0, tid, kSweepBlock);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        if (tid >= prod0 && c + 1 < nchunks) fill(c + 1, (c + 1) & 1, tid - prod0, nprod);
        if (tid < NG) {
            const double *src = s_ring + (size_t)(c & 1) * C * per_step + (size_t)tid * 6;
            const int s0 = c * C;
            const int ns = min(C, J - s0);
            double *ein = S.si_ein + ((size_t)s0 * NG + tid) * 2;
#pragma unroll 4
            for (int sl = 0; sl < ns; ++sl) {
                const double *v = src + (size_t)sl * per_step;
                ein[(size_t)sl * NG * 2 + 0] = e0;
                ein[(size_t)sl * NG * 2 + 1] = e1;
                const double n0 = v[0] + v[2] * e0 + v[3] * e1;
                const double n1 = v[1] + v[4] * e0 + v[5] * e1;
                e0 = n0;
                e1 = n1;
            }
        }
        __syncthreads();
    }
}

// One (cell, group, corner/level) entry of the flux pass: the iterate's
// corner values from the base and the recorded incident edges, their
// scalar flux (ascending m); returns its squared change.
__device__ inline double si_flux_elem(const Slab &S, size_t t, int cur) {
    const int u = t & 3;
    const int N = S.N, G = S.G, NG = N * G;
    const size_t jg = t >> 2;
    const int g = (unsigned)jg % (unsigned)G, j = (unsigned)jg / (unsigned)G;
    double *p = S.psi[cur ^ 1] + jg * N * 4 + u;
    const double *rs = S.si_resp + jg * N * 8 + u;
    double f = 0.0;
#pragma unroll 4
    for (int m = 0; m < N; ++m) {
        const int step = S.mu[m] > 0.0 ? j : S.J - 1 - j;
        const double *ei = S.si_ein + ((size_t)step * NG + g * N + m) * 2;
        const double x = p[m * 4] + rs[m * 8] * ei[0] + rs[m * 8 + 4] * ei[1];
        p[m * 4] = x;
        f += S.w[m] * x;
    }
    const double f0 = S.phi[cur][t];
    S.phi[cur ^ 1][t] = f;
    return (f - f0) * (f - f0);
}

__global__ __launch_bounds__(kBlock) void k_si_pre(Slab S) {
    const Ctl *c = S.ctl;
    if (c->done) return;
    const int cur = (c->base + c->iter) & 1;
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < (size_t)S.J * S.G * S.N) si_pre_row(S, t, cur);
}

__global__ __launch_bounds__(kSweepBlock) void k_si_sweep(Slab S, StepIO io, int C) {
    extern __shared__ __align__(16) double s_ring[];
    if (S.ctl->done) return;
    si_sweep_body(S, io, C, s_ring);
}

// phi of the sweep, its change, and the decision (last block to finish).
__global__ __launch_bounds__(kBlock) void k_si_flux(Slab S) {
    __shared__ double s_tmp[kBlock / 64 + 1];
    __shared__ int s_last;
    Ctl *c = S.ctl;
    if (c->done) return;
    const int cur = (c->base + c->iter) & 1;
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const double dsq = t < (size_t)S.J * S.G * 4 ? si_flux_elem(S, t, cur) : 0.0;
    const double part = block_sum(dsq, s_tmp);
    if (threadIdx.x == 0) {
        S.partials[blockIdx.x] = part;
        __threadfence();
        const unsigned old = __hip_atomic_fetch_add(&c->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (old == gridDim.x - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    double v = 0.0;
    for (unsigned k = threadIdx.x; k < gridDim.x; k += kBlock) v += S.partials[k];
    const double tot = block_sum(v, s_tmp);
    if (threadIdx.x == 0) {
        c->bar_count = 0;
        decide(S, sqrt(tot));
    }
}

// The whole SI iteration loop of a step in one persistent launch: per
// iteration the pre pass (grid-stride), a barrier, the chain sweep by
// workgroup 0, a barrier, the flux pass and the norm, a barrier carrying the
// norm; every workgroup then applies the stopping rule to the same total.
// MULTI = false: one workgroup, workgroup barriers.  MULTI = true: grid
// barriers whose agent-scope release/acquire make each phase's global
// writes visible to every workgroup (grid_sync_sum).
template <bool MULTI>
__global__ __launch_bounds__(kSweepBlock) void k_si_loop(Slab S, StepIO io, int C) {
    extern __shared__ __align__(16) double s_ring[];
    __shared__ double s_tmp[kSweepBlock / 64 + 1];
    __shared__ int s_flag[4];
    const unsigned wg = blockIdx.x, nwg = gridDim.x;
    const int base = S.ctl->base;
    const size_t rows = (size_t)S.J * S.G * S.N, elems = (size_t)S.J * S.G * 4;
    const size_t stride = (size_t)nwg * kSweepBlock, t0 = (size_t)wg * kSweepBlock + threadIdx.x;
    double e_prev = __builtin_nan("");
    int round = 0;
    // a barrier between phases; the sum of the workgroups' v (valid in thread 0) in *total
    auto barrier = [&](double v, double *total) -> bool {
        if constexpr (MULTI) {
            return grid_sync_sum<kSweepBlock>(S, wg, nwg, round++, v, s_flag, s_tmp, total);
        } else {
            __syncthreads();
            if (threadIdx.x == 0) s_tmp[kSweepBlock / 64] = v;
            __syncthreads();
            *total = s_tmp[kSweepBlock / 64];
            return true;
        }
    };
    for (int l = 0;; ++l) {
        const int cur = (base + l) & 1;
        for (size_t t = t0; t < rows; t += stride) si_pre_row(S, t, cur);
        double unused = 0.0;
        if (!barrier(0.0, &unused)) return;
        if (wg == 0) si_sweep_body(S, io, C, s_ring);
        if (!barrier(0.0, &unused)) return;
        double dsq = 0.0;
        for (size_t t = t0; t < elems; t += stride) dsq += si_flux_elem(S, t, cur);
        const double part = block_sum_t<kSweepBlock>(dsq, s_tmp);   // valid in thread 0
        double tot = 0.0;
        if (!barrier(part, &tot)) return;
        const int iters = l + 1;
        const double e = sqrt(tot);
        int status = OK;
        const int done = stop_rule(S, iters, e, e_prev, &status);
        if (wg == 0 && threadIdx.x == 0) {
            Ctl *c = S.ctl;
            c->iter = iters;
            c->e_last = e;
            c->rho = iters >= 2 ? e / e_prev : __builtin_nan("");
            c->e_prev = e;
            c->status = status;
            c->done = done;
        }
        e_prev = e;
        if (done) return;
    }
}

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }

// ------------------------------------------------------------ batched slabs
// Many independent slab problems (uneven J, N, G) in one persistent launch.
// Slab k owns the workgroups [wg0, wg0 + nwg) of the grid; each runs the
// global-memory iteration body of its own cell size on its own control block,
// partial sums and barrier counters, so slabs converge independently and the
// launch ends when the last one has.
template <typename T, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4)))
void k_oci_batch(const BatchEntry *__restrict__ tab, int nslab) {
    // one workgroup runs one body: their LDS overlays
    constexpr size_t kLds = cmax(cmax(cmax(sizeof(GlobalLds<T, 8, false, BS>), sizeof(GlobalLds<T, 16, false, BS>)),
                                      cmax(sizeof(GlobalLds<T, 32, false, BS>), sizeof(GlobalLds<T, 64, false, BS>))),
                                 cmax(cmax(sizeof(GlobalLds<T, 128, false, BS>), sizeof(GlobalLds<T, 256, false, BS>)),
                                      sizeof(GlobalLds<T, 512, false, BS>)));
    __shared__ __align__(16) unsigned char s_lds[kLds];
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
    // the slab's view stays in the table (read through the scalar cache): a
    // local copy would sit in scratch memory, as the body indexes its
    // ping-pong pointer arrays with the run-time buffer parity
    const BatchEntry &e = tab[__builtin_amdgcn_readfirstlane(s_k)];
    const int lw = (int)blockIdx.x - e.wg0;
    if (lw < 0 || lw >= e.nwg) return;
    const Slab &S = e.S;
    const StepIO &io = e.io;
    switch (S.np) {
    case 8: oci_global_body<T, 8, false, BS>(S, io, e.ntiles, lw, e.nwg, s_lds); break;
    case 16: oci_global_body<T, 16, false, BS>(S, io, e.ntiles, lw, e.nwg, s_lds); break;
    case 32: oci_global_body<T, 32, false, BS>(S, io, e.ntiles, lw, e.nwg, s_lds); break;
    case 64: oci_global_body<T, 64, false, BS>(S, io, e.ntiles, lw, e.nwg, s_lds); break;
    case 128: oci_global_body<T, 128, false, BS>(S, io, e.ntiles, lw, e.nwg, s_lds); break;
    case 256: oci_global_body<T, 256, false, BS>(S, io, e.ntiles, lw, e.nwg, s_lds); break;
    case 512: oci_global_body<T, 512, false, BS>(S, io, e.ntiles, lw, e.nwg, s_lds); break;
    default: break;
    }
}

// Bookkeeping over every slab of the table: blockIdx.y = slab, grid-stride x.
__global__ void k_batch_begin(const BatchEntry *tab) { begin_one(tab[blockIdx.x].S); }

__global__ __launch_bounds__(kBlock) void k_batch_elems(const BatchEntry *tab, int what, int broadcast) {
    const BatchEntry &e = tab[blockIdx.y];
    const Slab &S = e.S;
    const size_t stride = (size_t)gridDim.x * kBlock;
    const size_t t0 = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (what == 0) {           // first iterate (when the state was replaced) and the constant RHS
        if (broadcast || S.ctl->bcast)
            for (size_t t = t0; t < (size_t)S.J * S.n; t += stride) broadcast_elem(S, t);
        if (!S.wb)
            for (size_t t = t0; t < (size_t)S.J * S.n; t += stride) const_rhs_elem(S, e.io, t);
    } else if (what == 1) {    // phi of the first iterate
        for (size_t t = t0; t < (size_t)S.J * S.G * 4; t += stride) phi0_elem(S, t);
        if (t0 == 0) S.ctl->bcast = 0;
    } else {                   // end of step
        const size_t ne = end_elems(S);
        for (size_t t = t0; t < ne; t += stride) end_elem(S, e.io, t);
    }
}

template <typename T, int BS>
static hipError_t batch_launch_t(const BatchEntry *tab, int nslab, int nwg, hipStream_t st, bool coop) {
    if (coop) {
        void *args[] = {(void *)&tab, (void *)&nslab};
        return hipLaunchCooperativeKernel((const void *)&k_oci_batch<T, BS>, dim3(nwg), dim3(BS), args, 0, st);
    }
    hipLaunchKernelGGL((k_oci_batch<T, BS>), dim3(nwg), dim3(BS), 0, st, tab, nslab);
    return hipGetLastError();
}

constexpr int kBatchBlock = 256;

hipError_t batch_occupancy(bool fp32, int *blocks) {
    return fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void *)&k_oci_batch<float, kBatchBlock>,
                                                              kBatchBlock, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void *)&k_oci_batch<double, kBatchBlock>,
                                                              kBatchBlock, 0);
}

int batch_block() { return kBatchBlock; }

__global__ void k_flag_broadcast(Slab S) { S.ctl->bcast = 1; }
hipError_t launch_flag_broadcast(const Slab &S, hipStream_t st) {
    hipLaunchKernelGGL(k_flag_broadcast, dim3(1), dim3(1), 0, st, S);
    return hipGetLastError();
}

// One batched time step: bookkeeping for all slabs, the persistent launch,
// the end-of-step kernel.  No memset and no host synchronisation, so the
// sequence can be captured into a graph (then with a normal launch).
hipError_t launch_wb_batch(const BatchEntry *tab, int nslab, int nwg, bool staged, hipStream_t st);

hipError_t launch_batch_step(const BatchEntry *tab, int nslab, int nwg, bool fp32, bool structured, bool staged,
                             bool broadcast, hipStream_t st, bool coop) {
    hipLaunchKernelGGL(k_batch_begin, dim3(nslab), dim3(1), 0, st, tab);
    hipLaunchKernelGGL(k_batch_elems, dim3(256, nslab), dim3(kBlock), 0, st, tab, 0, broadcast ? 1 : 0);
    hipLaunchKernelGGL(k_batch_elems, dim3(64, nslab), dim3(kBlock), 0, st, tab, 1, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = structured ? launch_wb_batch(tab, nslab, nwg, staged, st)
        : fp32     ? batch_launch_t<float, kBatchBlock>(tab, nslab, nwg, st, coop)
                   : batch_launch_t<double, kBatchBlock>(tab, nslab, nwg, st, coop);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_elems, dim3(256, nslab), dim3(kBlock), 0, st, tab, 2, 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------- launchers
template <typename T, int NP, bool RES, int BS>
static hipError_t launch_oci_t(const Slab &S, const StepIO &io, int nwg, int ntiles, hipStream_t st,
                               bool cooperative) {
    void *args[] = {(void *)&S, (void *)&io, (void *)&ntiles};
    if (cooperative)
        return hipLaunchCooperativeKernel((const void *)&k_oci_step<T, NP, RES, BS>, dim3(nwg), dim3(BS), args, 0, st);
    hipLaunchKernelGGL((k_oci_step<T, NP, RES, BS>), dim3(nwg), dim3(BS), 0, st, S, io, ntiles);
    return hipGetLastError();
}

template <typename T, int NP, bool RES, int BS>
static hipError_t occupancy_t(int *blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void *)&k_oci_step<T, NP, RES, BS>, BS, 0);
}

// Register residency is compiled for rows of at most 64 floats (refined) or
// 32 doubles (FP64): 64 VGPRs of inverse per thread.
bool resident_supported(bool fp32, int np) { return fp32 ? np <= 64 : np <= 32; }

// Block sizes compiled for the step kernel.
bool block_supported(int bs) { return bs == 256 || bs == 1024; }

template <typename T, bool RES, int BS, typename F>
static hipError_t by_np(int np, F f) {
    switch (np) {
    case 8: return f.template operator()<T, 8, RES, BS>();
    case 16: return f.template operator()<T, 16, RES, BS>();
    case 32: return f.template operator()<T, 32, RES, BS>();
    case 64: return f.template operator()<T, 64, (RES && sizeof(T) == 4), BS>();
    case 128: return f.template operator()<T, 128, false, BS>();
    case 256: return f.template operator()<T, 256, false, BS>();
    case 512: return f.template operator()<T, 512, false, BS>();
    default: return hipErrorInvalidValue;
    }
}

template <typename F>
static hipError_t dispatch(bool fp32, int np, bool res, int bs, F f) {
    if (fp32) {
        if (res && np <= 64) return bs == 1024 ? by_np<float, true, 1024>(np, f) : by_np<float, true, 256>(np, f);
        return bs == 1024 ? by_np<float, false, 1024>(np, f) : by_np<float, false, 256>(np, f);
    }
    if (res && np <= 32) return bs == 1024 ? by_np<double, true, 1024>(np, f) : by_np<double, true, 256>(np, f);
    return bs == 1024 ? by_np<double, false, 1024>(np, f) : by_np<double, false, 256>(np, f);
}

// The workgroup-local kernel of a launch shape: register-resident rows run
// k_oci_res, streamed rows k_oci_local.
template <typename T, int NP, bool RES, int BS>
static const void *local_kernel() {
    if constexpr (RES) return (const void *)&k_oci_res<T, NP, BS>;
    else return (const void *)&k_oci_local<T, NP, BS>;
}

// Raises a kernel's dynamic LDS limit to all the LDS its static part leaves,
// once per device.
static hipError_t allow_dynamic_lds(const void *f, int *done) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (done[dev]) return hipSuccess;
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, f);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(160 * 1024 - a.sharedSizeBytes));
    if (e == hipSuccess) done[dev] = 1;
    return e;
}

// The persistent local kernels are launched as ordinary kernels: the grid
// never exceeds what the occupancy query says fits at once, so on an
// otherwise idle device every workgroup is resident; the bounded waits turn
// a violation into OCI_ERR_DEVICE instead of a hang.
template <typename T, int NP, bool RES, int BS>
static hipError_t launch_local_t(const Slab &S, const StepIO &io, int nwg, int ntiles, size_t dyn, hipStream_t st) {
    if (RES && nwg != ntiles) return hipErrorInvalidValue;
    static int attr_done[64] = {0};
    const void *f = local_kernel<T, NP, RES, BS>();
    hipError_t e = allow_dynamic_lds(f, attr_done);
    if (e != hipSuccess) return e;
    void *args[] = {(void *)&S, (void *)&io, (void *)&ntiles};
    return hipLaunchKernel(f, dim3(nwg), dim3(BS), args, dyn, st);
}

template <typename T, int NP, bool RES, int BS>
static hipError_t occupancy_local_t(int *blocks, size_t dyn) {
    static int attr_done[64] = {0};
    const void *f = local_kernel<T, NP, RES, BS>();
    hipError_t e = allow_dynamic_lds(f, attr_done);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, f, BS, dyn);
}

template <typename T, int NP, bool RES, int BS>
static size_t static_lds_local_t() {
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, local_kernel<T, NP, RES, BS>()) != hipSuccess) return (size_t)-1;
    return a.sharedSizeBytes;
}

struct OccLocalF {
    int *blocks; size_t dyn;
    template <typename T, int NP, bool RES, int BS> hipError_t operator()() {
        return occupancy_local_t<T, NP, RES, BS>(blocks, dyn);
    }
};
struct StaticLdsF {
    size_t *bytes;
    template <typename T, int NP, bool RES, int BS> hipError_t operator()() {
        *bytes = static_lds_local_t<T, NP, RES, BS>();
        return *bytes == (size_t)-1 ? hipErrorInvalidValue : hipSuccess;
    }
};
struct LaunchLocalF {
    const Slab &S; const StepIO &io; int nwg, ntiles; size_t dyn; hipStream_t st;
    template <typename T, int NP, bool RES, int BS> hipError_t operator()() {
        return launch_local_t<T, NP, RES, BS>(S, io, nwg, ntiles, dyn, st);
    }
};

struct OccF {
    int *blocks;
    template <typename T, int NP, bool RES, int BS> hipError_t operator()() { return occupancy_t<T, NP, RES, BS>(blocks); }
};
struct LaunchF {
    const Slab &S; const StepIO &io; int nwg, ntiles; hipStream_t st; bool coop;
    template <typename T, int NP, bool RES, int BS> hipError_t operator()() {
        return launch_oci_t<T, NP, RES, BS>(S, io, nwg, ntiles, st, coop);
    }
};

hipError_t oci_occupancy(bool fp32, int np, bool res, int bs, int *blocks) {
    return dispatch(fp32, np, res, bs, OccF{blocks});
}

hipError_t launch_oci_step(const Slab &S, const StepIO &io, bool fp32, int np, bool res, int bs, int nwg, int ntiles,
                           hipStream_t st, bool cooperative) {
    return dispatch(fp32, np, res, bs, LaunchF{S, io, nwg, ntiles, st, cooperative});
}

hipError_t local_static_lds(bool fp32, int np, bool res, int bs, size_t *bytes) {
    return dispatch(fp32, np, res, bs, StaticLdsF{bytes});
}

hipError_t local_occupancy(bool fp32, int np, bool res, int bs, size_t dyn, int *blocks) {
    return dispatch(fp32, np, res, bs, OccLocalF{blocks, dyn});
}

hipError_t launch_oci_local(const Slab &S, const StepIO &io, bool fp32, int np, bool res, int bs, int nwg,
                            int ntiles, size_t dyn, hipStream_t st) {
    return dispatch(fp32, np, res, bs, LaunchLocalF{S, io, nwg, ntiles, dyn, st});
}

// broadcast: 0 = continue from the last iterate, 1 = start from the state
// on both time levels, 2 = decide on the device (the control block's flag).
hipError_t launch_begin(const Slab &S, const StepIO &io, int broadcast, hipStream_t st, int local_nwg) {
    hipLaunchKernelGGL(k_begin_step, dim3(1), dim3(1), 0, st, S);
    if (!S.wb) {   // the structured solve forms the constant part of b itself
        const size_t tot = (size_t)S.J * S.n;
        hipLaunchKernelGGL(k_const_rhs, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S, io);
    }
    if (broadcast) {
        const size_t tot = (size_t)S.J * S.G * S.N * 4;
        hipLaunchKernelGGL(k_broadcast_state, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S,
                           broadcast == 2 ? 1 : 0);
    }
    size_t tot = (size_t)S.J * S.G * 4;
    const size_t nex = (size_t)8 * local_nwg * S.N * S.G;
    if (nex > tot) tot = nex;
    hipLaunchKernelGGL(k_phi0, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S, local_nwg);
    if (broadcast == 2) hipLaunchKernelGGL(k_clear_bcast, dim3(1), dim3(1), 0, st, S);
    return hipGetLastError();
}

hipError_t launch_open(const Slab &S, const StepIO &io, hipStream_t st, int local_nwg) {
    size_t tot = (size_t)S.J * S.n;
    const size_t nex = (size_t)8 * local_nwg * S.N * S.G;
    if (nex > tot) tot = nex;
    hipLaunchKernelGGL(k_step_open, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S, io, local_nwg);
    return hipGetLastError();
}

hipError_t launch_end(const Slab &S, const StepIO &io, hipStream_t st) {
    size_t tot = (size_t)S.J * S.G * S.N;           // one thread per (j, g, m) ...
    if ((size_t)S.J * S.G * 4 > tot) tot = (size_t)S.J * S.G * 4;  // ... and per phi entry
    hipLaunchKernelGGL(k_end_step, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S, io);
    return hipGetLastError();
}

// Steps per LDS chunk of the sweep: two chunks of C x NG x 6 doubles in at
// most 128 KiB.
int si_chunk(const Slab &S) {
    const int NG = S.N * S.G;
    int C = (int)(131072 / (96 * (size_t)NG));
    if (C > 256) C = 256;
    if (C < 1) C = 1;
    if (C > S.J) C = S.J;
    return C;
}

hipError_t launch_si_iteration(const Slab &S, const StepIO &io, hipStream_t st) {
    const size_t rows = (size_t)S.J * S.G * S.N;
    hipLaunchKernelGGL(k_si_pre, dim3((unsigned)((rows + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S);
    const int C = si_chunk(S);
    const size_t dyn = (size_t)2 * C * S.N * S.G * 6 * 8;
    hipError_t e = hipFuncSetAttribute((const void *)&k_si_sweep, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_si_sweep, dim3(1), dim3(kSweepBlock), dyn, st, S, io, C);
    const size_t tot = (size_t)S.J * S.G * 4;
    hipLaunchKernelGGL(k_si_flux, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S);
    return hipGetLastError();
}

// The persistent SI loop: its dynamic LDS (the sweep ring) and how many of
// its 1024-thread workgroups fit on one CU (0: not launchable).
static size_t si_loop_lds(const Slab &S) { return (size_t)2 * si_chunk(S) * S.N * S.G * 6 * 8; }
int si_loop_occupancy(const Slab &S, bool multi) {
    const size_t dyn = si_loop_lds(S);
    const void *f = multi ? (const void *)&k_si_loop<true> : (const void *)&k_si_loop<false>;
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) != hipSuccess) return 0;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, kSweepBlock, dyn) != hipSuccess) return 0;
    return occ;
}
hipError_t launch_si_loop(const Slab &S, const StepIO &io, int nwg, hipStream_t st) {
    const size_t dyn = si_loop_lds(S);
    const bool multi = nwg > 1;
    const void *f = multi ? (const void *)&k_si_loop<true> : (const void *)&k_si_loop<false>;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
    if (multi) hipLaunchKernelGGL(k_si_loop<true>, dim3(nwg), dim3(kSweepBlock), dyn, st, S, io, si_chunk(S));
    else hipLaunchKernelGGL(k_si_loop<false>, dim3(1), dim3(kSweepBlock), dyn, st, S, io, si_chunk(S));
    return hipGetLastError();
}

}  // namespace oci
