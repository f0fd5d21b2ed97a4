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
//   5. meets every workgroup at a grid barrier; the last to arrive sums the
//      partials in a fixed order and applies the stopping rule, so the whole
//      decision stays on the device and repeats bit for bit.
// SI (Appendix A, Algorithm 1): one kernel sweeps all (group, angle) chains
// cell by cell with the lagged scattering source, a second forms phi and the
// norm and takes the decision (last-block reduction).
#include "oci_internal.hpp"

namespace oci {

constexpr int OK = 0, NOT_CONVERGED = 1, NONFINITE = 2;

// --------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Fixed-shape workgroup sum (same pairing every call, so deterministic).
__device__ inline double block_sum(double v, double *s_tmp) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s_tmp[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / 64; ++w) t += s_tmp[w];
    __syncthreads();
    return t;  // valid in thread 0
}

// Stopping rule of section 2.1 / Algorithms 1-2 applied to the new change e.
__device__ inline void decide(const Slab &S, double e) {
    Ctl *c = S.ctl;
    const int iters = c->iter + 1;
    const double e_prev = c->e_prev;
    const double rho = iters >= 2 ? e / e_prev : __builtin_nan("");
    int done = 0, status = OK;
    if (!isfinite(e)) {
        done = 1;
        status = NONFINITE;
    } else if (S.fixed_iters > 0) {
        done = iters >= S.fixed_iters;
    } else if (iters >= 2 && (e == 0.0 || e < S.tol * (1.0 - e / e_prev))) {
        done = 1;
    } else if (iters >= S.max_iters) {
        done = 1;
        status = NOT_CONVERGED;
    }
    c->iter = iters;
    c->e_last = e;
    c->rho = rho;
    c->e_prev = e;
    c->status = status;
    c->done = done;
}

// ------------------------------------------------------- step bookkeeping
// Before a step: the first iterate is where the previous step ended.
__global__ void k_begin_step(Slab S) {
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

// phi of the first iterate: one thread per (j, g, u), m summed in order.
__global__ __launch_bounds__(kBlock) void k_phi0(Slab S) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const size_t total = (size_t)S.J * S.G * 4;
    if (t >= total) return;
    const int b = S.ctl->base;
    const int u = t & 3;
    const size_t jg = t >> 2;
    const double *p = S.psi[b] + jg * S.N * 4 + u;
    double s = 0.0;
    for (int m = 0; m < S.N; ++m) s += S.w[m] * p[m * 4];
    S.phi[b][t] = s;
}

// psi of the first iterate from the state (both time levels).
__global__ __launch_bounds__(kBlock) void k_broadcast_state(Slab S) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const size_t total = (size_t)S.J * S.G * S.N * 4;
    if (t >= total) return;
    const int b = S.ctl->base;
    S.psi[b][t] = S.psi_prev[(t >> 2) * 2 + (t & 1)];
}

// After a step: time update psi_{k-1/2} <- psi_{k+1/2} and the outputs.
__global__ __launch_bounds__(kBlock) void k_end_step(Slab S, StepIO io) {
    const Ctl *c = S.ctl;
    const int fin = (c->base + c->iter) & 1;
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
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
    }
}

// -------------------------------------------------------------- OCI kernel
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 type; };
template <> struct Vec16<double> { typedef double2 type; };

__device__ inline float dot16(const float4 &a, const float4 &b) {
    return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
}
__device__ inline double dot16(const double2 &a, const double2 &b) { return a.x * b.x + a.y * b.y; }

template <int BS>
__device__ inline double block_sum_t(double v, double *s_tmp) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) s_tmp[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BS / 64; ++w) t += s_tmp[w];
    __syncthreads();
    return t;  // valid in thread 0
}

// Grid barrier over the co-resident workgroups of one launch, used once per
// iteration (index l).  Counters only grow during a step (reset before it),
// so a workgroup knows the target of barrier l without reading shared state:
// workgroups arrive at their group's counter; the last of a group arrives at
// the top counter; the last of all runs `last()` (the reduction and the
// stopping decision) and then raises the release flag to l + 1.  Each
// workgroup publishes its stores with one agent-scope release (its arrival)
// and waits with relaxed loads followed by one agent-scope acquire, so no
// cache maintenance happens inside the spin.  The spin is bounded: on expiry
// the control block's err flag is raised and every workgroup leaves its loop.
constexpr long kSpinLimit = 1L << 25;

template <typename F>
__device__ inline bool grid_barrier(const Slab &S, unsigned nwg, int l, int *s_flag, F last) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned wg = blockIdx.x;
        const unsigned grp = wg / kBarGroup;
        const unsigned ngrp = (nwg + kBarGroup - 1) / kBarGroup;
        const unsigned gsz = (grp + 1 == ngrp) ? nwg - grp * kBarGroup : kBarGroup;
        const uint64_t round = (uint64_t)l + 1;
        uint64_t *gc = S.bar + (size_t)(2 + grp) * kBarStride;
        const uint64_t og = __hip_atomic_fetch_add(gc, (uint64_t)1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        int is_last = 0;
        if (og + 1 == round * gsz) {
            const uint64_t ot = __hip_atomic_fetch_add(S.bar, (uint64_t)1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            is_last = (ot + 1 == round * ngrp);
        }
        s_flag[0] = is_last;
        s_flag[2] = 0;
    }
    __syncthreads();
    if (s_flag[0]) {
        last();
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(S.bar + kBarStride, (uint64_t)l + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else if (threadIdx.x == 0) {
        long spins = 0;
        while (__hip_atomic_load(S.bar + kBarStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (uint64_t)l + 1) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kSpinLimit) {
                __hip_atomic_store(&S.ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_flag[2] = 1;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (__hip_atomic_load(&S.ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) s_flag[2] = 1;
    }
    __syncthreads();
    return s_flag[2] == 0;
}

// The persistent OCI kernel.  T = float: refined path (FP32 inverse applied
// to the power-of-two scaled FP64 residual); T = double: plain FP64 path.
// NP: padded cell size (power of two >= n); RES: each thread keeps its row of
// the inverse in registers for the whole step (one tile per workgroup);
// BS: threads per workgroup.  At most 128 VGPRs (4 waves per SIMD).
template <typename T, int NP, bool RES, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4)))
void k_oci_step(Slab S, StepIO io, int ntiles) {
    constexpr bool REF = sizeof(T) == 4;
    constexpr int RPT = NP > BS ? NP / BS : 1;   // rows per thread
    constexpr int TPC = NP / RPT;                 // threads per cell
    constexpr int CPT = BS / TPC;                 // cells per tile
    constexpr int V = 16 / sizeof(T);
    constexpr int NV = NP / V;
    typedef typename Vec16<T>::type VT;

    __shared__ __align__(16) T s_vec[CPT][NP];
    __shared__ double s_psi[REF ? CPT : 1][REF ? NP : 1];
    __shared__ double s_wx[CPT][NP];
    __shared__ double s_phi[REF ? CPT : 1][REF ? NP / 2 : 1];
    __shared__ double s_mu[NP / 4], s_w[NP / 4];
    __shared__ double s_tmp[BS / 64 + 1];
    __shared__ double s_max[BS / 64];
    __shared__ int s_flag[4];

    const int tid = threadIdx.x;
    const int cl = tid / TPC;
    const int t = tid % TPC;
    const int J = S.J, N = S.N, G = S.G, n = S.n;
    const unsigned nwg = gridDim.x;
    const int wg = blockIdx.x;
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

            // (1) b (eq. rhs_sg) with the lagged incident edge; refined: the
            //     own iterate and its scalar flux into LDS for the residual
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = t + r * TPC;
                double b = 0.0;
                xold[r] = 0.0;
                if (live && i < n) {
                    const int g = i / (4 * N), m = (i >> 2) % N, u = i & 3;
                    const double dx = S.dx[j];
                    const double mu = s_mu[m];
                    const size_t jg = (size_t)j * G + g;
                    xold[r] = psi_in[(size_t)j * n + i];
                    if (io.q) b = 0.25 * dx * io.q[jg * 4 + u];
                    if (u < 2) b += dx / (2.0 * S.speed[g] * S.dt) * S.psi_prev[(jg * N + m) * 2 + u];
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
                // (2) FP64 residual r = b - A_j Psi^(l), matrix-free
                double rr[RPT];
                double mx = 0.0;
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int i = t + r * TPC;
                    double res = 0.0;
                    if (live && i < n) {
                        const int g = i / (4 * N), m = (i >> 2) % N, u = i & 3;
                        const double dx = S.dx[j];
                        const double mu = s_mu[m];
                        const size_t jg = (size_t)j * G + g;
                        const double a = dx / (S.speed[g] * S.dt);
                        const double d = 0.5 * (fabs(mu) + dx * S.sigma_t[jg]);
                        const double h = 0.5 * mu;
                        const double *p = &s_psi[cl][i & ~3];
                        double lp;
                        if (u == 0) lp = d * p[0] + h * p[1] + 0.5 * a * p[2];
                        else if (u == 1) lp = -h * p[0] + d * p[1] + 0.5 * a * p[3];
                        else if (u == 2) lp = -a * p[0] + (a + d) * p[2] + h * p[3];
                        else lp = -a * p[1] - h * p[2] + (a + d) * p[3];
                        double sc = 0.0;
                        for (int gp = 0; gp < G; ++gp) sc += S.sigma_s[jg * G + gp] * s_phi[cl][gp * 4 + u];
                        res = s_wx[cl][i] - lp + 0.25 * dx * sc;
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
        if (tid == 0) S.partials[wg] = wg_sum;

        // (5) grid barrier; the last workgroup reduces and decides
        const bool ok = grid_barrier(S, nwg, l, s_flag, [&]() {
            double v = 0.0;
            for (unsigned k = tid; k < nwg; k += BS) v += S.partials[k];
            const double tot = block_sum_t<BS>(v, s_tmp);
            if (tid == 0) decide(S, sqrt(tot));
        });
        if (!ok) break;
        if (tid == 0) s_flag[3] = __hip_atomic_load(&S.ctl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        if (s_flag[3]) break;
    }
}

// --------------------------------------------------------------- SI kernels
// One thread per (g, m) chain sweeping all cells in its direction.
__global__ __launch_bounds__(64) void k_si_sweep(Slab S, StepIO io) {
    const Ctl *c = S.ctl;
    if (c->done) return;
    const int cur = (c->base + c->iter) & 1;
    const int k = blockIdx.x * 64 + threadIdx.x;
    const int N = S.N, G = S.G, J = S.J;
    if (k >= N * G) return;
    const int g = k / N, m = k % N;
    const double mu = S.mu[m];
    const bool pos = mu > 0.0;
    const double *phi_in = S.phi[cur];
    double *psi_out = S.psi[cur ^ 1];
    double e0, e1;
    if (pos) {
        e0 = io.inc_l ? io.inc_l[(size_t)g * (N / 2) + (m - N / 2)] : 0.0;
        e1 = io.inc_l ? io.inc_l[((size_t)G + g) * (N / 2) + (m - N / 2)] : 0.0;
    } else {
        e0 = io.inc_r ? io.inc_r[(size_t)g * (N / 2) + m] : 0.0;
        e1 = io.inc_r ? io.inc_r[((size_t)G + g) * (N / 2) + m] : 0.0;
    }
    const double a2c = 1.0 / (2.0 * S.speed[g] * S.dt);
    for (int s = 0; s < J; ++s) {
        const int j = pos ? s : J - 1 - s;
        const size_t jg = (size_t)j * G + g;
        const double dx = S.dx[j];
        double d[4];
        for (int u = 0; u < 4; ++u) {
            double sc = 0.0;
            for (int gp = 0; gp < G; ++gp) sc += S.sigma_s[jg * G + gp] * phi_in[((size_t)j * G + gp) * 4 + u];
            d[u] = 0.25 * dx * ((io.q ? io.q[jg * 4 + u] : 0.0) + sc);
        }
        d[0] += dx * a2c * S.psi_prev[(jg * N + m) * 2 + 0];
        d[1] += dx * a2c * S.psi_prev[(jg * N + m) * 2 + 1];
        if (pos) { d[0] += mu * e0; d[2] += mu * e1; }
        else { d[1] -= mu * e0; d[3] -= mu * e1; }
        const double *Li = S.si_linv + (jg * N + m) * 16;
        double x[4];
        for (int r = 0; r < 4; ++r) x[r] = Li[r * 4 + 0] * d[0] + Li[r * 4 + 1] * d[1] + Li[r * 4 + 2] * d[2] + Li[r * 4 + 3] * d[3];
        double *o = psi_out + (jg * N + m) * 4;
        o[0] = x[0]; o[1] = x[1]; o[2] = x[2]; o[3] = x[3];
        e0 = pos ? x[1] : x[0];
        e1 = pos ? x[3] : x[2];
    }
}

// phi of the sweep, its change, and the decision (last block to finish).
__global__ __launch_bounds__(kBlock) void k_si_flux(Slab S) {
    __shared__ double s_tmp[kBlock / 64 + 1];
    __shared__ int s_last;
    Ctl *c = S.ctl;
    if (c->done) return;
    const int cur = (c->base + c->iter) & 1;
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const size_t total = (size_t)S.J * S.G * 4;
    double dsq = 0.0;
    if (t < total) {
        const int u = t & 3;
        const double *p = S.psi[cur ^ 1] + (t >> 2) * S.N * 4 + u;
        double f = 0.0;
        for (int m = 0; m < S.N; ++m) f += S.w[m] * p[m * 4];
        const double f0 = S.phi[cur][t];
        S.phi[cur ^ 1][t] = f;
        dsq = (f - f0) * (f - f0);
    }
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

hipError_t launch_begin(const Slab &S, bool broadcast_state, hipStream_t st) {
    hipLaunchKernelGGL(k_begin_step, dim3(1), dim3(1), 0, st, S);
    if (broadcast_state) {
        const size_t tot = (size_t)S.J * S.G * S.N * 4;
        hipLaunchKernelGGL(k_broadcast_state, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S);
    }
    const size_t tot = (size_t)S.J * S.G * 4;
    hipLaunchKernelGGL(k_phi0, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S);
    return hipGetLastError();
}

hipError_t launch_end(const Slab &S, const StepIO &io, hipStream_t st) {
    size_t tot = (size_t)S.J * S.G * S.N;           // one thread per (j, g, m) ...
    if ((size_t)S.J * S.G * 4 > tot) tot = (size_t)S.J * S.G * 4;  // ... and per phi entry
    hipLaunchKernelGGL(k_end_step, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S, io);
    return hipGetLastError();
}

hipError_t launch_si_iteration(const Slab &S, const StepIO &io, hipStream_t st) {
    const int chains = S.N * S.G;
    hipLaunchKernelGGL(k_si_sweep, dim3((chains + 63) / 64), dim3(64), 0, st, S, io);
    const size_t tot = (size_t)S.J * S.G * 4;
    hipLaunchKernelGGL(k_si_flux, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S);
    return hipGetLastError();
}

size_t si_flux_blocks(const Slab &S) { return ((size_t)S.J * S.G * 4 + kBlock - 1) / kBlock; }

}  // namespace oci
