// oci_api.hip -- host side of the liboci C ABI (include/oci.h): argument
// validation, quadrature, workspace layout and the launch sequence of setup
// and time steps.  Every step of the method runs in the device kernels of
// oci_setup.hip and oci_step.hip; nothing here computes on the host beyond
// the quadrature rule and launch geometry.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/oci.h"
#include "oci_internal.hpp"

namespace oci {
hipError_t launch_setup(const Slab &S, bool fp32, hipStream_t st);
hipError_t launch_begin(const Slab &S, const StepIO &io, int broadcast, hipStream_t st, int local_nwg);
hipError_t launch_open(const Slab &S, const StepIO &io, hipStream_t st, int local_nwg);
hipError_t launch_end(const Slab &S, const StepIO &io, hipStream_t st);
hipError_t launch_oci_step(const Slab &S, const StepIO &io, bool fp32, int np, bool res, int bs, int nwg, int ntiles,
                           hipStream_t st, bool cooperative);
hipError_t oci_occupancy(bool fp32, int np, bool res, int bs, int *blocks);
hipError_t local_static_lds(bool fp32, int np, bool res, int bs, size_t *bytes);
hipError_t local_occupancy(bool fp32, int np, bool res, int bs, size_t dyn, int *blocks);
hipError_t launch_oci_local(const Slab &S, const StepIO &io, bool fp32, int np, bool res, int bs, int nwg,
                            int ntiles, size_t dyn, hipStream_t st);
bool resident_supported(bool fp32, int np);
bool block_supported(int bs);
int si_loop_occupancy(const Slab &S, bool multi);
hipError_t launch_si_loop(const Slab &S, const StepIO &io, int nwg, hipStream_t st);
hipError_t launch_si_iteration(const Slab &S, const StepIO &io, hipStream_t st);
hipError_t batch_occupancy(bool fp32, int *blocks);
int batch_block();
hipError_t launch_batch_step(const BatchEntry *tab, int nslab, int nwg, bool fp32, bool structured, bool staged,
                             bool broadcast, hipStream_t st, bool coop);
hipError_t wb_batch_occupancy(bool staged, int *blocks);
hipError_t launch_flag_broadcast(const Slab &S, hipStream_t st);
hipError_t launch_wb_setup(const Slab &S, hipStream_t st);
hipError_t launch_checkpoint(const Slab &S, double *out, const double *in, bool from_state, hipStream_t st);
hipError_t launch_oci_wb(const Slab &S, const StepIO &io, int nwg, int ntiles, bool staged, hipStream_t st);
hipError_t wb_occupancy(int N, int G, bool staged, int *blocks);
bool wb_staged(long J, int N, int G);
int wb_cells_per_tile(int N, int G);
int wb_block();
}  // namespace oci

using namespace oci;

struct oci_handle {
    oci_desc d;            // scalars only (host pointers cleared)
    int n, np;             // 4 N G and its padded power of two
    bool fp32;
    hipStream_t st;
    int device, num_cu;
    Slab S;
    unsigned char *ws;
    size_t ws_bytes;
    int nwg, ntiles;       // OCI persistent launch geometry
    int block;             // threads per workgroup of the OCI kernel
    int max_wg;            // cap on its workgroups (0: none; testing override)
    bool resident;
    bool local;            // workgroup-local kernel (iterate kept in LDS)
    bool structured;       // structured cell solve (OCI_SOLVE_STRUCTURED)
    bool wb_staged;        // ... with the staged iteration body (shape permitting)
    size_t dyn_lds;        // its dynamic LDS bytes
    bool need_broadcast;   // next step starts from psi_prev on both levels
    bool profiling;
    hipGraphExec_t graph;              // steps captured by oci_capture_steps
    std::vector<hipEvent_t> ev_pool;   // recorded pairs: [2k] start, [2k+1] stop
    size_t ev_used;
    int32_t prof_steps;                // time steps those pairs cover
};

// Two events bracketing the iteration kernels of one step (instrumentation).
static hipEvent_t prof_event(oci_handle *h) {
    if (h->ev_used == h->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->ev_pool.push_back(e);
    }
    return h->ev_pool[h->ev_used++];
}

// ------------------------------------------------------------- validation
static bool finite_nonneg(const double *a, size_t n, bool strictly_pos) {
    for (size_t i = 0; i < n; ++i) {
        if (!isfinite(a[i])) return false;
        if (strictly_pos ? !(a[i] > 0.0) : !(a[i] >= 0.0)) return false;
    }
    return true;
}

static int pad_pow2(int n) {
    int p = 8;
    while (p < n) p <<= 1;
    return p;
}

static int check_desc(const oci_desc *d) {
    if (!d) return OCI_ERR_INVALID;
    if (d->J < 1 || d->N < 2 || (d->N & 1) || d->G < 1) return OCI_ERR_INVALID;
    if ((long)4 * d->N * d->G > kMaxN) return OCI_ERR_UNSUPPORTED;
    if (!d->dx || !d->sigma_t || !d->sigma_s || !d->speed) return OCI_ERR_INVALID;
    if (!(d->dt > 0.0) || !isfinite(d->dt)) return OCI_ERR_INVALID;
    if (!(d->tol >= 0.0) || !isfinite(d->tol)) return OCI_ERR_INVALID;
    if (d->max_iters < 1 || d->fixed_iters < 0) return OCI_ERR_INVALID;
    if (d->precision != OCI_FP64 && d->precision != OCI_FP32_REFINED) return OCI_ERR_INVALID;
    if (d->norm != OCI_NORM_SCALAR && d->norm != OCI_NORM_ANGULAR) return OCI_ERR_INVALID;
    if (d->solver != OCI_SOLVE_DENSE && d->solver != OCI_SOLVE_STRUCTURED) return OCI_ERR_INVALID;
    if (d->ordering != OCI_ORDER_JACOBI && d->ordering != OCI_ORDER_RED_BLACK) return OCI_ERR_INVALID;
    if (d->boundary != OCI_BOUNDARY_INCIDENT && d->boundary != OCI_BOUNDARY_PERIODIC) return OCI_ERR_INVALID;
    if (d->solver == OCI_SOLVE_STRUCTURED &&
        (d->precision != OCI_FP64 || d->norm != OCI_NORM_SCALAR || d->G > 8))
        return OCI_ERR_UNSUPPORTED;
    if (d->solver != OCI_SOLVE_STRUCTURED && (d->ordering != OCI_ORDER_JACOBI || d->boundary != OCI_BOUNDARY_INCIDENT))
        return OCI_ERR_UNSUPPORTED;
    const size_t J = d->J, G = d->G;
    if (!finite_nonneg(d->dx, J, true)) return OCI_ERR_INVALID;
    if (!finite_nonneg(d->sigma_t, J * G, false)) return OCI_ERR_INVALID;
    if (!finite_nonneg(d->sigma_s, J * G * G, false)) return OCI_ERR_INVALID;
    if (!finite_nonneg(d->speed, G, true)) return OCI_ERR_INVALID;
    return OCI_OK;
}

// ------------------------------------------------------------- quadrature
// Gauss-Legendre nodes (ascending) and weights: Newton's method on P_N from
// Tricomi's asymptotic guess, weights 2 / ((1 - x^2) P_N'(x)^2); the negative
// half mirrors the positive half so the rule is exactly symmetric.
static void gauss_legendre(int N, double *mu, double *w) {
    const int h = N / 2;
    for (int k = 1; k <= h; ++k) {
        const double th = M_PI * (4.0 * k - 1.0) / (4.0 * N + 2.0);
        double x = (1.0 - 1.0 / (8.0 * N * N) + 1.0 / (8.0 * (double)N * N * N)) * cos(th);
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double pm = 1.0, p = x;
            for (int l = 2; l <= N; ++l) {
                const double pn = ((2 * l - 1) * x * p - (l - 1) * pm) / l;
                pm = p;
                p = pn;
            }
            dp = N * (x * p - pm) / (x * x - 1.0);
            const double dx = p / dp;
            x -= dx;
            if (fabs(dx) <= 1e-16) break;
        }
        double pm = 1.0, p = x;
        for (int l = 2; l <= N; ++l) {
            const double pn = ((2 * l - 1) * x * p - (l - 1) * pm) / l;
            pm = p;
            p = pn;
        }
        dp = N * (x * p - pm) / (x * x - 1.0);
        const double wk = 2.0 / ((1.0 - x * x) * dp * dp);
        // k = 1 is the largest root
        mu[N - k] = x;
        w[N - k] = wk;
        mu[k - 1] = -x;
        w[k - 1] = wk;
    }
}

// --------------------------------------------------------------- workspace
struct Layout {
    size_t ctl, bar, mu, w, dx, st, ss, sp, X, psi0, psi1, phi0, phi1, prev, crhs, exch, linv, resp, msw, alpha, ein,
        part, wb, edge, total;
    int bar_groups;
};

static int device_cus() {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) return 256;
    return cu;
}

static Layout layout(const oci_desc *d, int num_cu) {
    const size_t J = d->J, N = d->N, G = d->G, n = 4 * N * G;
    const size_t np = pad_pow2((int)n);
    const size_t es = d->precision == OCI_FP32_REFINED ? 4 : 8;
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    L.ctl = take(sizeof(Ctl));
    L.bar_groups = num_cu * 8;  // enough for any arrival-group size >= 1
    L.bar = take((size_t)(2 + L.bar_groups) * kBarStride * 8);
    L.mu = take(N * 8);
    L.w = take(N * 8);
    L.dx = take(J * 8);
    L.st = take(J * G * 8);
    L.ss = take(J * G * G * 8);
    L.sp = take(G * 8);
    const bool structured = d->solver == OCI_SOLVE_STRUCTURED;
    L.X = take(structured ? 0 : J * np * np * es);
    L.psi0 = take(J * n * 8);
    L.psi1 = take(J * n * 8);
    L.phi0 = take(J * G * 4 * 8);
    L.phi1 = take(J * G * 4 * 8);
    L.prev = take(J * n / 2 * 8);
    L.crhs = take(J * n * 8);
    L.exch = take((size_t)2 * num_cu * 8 * 2 * N * G * 16);
    L.linv = take(J * G * N * 16 * 8);
    L.resp = take(J * G * N * 8 * 8);
    L.msw = take(J * G * N * 4 * 8);
    L.alpha = take(J * G * N * 2 * 8);
    L.ein = take(J * G * N * 2 * 8);
    const size_t si_blocks = (J * G * 4 + kBlock - 1) / kBlock;
    size_t parts = (size_t)num_cu * 8 * kPartSlots;   // the local kernel's ring of partial sums
    if (si_blocks > parts) parts = si_blocks;
    L.part = take(parts * 8);
    L.wb = take(structured ? J * 16 * G * G * 8 : 0);   // [J][4G][2G] complex
    L.edge = take(structured ? 2 * J * N * G * 2 * 8 : 0);
    L.total = o;
    return L;
}

extern "C" int oci_workspace_bytes(const oci_desc *desc, size_t *bytes) {
    const int rc = check_desc(desc);
    if (rc) return rc;
    if (!bytes) return OCI_ERR_INVALID;
    *bytes = layout(desc, device_cus()).total;
    return OCI_OK;
}

#define HIPCHECK(x)                                  \
    do {                                             \
        if ((x) != hipSuccess) return OCI_ERR_HIP;   \
    } while (0)

// Launch geometry of the persistent OCI kernel for one block size: prefer
// the workgroup-local kernel (iterate in LDS) with register-resident
// inverse rows, then local with streamed rows, then the global-memory kernel
// (resident, then streamed).  One tile = block / (threads per cell) cells.
static int configure_structured(oci_handle *h, int gsz) {
    const int cpt = wb_cells_per_tile(h->d.N, h->d.G);
    const long cells = h->S.ordering == OCI_ORDER_RED_BLACK ? (h->d.J + 1) / 2 : h->d.J;   // per half-sweep
    const long ntiles = (cells + cpt - 1) / cpt;
    long cap = (long)h->num_cu * 8;   // partial-sum and barrier slots in the workspace
    if (h->max_wg > 0 && h->max_wg < cap) cap = h->max_wg;
    int occ = 0;
    if (wb_occupancy(h->d.N, h->d.G, h->wb_staged, &occ) != hipSuccess || occ < 1) return OCI_ERR_HIP;
    if ((long)occ * h->num_cu < cap) cap = (long)occ * h->num_cu;
    const long nwg = ntiles < cap ? ntiles : cap;
    h->block = wb_block();
    h->ntiles = (int)ntiles;
    h->nwg = (int)nwg;
    h->local = false;
    h->resident = false;
    h->dyn_lds = 0;
    h->S.bar_gsz = gsz;
    h->S.bar_groups = (h->nwg + gsz - 1) / gsz;
    return OCI_OK;
}

static int configure(oci_handle *h, int block, bool allow_local, bool allow_res, int gsz) {
    if (h->structured) return configure_structured(h, gsz);
    const int num_cu = h->num_cu;
    const int N = h->d.N, G = h->d.G;
    const int rpt = h->np > block ? h->np / block : 1;
    const int tpc = h->np / rpt;
    const int cpt = block / tpc;
    const long ntiles = (h->d.J + cpt - 1) / cpt;
    long wg_cap = (long)num_cu * 8;  // partial-sum and exchange slots in the workspace
    if (h->max_wg > 0 && h->max_wg < wg_cap) wg_cap = h->max_wg;
    int occ_res = 0, occ = 0;
    if (oci_occupancy(h->fp32, h->np, false, block, &occ) != hipSuccess || occ < 1) return OCI_ERR_HIP;
    bool local = false, res = false;
    long nwg = 0;
    size_t dyn_lds = 0;
    // dynamic LDS of the local kernel: cells x (n + 4G) (kResidentCopies
    // times with resident rows) + internal tile boundaries x 2NG doubles
    // (+ the flux scratch)
    auto try_local = [&](bool r) -> bool {
        size_t stat = 0;
        if (local_static_lds(h->fp32, h->np, r, block, &stat) != hipSuccess) return false;
        const size_t lds_max = 160 * 1024;
        int occ0 = 0;
        if (local_occupancy(h->fp32, h->np, r, block, 0, &occ0) != hipSuccess || occ0 < 1) return false;
        long w = ntiles < (long)occ0 * num_cu ? ntiles : (long)occ0 * num_cu;
        if (w > wg_cap) w = wg_cap;
        for (int it = 0; it < 8 && w >= 1; ++it) {
            const long tpw = (ntiles + w - 1) / w;
            // resident rows keep kResidentCopies copies of the range's Psi and
            // phi; streamed rows sum phi through LDS ([cells per tile][np])
            // unless N is a power of two up to 16 with one row per thread
            const bool wx = !r && !(rpt == 1 && (N & (N - 1)) == 0 && N <= 16);
            const size_t dyn = ((size_t)(r ? kResidentCopies : 1) * tpw * cpt * (h->n + 4 * G) +
                                (size_t)(r ? tpw : tpw - 1) * 2 * N * G + (wx ? (size_t)cpt * h->np : 0)) * 8;
            if (stat + dyn > lds_max) return false;
            int o = 0;
            if (local_occupancy(h->fp32, h->np, r, block, dyn, &o) != hipSuccess || o < 1) return false;
            if ((long)o * num_cu >= w) {
                if (r && w != ntiles) return false;
                nwg = w;
                dyn_lds = dyn;
                return true;
            }
            if (r) return false;
            w = (long)o * num_cu;
        }
        return false;
    };
    if (allow_local && allow_res && resident_supported(h->fp32, h->np) && try_local(true)) {
        local = res = true;
    } else if (allow_local && try_local(false)) {
        local = true;
    } else if (allow_res && resident_supported(h->fp32, h->np) &&
               oci_occupancy(h->fp32, h->np, true, block, &occ_res) == hipSuccess &&
               (long)occ_res * num_cu >= ntiles && ntiles <= wg_cap) {
        res = true;
        nwg = ntiles;
    } else {
        const long cap = (long)occ * num_cu;
        nwg = ntiles < cap ? ntiles : cap;
    }
    if (nwg > wg_cap) nwg = wg_cap;
    if (nwg < 1) return OCI_ERR_UNSUPPORTED;
    h->block = block;
    h->ntiles = (int)ntiles;
    h->nwg = (int)nwg;
    h->local = local;
    h->resident = res;
    h->dyn_lds = dyn_lds;
    h->S.bar_gsz = gsz;
    h->S.bar_groups = (h->nwg + gsz - 1) / gsz;  // counters the barrier uses
    return OCI_OK;
}

extern "C" int oci_setup(const oci_desc *desc, void *workspace_dev, size_t workspace_bytes, void *stream,
                         oci_handle **out) {
    int rc = check_desc(desc);
    if (rc) return rc;
    if (!out) return OCI_ERR_INVALID;
    *out = nullptr;
    const int num_cu = device_cus();
    const Layout L = layout(desc, num_cu);
    if (!workspace_dev || ((uintptr_t)workspace_dev & 255) || workspace_bytes < L.total) return OCI_ERR_WORKSPACE;

    oci_handle *h = new (std::nothrow) oci_handle();
    if (!h) return OCI_ERR_HIP;
    h->d = *desc;
    h->d.dx = h->d.sigma_t = h->d.sigma_s = h->d.speed = nullptr;
    h->n = 4 * desc->N * desc->G;
    h->np = pad_pow2(h->n);
    h->fp32 = desc->precision == OCI_FP32_REFINED;
    h->st = (hipStream_t)stream;
    h->num_cu = num_cu;
    h->ws = (unsigned char *)workspace_dev;
    h->ws_bytes = workspace_bytes;
    if (hipGetDevice(&h->device) != hipSuccess) { delete h; return OCI_ERR_HIP; }

    unsigned char *ws = h->ws;
    Slab &S = h->S;
    S.J = desc->J; S.N = desc->N; S.G = desc->G; S.n = h->n; S.np = h->np;
    S.dt = desc->dt;
    S.mu = (const double *)(ws + L.mu);
    S.w = (const double *)(ws + L.w);
    S.dx = (const double *)(ws + L.dx);
    S.sigma_t = (const double *)(ws + L.st);
    S.sigma_s = (const double *)(ws + L.ss);
    S.speed = (const double *)(ws + L.sp);
    S.X = ws + L.X;
    S.psi[0] = (double *)(ws + L.psi0);
    S.psi[1] = (double *)(ws + L.psi1);
    S.phi[0] = (double *)(ws + L.phi0);
    S.phi[1] = (double *)(ws + L.phi1);
    S.psi_prev = (double *)(ws + L.prev);
    S.crhs = (double *)(ws + L.crhs);
    S.exch = (double *)(ws + L.exch);
    S.si_linv = (double *)(ws + L.linv);
    S.si_resp = (double *)(ws + L.resp);
    S.si_msw = (double *)(ws + L.msw);
    S.si_alpha = (double *)(ws + L.alpha);
    S.si_ein = (double *)(ws + L.ein);
    S.partials = (double *)(ws + L.part);
    S.wb = desc->solver == OCI_SOLVE_STRUCTURED ? (double *)(ws + L.wb) : nullptr;
    S.edge = desc->solver == OCI_SOLVE_STRUCTURED ? (double *)(ws + L.edge) : nullptr;
    h->structured = S.wb != nullptr;
    // the staged structured body where the shape allows it; OCI_WB_DIRECT=1
    // selects the direct body (testing both on one shape)
    const char *direct = getenv("OCI_WB_DIRECT");
    h->wb_staged = h->structured && wb_staged(desc->J, desc->N, desc->G) && !(direct && atoi(direct) == 1);
    S.ctl = (Ctl *)(ws + L.ctl);
    S.bar = (uint64_t *)(ws + L.bar);
    S.bar_groups = L.bar_groups;
    S.bar_gsz = kBarGroup;
    if (const char *env = getenv("OCI_BAR_GROUP")) {
        const int g = atoi(env);
        if (g >= 1 && g <= 4096) S.bar_gsz = g;
    }
    S.zero_cell = -1;
    S.ordering = desc->ordering;
    S.periodic = desc->boundary == OCI_BOUNDARY_PERIODIC ? 1 : 0;
    S.hist = nullptr;
    S.hist_cap = 0;
    if (const char *env = getenv("OCI_TEST_ZERO_PIVOT_CELL")) {   // test hook (singular-cell path)
        const int j = atoi(env);
        if (j >= 0 && j < desc->J) S.zero_cell = j;
    }
    S.tol = desc->tol;
    S.max_iters = desc->max_iters;
    S.fixed_iters = desc->fixed_iters;
    S.norm = desc->norm;
    S.refined = h->fp32 ? 1 : 0;

    double *mu = (double *)malloc(sizeof(double) * desc->N * 2);
    if (!mu) { oci_destroy(h); return OCI_ERR_HIP; }
    gauss_legendre(desc->N, mu, mu + desc->N);
    const size_t J = desc->J, G = desc->G;
    hipError_t e = hipSuccess;
    hipStream_t st = h->st;
    auto up = [&](size_t off, const void *src, size_t bytes) {
        if (e == hipSuccess) e = hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, st);
    };
    up(L.mu, mu, desc->N * 8);
    up(L.w, mu + desc->N, desc->N * 8);
    up(L.dx, desc->dx, J * 8);
    up(L.st, desc->sigma_t, J * G * 8);
    up(L.ss, desc->sigma_s, J * G * G * 8);
    up(L.sp, desc->speed, G * 8);
    if (e == hipSuccess) e = hipMemsetAsync(ws + L.ctl, 0, L.mu - L.ctl, st);
    if (e == hipSuccess) e = hipMemsetAsync(ws + L.psi0, 0, L.prev + J * h->n / 2 * 8 - L.psi0, st);
    if (e == hipSuccess) e = launch_setup(S, h->fp32, st);
    if (e == hipSuccess && h->structured) e = launch_wb_setup(S, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    free(mu);
    if (e != hipSuccess) { oci_destroy(h); return OCI_ERR_HIP; }
    Ctl c;
    if (hipMemcpy(&c, S.ctl, sizeof(Ctl), hipMemcpyDeviceToHost) != hipSuccess) { oci_destroy(h); return OCI_ERR_HIP; }
    if (c.singular) { oci_destroy(h); return OCI_ERR_SINGULAR; }

    // persistent launch geometry; environment overrides: OCI_BLOCK (256 or
    // 1024), OCI_MODE=global, OCI_NO_RESIDENT=1, OCI_MAX_WG (a cap on the
    // workgroups, so that each owns several tiles; OCI_BAR_GROUP read above)
    if (const char *env = getenv("OCI_MAX_WG")) {
        const int w = atoi(env);
        if (w >= 1) h->max_wg = w;
    }
    int block = 1024;
    if (const char *env = getenv("OCI_BLOCK")) {
        const int b = atoi(env);
        if (block_supported(b)) block = b;
    }
    const char *nores = getenv("OCI_NO_RESIDENT");
    const char *mode = getenv("OCI_MODE");
    rc = configure(h, block, !(mode && strcmp(mode, "global") == 0), !(nores && atoi(nores)), S.bar_gsz);
    if (rc) { oci_destroy(h); return rc; }
    h->need_broadcast = true;
    *out = h;
    return OCI_OK;
}

// ------------------------------------------------------- static workspace
// The device memory of oci_setup_static: one fixed array per device, created
// when the library's code object is loaded on that device and held until the
// process ends.  Host code never uses the array's name as an address: the
// device address is looked up once per device (hipGetSymbolAddress, with that
// device current) and kept in g_scratch.
constexpr size_t kStaticWorkspaceBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];
constexpr int kMaxDevices = 64;
static void *g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

static void *static_workspace(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

extern "C" int oci_setup_static(const oci_desc *desc, void *stream, oci_handle **out) {
    const int rc = check_desc(desc);
    if (rc) return rc;
    if (!out) return OCI_ERR_INVALID;
    *out = nullptr;
    if (layout(desc, device_cus()).total > kStaticWorkspaceBytes) return OCI_ERR_TOO_LARGE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return OCI_ERR_HIP;
    void *ws = static_workspace(dev);
    if (!ws) return OCI_ERR_HIP;
    return oci_setup(desc, ws, kStaticWorkspaceBytes, stream, out);
}

extern "C" int oci_set_state(oci_handle *h, const double *psi_prev_dev) {
    if (!h) return OCI_ERR_INVALID;
    const size_t bytes = (size_t)h->d.J * h->n / 2 * 8;
    hipError_t e = psi_prev_dev ? hipMemcpyAsync(h->S.psi_prev, psi_prev_dev, bytes, hipMemcpyDeviceToDevice, h->st)
                                : hipMemsetAsync(h->S.psi_prev, 0, bytes, h->st);
    if (e != hipSuccess) return OCI_ERR_HIP;
    h->need_broadcast = true;
    return OCI_OK;
}

extern "C" int oci_get_state(const oci_handle *h, double *psi_prev_dev) {
    if (!h || !psi_prev_dev) return OCI_ERR_INVALID;
    const size_t bytes = (size_t)h->d.J * h->n / 2 * 8;
    if (hipMemcpyAsync(psi_prev_dev, h->S.psi_prev, bytes, hipMemcpyDeviceToDevice, h->st) != hipSuccess)
        return OCI_ERR_HIP;
    return OCI_OK;
}

extern "C" int oci_get_checkpoint(const oci_handle *h, double *psi_prev_dev, double *psi_iter_dev) {
    if (!h || !psi_prev_dev || !psi_iter_dev) return OCI_ERR_INVALID;
    const size_t bytes = (size_t)h->d.J * h->n / 2 * 8;
    if (hipMemcpyAsync(psi_prev_dev, h->S.psi_prev, bytes, hipMemcpyDeviceToDevice, h->st) != hipSuccess)
        return OCI_ERR_HIP;
    if (launch_checkpoint(h->S, psi_iter_dev, nullptr, h->need_broadcast, h->st) != hipSuccess) return OCI_ERR_HIP;
    return OCI_OK;
}

extern "C" int oci_set_checkpoint(oci_handle *h, const double *psi_prev_dev, const double *psi_iter_dev) {
    if (!h || !psi_prev_dev || !psi_iter_dev) return OCI_ERR_INVALID;
    const size_t bytes = (size_t)h->d.J * h->n / 2 * 8;
    if (hipMemcpyAsync(h->S.psi_prev, psi_prev_dev, bytes, hipMemcpyDeviceToDevice, h->st) != hipSuccess)
        return OCI_ERR_HIP;
    if (launch_checkpoint(h->S, nullptr, psi_iter_dev, false, h->st) != hipSuccess) return OCI_ERR_HIP;
    h->need_broadcast = false;
    return OCI_OK;
}

static int check_step_args(oci_handle *h, double *phi_out_dev, oci_step_info *info_dev) {
    if (!h || !phi_out_dev || !info_dev) return OCI_ERR_INVALID;
    return OCI_OK;
}

extern "C" int oci_step(oci_handle *h, const double *q_dev, const double *inc_left_dev, const double *inc_right_dev,
                        double *phi_out_dev, double *psi_out_dev, oci_step_info *info_dev) {
    int rc = check_step_args(h, phi_out_dev, info_dev);
    if (rc) return rc;
    StepIO io{q_dev, inc_left_dev, inc_right_dev, phi_out_dev, psi_out_dev, info_dev};
    if (h->need_broadcast || !h->local) HIPCHECK(launch_begin(h->S, io, h->need_broadcast, h->st, h->local ? h->nwg : 0));
    else HIPCHECK(launch_open(h->S, io, h->st, h->nwg));
    h->need_broadcast = false;
    hipEvent_t e0 = h->profiling ? prof_event(h) : nullptr, e1 = h->profiling ? prof_event(h) : nullptr;
    if (e0) HIPCHECK(hipEventRecord(e0, h->st));
    if (h->structured)
        HIPCHECK(launch_oci_wb(h->S, io, h->nwg, h->ntiles, h->wb_staged, h->st));
    else if (h->local)
        HIPCHECK(launch_oci_local(h->S, io, h->fp32, h->np, h->resident, h->block, h->nwg, h->ntiles, h->dyn_lds, h->st));
    else
        HIPCHECK(launch_oci_step(h->S, io, h->fp32, h->np, h->resident, h->block, h->nwg, h->ntiles, h->st, true));
    if (e1) HIPCHECK(hipEventRecord(e1, h->st));
    if (e1) h->prof_steps += 1;
    HIPCHECK(launch_end(h->S, io, h->st));
    return OCI_OK;
}

extern "C" int oci_run_steps(oci_handle *h, int32_t nsteps, const double *q_dev, int64_t q_stride,
                             const double *inc_left_dev, const double *inc_right_dev, int64_t inc_stride,
                             double *phi_out_dev, double *psi_out_dev, oci_step_info *info_dev) {
    if (nsteps < 1 || q_stride < 0 || inc_stride < 0) return OCI_ERR_INVALID;
    int rc = check_step_args(h, phi_out_dev, info_dev);
    if (rc) return rc;
    const size_t phi_stride = (size_t)h->d.J * h->d.G * 4;
    auto step_src = [](const double *p, int64_t stride, int k) { return p ? p + (size_t)k * stride : p; };
    if (!(h->local && h->resident) || nsteps == 1) {
        for (int k = 0; k < nsteps; ++k) {
            rc = oci_step(h, step_src(q_dev, q_stride, k), step_src(inc_left_dev, inc_stride, k),
                          step_src(inc_right_dev, inc_stride, k), phi_out_dev + k * phi_stride,
                          k == nsteps - 1 ? psi_out_dev : nullptr, info_dev + k);
            if (rc) return rc;
        }
        return OCI_OK;
    }
    // one launch of the register-resident kernel for all steps; the first
    // step opens and the last closes as in oci_step, the others turn over
    // inside the kernel (each taking its own sources through the strides)
    StepIO io{q_dev, inc_left_dev, inc_right_dev, phi_out_dev, nullptr, info_dev, nsteps, 0, q_stride, inc_stride};
    if (h->need_broadcast) HIPCHECK(launch_begin(h->S, io, 1, h->st, h->nwg));
    else HIPCHECK(launch_open(h->S, io, h->st, h->nwg));
    h->need_broadcast = false;
    hipEvent_t e0 = h->profiling ? prof_event(h) : nullptr, e1 = h->profiling ? prof_event(h) : nullptr;
    if (e0) HIPCHECK(hipEventRecord(e0, h->st));
    HIPCHECK(launch_oci_local(h->S, io, h->fp32, h->np, h->resident, h->block, h->nwg, h->ntiles, h->dyn_lds, h->st));
    if (e1) HIPCHECK(hipEventRecord(e1, h->st));
    if (e1) h->prof_steps += nsteps;
    const int kl = nsteps - 1;
    const StepIO last{step_src(q_dev, q_stride, kl), step_src(inc_left_dev, inc_stride, kl),
                      step_src(inc_right_dev, inc_stride, kl), phi_out_dev + kl * phi_stride, psi_out_dev,
                      info_dev + kl, 1};
    HIPCHECK(launch_end(h->S, last, h->st));
    return OCI_OK;
}

// The iteration kernels of one step as oci_step launches them, with the
// opening deciding on the device whether to start from the state (steps in
// a graph cannot ask the host), and no cooperative launch (not capturable).
static hipError_t enqueue_step_for_graph(oci_handle *h, const StepIO &io) {
    hipError_t e = launch_begin(h->S, io, 2, h->st, h->local ? h->nwg : 0);
    if (e != hipSuccess) return e;
    if (h->structured) e = launch_oci_wb(h->S, io, h->nwg, h->ntiles, h->wb_staged, h->st);
    else if (h->local)
        e = launch_oci_local(h->S, io, h->fp32, h->np, h->resident, h->block, h->nwg, h->ntiles, h->dyn_lds, h->st);
    else e = launch_oci_step(h->S, io, h->fp32, h->np, h->resident, h->block, h->nwg, h->ntiles, h->st, false);
    if (e != hipSuccess) return e;
    return launch_end(h->S, io, h->st);
}

extern "C" int oci_capture_steps(oci_handle *h, int32_t n_steps, const double *const *q_dev,
                                 const double *const *inc_left_dev, const double *const *inc_right_dev,
                                 double *const *phi_out_dev, double *const *psi_out_dev, oci_step_info *info_dev) {
    if (!h || n_steps < 1 || !phi_out_dev || !info_dev || !h->st) return OCI_ERR_INVALID;
    for (int k = 0; k < n_steps; ++k)
        if (!phi_out_dev[k]) return OCI_ERR_INVALID;
    if (h->graph) { (void)hipGraphExecDestroy(h->graph); h->graph = nullptr; }
    HIPCHECK(hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < n_steps && e == hipSuccess; ++k) {
        const StepIO io{q_dev ? q_dev[k] : nullptr, inc_left_dev ? inc_left_dev[k] : nullptr,
                        inc_right_dev ? inc_right_dev[k] : nullptr, phi_out_dev[k],
                        psi_out_dev ? psi_out_dev[k] : nullptr, info_dev + k, 1};
        e = enqueue_step_for_graph(h, io);
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(h->st, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return OCI_ERR_HIP;
    }
    e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { h->graph = nullptr; return OCI_ERR_HIP; }
    return OCI_OK;
}

extern "C" int oci_replay_steps(oci_handle *h) {
    if (!h || !h->graph) return OCI_ERR_INVALID;
    if (h->need_broadcast) {   // the state was replaced: the graph's first step starts from it
        HIPCHECK(launch_flag_broadcast(h->S, h->st));
        h->need_broadcast = false;
    }
    HIPCHECK(hipGraphLaunch(h->graph, h->st));
    return OCI_OK;
}

extern "C" int si_step(oci_handle *h, const double *q_dev, const double *inc_left_dev, const double *inc_right_dev,
                       double *phi_out_dev, double *psi_out_dev, oci_step_info *info_dev) {
    int rc = check_step_args(h, phi_out_dev, info_dev);
    if (rc) return rc;
    StepIO io{q_dev, inc_left_dev, inc_right_dev, phi_out_dev, psi_out_dev, info_dev};
    // Small problems (up to kSiOneWorkgroup (cell, group, angle) rows) run the
    // whole iteration loop in one persistent launch on one 1024-thread
    // workgroup (the decision stays on the device; 2.6x faster than the launch
    // sequence at 80 rows).  Larger ones run the per-phase launch sequence,
    // which measured faster than the persistent loop there (one or many
    // workgroups: 1.0-1.5x slower from 3648 rows up).  OCI_SI_MODE = launches
    // | one | many (testing) forces a layout; many = about one workgroup per
    // 4096 rows, at most one per CU, grid barriers between the phases.
    constexpr long kSiOneWorkgroup = 1024;
    const long rows = (long)h->d.J * h->d.G * h->d.N;
    int kind = rows <= kSiOneWorkgroup ? 1 : 0;
    if (const char *m = getenv("OCI_SI_MODE")) {
        if (!strcmp(m, "launches")) kind = 0;
        else if (!strcmp(m, "one")) kind = 1;
        else if (!strcmp(m, "many")) kind = 2;
    }
    long nwg = 1;
    if (kind == 2) {
        nwg = (rows + 4095) / 4096;
        if (nwg > h->num_cu) nwg = h->num_cu;
        if (nwg < 2) nwg = 2;
    }
    if (kind > 0 && si_loop_occupancy(h->S, kind == 2) < 1) return OCI_ERR_UNSUPPORTED;
    Slab S = h->S;
    S.bar_groups = (int)((nwg + S.bar_gsz - 1) / S.bar_gsz);   // the barrier words the launch uses
    HIPCHECK(launch_begin(S, io, h->need_broadcast, h->st, 0));
    h->need_broadcast = false;
    hipEvent_t e0 = h->profiling ? prof_event(h) : nullptr, e1 = h->profiling ? prof_event(h) : nullptr;
    if (e0) HIPCHECK(hipEventRecord(e0, h->st));
    if (kind > 0) {
        HIPCHECK(launch_si_loop(S, io, (int)nwg, h->st));
    } else {
        // host-driven: the iterations stop themselves on the device; the host
        // polls the done flag between growing batches of launches
        const int cap = h->d.fixed_iters > 0 ? h->d.fixed_iters : h->d.max_iters;
        int launched = 0, batch = 4;
        int32_t flag = 0;
        for (;;) {
            const int k = (cap - launched) < batch ? (cap - launched) : batch;
            for (int i = 0; i < k; ++i) HIPCHECK(launch_si_iteration(S, io, h->st));
            launched += k;
            if (launched >= cap) break;
            HIPCHECK(hipMemcpyAsync(&flag, &S.ctl->done, sizeof(int32_t), hipMemcpyDeviceToHost, h->st));
            HIPCHECK(hipStreamSynchronize(h->st));
            if (flag) break;
            if (batch < 64) batch *= 2;
        }
    }
    if (e1) HIPCHECK(hipEventRecord(e1, h->st));
    if (e1) h->prof_steps += 1;
    HIPCHECK(launch_end(S, io, h->st));
    return OCI_OK;
}

extern "C" int oci_profile_enable(oci_handle *h, int on) {
    if (!h) return OCI_ERR_INVALID;
    h->profiling = on != 0;
    h->ev_used = 0;
    h->prof_steps = 0;
    return OCI_OK;
}

extern "C" int oci_profile_read(oci_handle *h, double *ms, int32_t *steps) {
    if (!h || !ms || !steps) return OCI_ERR_INVALID;
    double tot = 0.0;
    for (size_t k = 0; k + 1 < h->ev_used; k += 2) {
        float t = 0.f;
        if (hipEventSynchronize(h->ev_pool[k + 1]) != hipSuccess) return OCI_ERR_HIP;
        if (hipEventElapsedTime(&t, h->ev_pool[k], h->ev_pool[k + 1]) != hipSuccess) return OCI_ERR_HIP;
        tot += t;
    }
    *ms = tot;
    *steps = h->prof_steps;
    h->ev_used = 0;
    h->prof_steps = 0;
    return OCI_OK;
}

// Candidate launch shapes are timed on the handle's own problem: each runs
// `iters` iterations of one step (no stopping test) from the zero state,
// bracketed by HIP events; the fastest is kept.  The state is zero again
// afterwards.
extern "C" int oci_autotune(oci_handle *h, int32_t iters, int32_t *config) {
    if (!h || iters < 1) return OCI_ERR_INVALID;
    if (h->structured) {   // one launch shape: nothing to choose
        if (oci_set_state(h, nullptr) != OCI_OK) return OCI_ERR_HIP;
        if (config) oci_get_config(h, config);
        return OCI_OK;
    }
    struct Cand { int block; bool local, res; int gsz; };
    std::vector<Cand> cands;
    for (int block : {1024, 256})
        for (int gsz : {16, 64})
            for (int lr = 0; lr < 3; ++lr)
                cands.push_back(Cand{block, lr < 2, lr == 0, gsz});
    const int32_t saved_fixed = h->S.fixed_iters;
    const bool saved_prof = h->profiling;
    h->profiling = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return OCI_ERR_HIP;
    float best = 1e30f;
    int best_k = -1;
    StepIO io{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int rc = OCI_OK;
    for (size_t k = 0; k < cands.size() && rc == OCI_OK; ++k) {
        const Cand &c = cands[k];
        if (configure(h, c.block, c.local, c.res, c.gsz) != OCI_OK) continue;
        if (c.local != h->local || c.res != h->resident) continue;   // shape not available: skip duplicate
        h->S.fixed_iters = iters;
        float ms = 0.f;
        for (int rep = 0; rep < 2 && rc == OCI_OK; ++rep) {   // first run warms up
            if (oci_set_state(h, nullptr) != OCI_OK) { rc = OCI_ERR_HIP; break; }
            if (launch_begin(h->S, io, true, h->st, h->local ? h->nwg : 0) != hipSuccess) { rc = OCI_ERR_HIP; break; }
            h->need_broadcast = false;
            if (hipEventRecord(e0, h->st) != hipSuccess) { rc = OCI_ERR_HIP; break; }
            hipError_t e = h->local ? launch_oci_local(h->S, io, h->fp32, h->np, h->resident, h->block, h->nwg,
                                                       h->ntiles, h->dyn_lds, h->st)
                                    : launch_oci_step(h->S, io, h->fp32, h->np, h->resident, h->block, h->nwg,
                                                      h->ntiles, h->st, true);
            if (e != hipSuccess || hipEventRecord(e1, h->st) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                rc = OCI_ERR_HIP;
        }
        if (rc == OCI_OK && ms < best) { best = ms; best_k = (int)k; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->S.fixed_iters = saved_fixed;
    h->profiling = saved_prof;
    if (rc != OCI_OK) return rc;
    if (best_k < 0) return OCI_ERR_UNSUPPORTED;
    const Cand &c = cands[best_k];
    rc = configure(h, c.block, c.local, c.res, c.gsz);
    if (rc) return rc;
    if (oci_set_state(h, nullptr) != OCI_OK) return OCI_ERR_HIP;
    if (config) oci_get_config(h, config);
    return OCI_OK;
}

extern "C" int oci_set_history(oci_handle *h, double *e_hist_dev, int32_t capacity) {
    if (!h || (e_hist_dev && capacity < 1)) return OCI_ERR_INVALID;
    h->S.hist = e_hist_dev;
    h->S.hist_cap = e_hist_dev ? capacity : 0;
    return OCI_OK;
}

extern "C" int oci_get_config(const oci_handle *h, int32_t *config) {
    if (!h || !config) return OCI_ERR_INVALID;
    config[0] = h->block;
    config[1] = (h->structured ? h->wb_staged : h->local) ? 1 : 0;
    config[2] = h->resident ? 1 : 0;
    config[3] = h->S.bar_gsz;
    config[4] = h->nwg;
    config[5] = h->ntiles;
    return OCI_OK;
}

extern "C" int oci_destroy(oci_handle *h) {
    if (!h) return OCI_ERR_INVALID;
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    delete h;
    return OCI_OK;
}

// ================================================================ batches
// Step argument sets a batch can hold at once (one launch table each).
constexpr int kMaxBatchSteps = 64;

struct oci_batch {
    int nslab;
    bool fp32;
    bool structured;
    bool wb_staged;   // every slab takes the staged structured body
    hipStream_t st;
    std::vector<oci_handle *> slabs;
    std::vector<BatchEntry> tab;   // host copy of the device tables, [nbound][nslab]
    BatchEntry *d_tab;             // in the workspace: kMaxBatchSteps tables, tstride bytes apart
    size_t tstride;
    int nbound;                    // bound step argument sets (0: none)
    int cursor;                    // argument set of the next eager step
    int last;                      // argument set of the last step enqueued (-1: none)
    int nwg;                       // workgroups of the batched launch
    int occ;                       // co-resident batch workgroups per CU
    oci_step_info *info_dev;       // bound results, [nbound][nslab]
    hipGraphExec_t graph;
    int graph_steps, graph_first;  // captured steps and the argument set of the first
};

static size_t batch_table_bytes(int nslab) { return align256((size_t)nslab * sizeof(BatchEntry)); }
static const BatchEntry *batch_dtab(const oci_batch *b, int i) {
    return (const BatchEntry *)((const unsigned char *)b->d_tab + (size_t)i * b->tstride);
}

extern "C" int oci_batch_workspace_bytes(int32_t nslab, const oci_desc *descs, size_t *bytes) {
    if (nslab < 1 || !descs || !bytes) return OCI_ERR_INVALID;
    size_t tot = (size_t)kMaxBatchSteps * batch_table_bytes(nslab);
    for (int k = 0; k < nslab; ++k) {
        size_t b = 0;
        const int rc = oci_workspace_bytes(&descs[k], &b);
        if (rc) return rc;
        if (descs[k].precision != descs[0].precision || descs[k].solver != descs[0].solver) return OCI_ERR_INVALID;
        tot += align256(b);
    }
    *bytes = tot;
    return OCI_OK;
}

extern "C" int oci_batch_destroy(oci_batch *b) {
    if (!b) return OCI_ERR_INVALID;
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    for (oci_handle *h : b->slabs)
        if (h) oci_destroy(h);
    delete b;
    return OCI_OK;
}

// Workgroups per slab in proportion to `weight`, at least one, at most the
// slab's tile count, all co-resident (at most occupancy x CUs in total).
// Workgroups per slab for one launch.  A slab's time is about its iterations
// x (tiles per workgroup x cost of a tile + the grid barrier), so the blocks
// are sized to minimise the largest such time (binary search on the time;
// each slab then takes the fewest workgroups that meet it), within the
// co-resident capacity and at least one and at most one per tile a slab.
// its[k]: iterations of slab k's last step (1 before any step).  Tile cost:
// the structured solve, measured when `ticks` holds each slab's device time of
// that step (the time per iteration, less a 5 us barrier, over the tiles per
// workgroup it had), else pairs per lane (1 or 2) with the barrier worth 1.5
// tiles; the dense solve, the inverse rows streamed per tile (cells x n^2),
// barrier negligible.
static int batch_allocate(oci_batch *b, const std::vector<double> &its,
                          const std::vector<double> &ticks = std::vector<double>()) {
    const int nslab = b->nslab;
    const int num_cu = b->slabs[0]->num_cu;
    long cap = (long)b->occ * num_cu;
    if (cap > (long)num_cu * 8) cap = (long)num_cu * 8;
    if (nslab > cap) return OCI_ERR_UNSUPPORTED;
    const int bs = batch_block();
    std::vector<long> ntile(nslab), alloc(nslab);
    std::vector<double> cost(nslab);
    double cmax = 0.0;
    for (int k = 0; k < nslab; ++k) {
        const oci_handle *h = b->slabs[k];
        const int rpt = h->np > bs ? h->np / bs : 1;
        const int cpt = b->structured ? wb_cells_per_tile(h->d.N, h->d.G) : bs / (h->np / rpt);
        const long cells = h->S.ordering == OCI_ORDER_RED_BLACK ? (h->d.J + 1) / 2 : h->d.J;
        ntile[k] = (cells + cpt - 1) / cpt;
        cost[k] = b->structured ? (h->d.N * h->d.G > 64 ? 2.0 : 1.0) : (double)cpt * h->np * h->np;
        if (cost[k] > cmax) cmax = cost[k];
    }
    double bar_abs = b->structured ? 1.5 : 0.0;
    if (b->structured && (int)ticks.size() == nslab) {
        constexpr double kBarTicks = 500.0;   // one grid barrier, 5 us of the 100 MHz device clock
        bool ok = true;
        std::vector<double> c(nslab);
        for (int k = 0; k < nslab && ok; ++k) {
            const long nw = b->tab[k].nwg > 0 ? b->tab[k].nwg : 1;
            const double tpw = (double)((ntile[k] + nw - 1) / nw);
            c[k] = (ticks[k] / its[k] - kBarTicks) / tpw;
            ok = ticks[k] > 0.0 && c[k] > 0.0;
        }
        if (ok) {
            cost = c;
            bar_abs = kBarTicks;
            cmax = *std::max_element(cost.begin(), cost.end());
        }
    }
    for (int k = 0; k < nslab; ++k) cost[k] /= cmax;
    const double bar = bar_abs / cmax;
    // fewest workgroups for slab k to finish within time T (0: cannot)
    auto need = [&](int k, double T) -> long {
        const double per = (T / its[k] - bar) / cost[k];   // tiles per workgroup allowed
        if (per < 1.0) return 0;
        const long p = per >= (double)ntile[k] ? ntile[k] : (long)per;
        return (ntile[k] + p - 1) / p;
    };
    auto time_of = [&](int k, long n) { return its[k] * (cost[k] * (double)((ntile[k] + n - 1) / n) + bar); };
    double lo = 0.0, hi = 0.0;
    for (int k = 0; k < nslab; ++k) hi = std::max(hi, time_of(k, 1));
    for (int it = 0; it < 100; ++it) {
        const double T = 0.5 * (lo + hi);
        long total = 0;
        bool ok = true;
        for (int k = 0; k < nslab && ok; ++k) {
            const long n = need(k, T);
            if (n == 0) ok = false;
            total += n;
        }
        if (ok && total <= cap) hi = T; else lo = T;
    }
    long used = 0;
    for (int k = 0; k < nslab; ++k) {
        alloc[k] = need(k, hi);
        if (alloc[k] < 1) alloc[k] = 1;
        used += alloc[k];
    }
    // spare workgroups to the slowest slabs while that shortens them
    while (used < cap) {
        int kmax = -1;
        double tmax = -1.0;
        for (int k = 0; k < nslab; ++k)
            if (alloc[k] < ntile[k] && time_of(k, alloc[k]) > tmax) { tmax = time_of(k, alloc[k]); kmax = k; }
        if (kmax < 0 || time_of(kmax, alloc[kmax] + 1) >= tmax) break;
        ++alloc[kmax];
        ++used;
    }
    int wg0 = 0;
    const int nsets = b->nbound > 0 ? b->nbound : 1;
    for (int k = 0; k < nslab; ++k) {
        for (int i = 0; i < nsets; ++i) {
            BatchEntry &e = b->tab[(size_t)i * nslab + k];
            e.S.bar_groups = (int)((alloc[k] + e.S.bar_gsz - 1) / e.S.bar_gsz);
            e.ntiles = (int)ntile[k];
            e.wg0 = wg0;
            e.nwg = (int)alloc[k];
        }
        wg0 += (int)alloc[k];
    }
    b->nwg = wg0;
    return OCI_OK;
}

static hipError_t batch_upload(oci_batch *b) {
    const int nsets = b->nbound > 0 ? b->nbound : 1;
    for (int i = 0; i < nsets; ++i) {
        const hipError_t e = hipMemcpyAsync((void *)batch_dtab(b, i), &b->tab[(size_t)i * b->nslab],
                                            sizeof(BatchEntry) * b->nslab, hipMemcpyHostToDevice, b->st);
        if (e != hipSuccess) return e;
    }
    return hipStreamSynchronize(b->st);
}

extern "C" int oci_batch_setup(int32_t nslab, const oci_desc *descs, void *workspace_dev, size_t workspace_bytes,
                               void *stream, oci_batch **out) {
    if (!out) return OCI_ERR_INVALID;
    *out = nullptr;
    size_t need = 0;
    int rc = oci_batch_workspace_bytes(nslab, descs, &need);
    if (rc) return rc;
    if (!workspace_dev || ((uintptr_t)workspace_dev & 255) || workspace_bytes < need) return OCI_ERR_WORKSPACE;
    oci_batch *b = new (std::nothrow) oci_batch();
    if (!b) return OCI_ERR_HIP;
    b->nslab = nslab;
    b->fp32 = descs[0].precision == OCI_FP32_REFINED;
    b->structured = descs[0].solver == OCI_SOLVE_STRUCTURED;
    b->st = (hipStream_t)stream;
    b->d_tab = (BatchEntry *)workspace_dev;
    b->tstride = batch_table_bytes(nslab);
    b->nbound = 0;
    b->cursor = 0;
    b->last = -1;
    b->graph = nullptr;
    unsigned char *ws = (unsigned char *)workspace_dev;
    size_t off = (size_t)kMaxBatchSteps * batch_table_bytes(nslab);
    for (int k = 0; k < nslab; ++k) {
        size_t bk = 0;
        oci_workspace_bytes(&descs[k], &bk);
        oci_handle *h = nullptr;
        rc = oci_setup(&descs[k], ws + off, align256(bk), stream, &h);
        if (rc) { oci_batch_destroy(b); return rc; }
        b->slabs.push_back(h);
        off += align256(bk);
    }
    int occ = 0;
    b->wb_staged = b->structured;
    for (int k = 0; k < nslab; ++k) b->wb_staged = b->wb_staged && b->slabs[k]->wb_staged;
    const hipError_t oe = b->structured ? wb_batch_occupancy(b->wb_staged, &occ) : batch_occupancy(b->fp32, &occ);
    if (oe != hipSuccess || occ < 1) { oci_batch_destroy(b); return OCI_ERR_HIP; }
    b->occ = occ;
    b->tab.resize(nslab);
    for (int k = 0; k < nslab; ++k) {
        memset(&b->tab[k], 0, sizeof(BatchEntry));
        b->tab[k].S = b->slabs[k]->S;
    }
    rc = batch_allocate(b, std::vector<double>(nslab, 1.0));
    if (rc) { oci_batch_destroy(b); return rc; }
    *out = b;
    return OCI_OK;
}

extern "C" int oci_batch_bind_steps(oci_batch *b, int32_t n_steps, const double *const *q_dev,
                                    const double *const *inc_left_dev, const double *const *inc_right_dev,
                                    double *const *phi_out_dev, oci_step_info *info_dev) {
    if (!b || n_steps < 1 || n_steps > kMaxBatchSteps || !phi_out_dev || !info_dev) return OCI_ERR_INVALID;
    const int ns = b->nslab;
    for (size_t i = 0; i < (size_t)n_steps * ns; ++i)
        if (!phi_out_dev[i]) return OCI_ERR_INVALID;
    // every argument set starts as a copy of set 0's slab views and geometry
    std::vector<BatchEntry> tab((size_t)n_steps * ns);
    for (int i = 0; i < n_steps; ++i)
        for (int k = 0; k < ns; ++k) {
            BatchEntry &e = tab[(size_t)i * ns + k];
            e = b->tab[k];
            const size_t a = (size_t)i * ns + k;
            StepIO &io = e.io;
            memset(&io, 0, sizeof(StepIO));
            io.q = q_dev ? q_dev[a] : nullptr;
            io.inc_l = inc_left_dev ? inc_left_dev[a] : nullptr;
            io.inc_r = inc_right_dev ? inc_right_dev[a] : nullptr;
            io.phi_out = phi_out_dev[a];
            io.psi_out = nullptr;
            io.info = info_dev + a;
        }
    if (b->graph) { (void)hipGraphExecDestroy(b->graph); b->graph = nullptr; }
    b->tab.swap(tab);
    b->nbound = n_steps;
    b->cursor = 0;
    b->last = -1;
    b->info_dev = info_dev;
    HIPCHECK(batch_upload(b));
    return OCI_OK;
}

extern "C" int oci_batch_bind(oci_batch *b, const double *const *q_dev, const double *const *inc_left_dev,
                              const double *const *inc_right_dev, double *const *phi_out_dev,
                              oci_step_info *info_dev) {
    return oci_batch_bind_steps(b, 1, q_dev, inc_left_dev, inc_right_dev, phi_out_dev, info_dev);
}

extern "C" int oci_batch_step(oci_batch *b) {
    if (!b || b->nbound < 1) return OCI_ERR_INVALID;
    HIPCHECK(launch_batch_step(batch_dtab(b, b->cursor), b->nslab, b->nwg, b->fp32, b->structured, b->wb_staged, false, b->st, true));
    b->last = b->cursor;
    b->cursor = (b->cursor + 1) % b->nbound;
    return OCI_OK;
}

extern "C" int oci_batch_capture(oci_batch *b, int32_t n_steps) {
    if (!b || b->nbound < 1 || n_steps < 1 || !b->st) return OCI_ERR_INVALID;
    if (b->graph) { (void)hipGraphExecDestroy(b->graph); b->graph = nullptr; }
    HIPCHECK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < n_steps && e == hipSuccess; ++k)
        e = launch_batch_step(batch_dtab(b, (b->cursor + k) % b->nbound), b->nslab, b->nwg, b->fp32, b->structured, b->wb_staged,
                              false, b->st, false);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->st, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return OCI_ERR_HIP;
    }
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { b->graph = nullptr; return OCI_ERR_HIP; }
    b->graph_steps = n_steps;
    b->graph_first = b->cursor;
    return OCI_OK;
}

extern "C" int oci_batch_replay(oci_batch *b) {
    if (!b || !b->graph) return OCI_ERR_INVALID;
    HIPCHECK(hipGraphLaunch(b->graph, b->st));
    b->last = (b->graph_first + b->graph_steps - 1) % b->nbound;
    return OCI_OK;
}

extern "C" int oci_batch_set_state(oci_batch *b, int32_t k, const double *psi_prev_dev) {
    if (!b || k < 0 || k >= b->nslab) return OCI_ERR_INVALID;
    const int rc = oci_set_state(b->slabs[k], psi_prev_dev);
    if (rc) return rc;
    b->slabs[k]->need_broadcast = false;   // batched steps use the device flag
    HIPCHECK(launch_flag_broadcast(b->slabs[k]->S, b->st));
    return OCI_OK;
}

extern "C" int oci_batch_get_state(const oci_batch *b, int32_t k, double *psi_prev_dev) {
    if (!b || k < 0 || k >= b->nslab) return OCI_ERR_INVALID;
    return oci_get_state(b->slabs[k], psi_prev_dev);
}

extern "C" int oci_batch_rebalance(oci_batch *b) {
    if (!b || b->nbound < 1 || b->last < 0) return OCI_ERR_INVALID;
    std::vector<oci_step_info> info(b->nslab);
    HIPCHECK(hipStreamSynchronize(b->st));
    HIPCHECK(hipMemcpy(info.data(), b->info_dev + (size_t)b->last * b->nslab, sizeof(oci_step_info) * b->nslab,
                       hipMemcpyDeviceToHost));
    std::vector<double> its(b->nslab), ticks;
    for (int k = 0; k < b->nslab; ++k) its[k] = info[k].iterations > 0 ? info[k].iterations : 1;
    if (b->structured) {   // each slab's device time of that step
        ticks.resize(b->nslab);
        for (int k = 0; k < b->nslab; ++k) {
            Ctl c;
            HIPCHECK(hipMemcpy(&c, b->slabs[k]->S.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
            ticks[k] = c.t_end > c.t_begin ? (double)(c.t_end - c.t_begin) : 0.0;
        }
    }
    const int rc = batch_allocate(b, its, ticks);
    if (rc) return rc;
    HIPCHECK(batch_upload(b));
    if (b->graph) { (void)hipGraphExecDestroy(b->graph); b->graph = nullptr; }
    return OCI_OK;
}

extern "C" int oci_batch_info(const oci_batch *b, int32_t *nwg_total, int32_t *nwg_per_slab) {
    if (!b || !nwg_total) return OCI_ERR_INVALID;
    *nwg_total = b->nwg;
    if (nwg_per_slab)
        for (int k = 0; k < b->nslab; ++k) nwg_per_slab[k] = b->tab[k].nwg;
    return OCI_OK;
}

extern "C" const char *oci_status_string(int s) {
    switch (s) {
    case OCI_OK: return "ok";
    case OCI_NOT_CONVERGED: return "not converged (iteration cap reached)";
    case OCI_NONFINITE: return "non-finite change (iteration diverged or bad input)";
    case OCI_ERR_INVALID: return "invalid argument";
    case OCI_ERR_HIP: return "HIP runtime error";
    case OCI_ERR_SINGULAR: return "singular cell matrix (zero pivot)";
    case OCI_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case OCI_ERR_UNSUPPORTED: return "cell system larger than the compiled kernels (4 N G > 512)";
    case OCI_ERR_TOO_LARGE: return "problem needs more than the 64 MiB static workspace of oci_setup_static";
    case OCI_ERR_DEVICE: return "device-side wait expired (a workgroup of the persistent launch was not co-resident)";
    default: return "unknown status";
    }
}
