// oci_internal.hpp -- layouts and launch parameters shared by the host side of
// liboci and its gfx950 kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace oci {

// Largest cell system the kernels are compiled for (n = 4 N G).
constexpr int kMaxN = 512;
// Threads per workgroup of the setup and bookkeeping kernels.
constexpr int kBlock = 256;
// Barrier words are kBarStride uint64 apart; workgroups arrive in groups of
// kBarGroup before one leader per group arrives at the top counter.
constexpr int kBarStride = 32;
constexpr int kBarGroup = 16;
// Hand-off slots of the workgroup-local kernel.  An edge value travels as two
// 64-bit words, each holding one 32-bit half of the double below a 32-bit tag
// (the iteration that will read it); a slot reset to kSlotEmpty carries no
// valid tag.  A partial-sum slot holds the bits of a non-negative double whose
// low kPartTagBits mantissa bits carry the iteration number modulo
// 2^kPartTagBits; kSlotEmpty (sign bit set) never matches a tag either.
constexpr uint64_t kSlotEmpty = ~0ull;
constexpr int kPartTagBits = 4;
// Partial-sum slots per workgroup (a ring over iterations) and, with
// register-resident rows, how many iterations behind the partials read for a
// decision are; that decision takes effect one iteration later still, so the
// kernel keeps kResidentCopies = kResidentLag + 2 LDS copies of the range's
// iterate.  A slot is rewritten kPartSlots iterations later, which needs
// kPartSlots > kResidentLag + 1; the tag period 2^kPartTagBits exceeds
// kPartSlots.  A multi-step launch skips iteration numbers at each step
// turnover; it resets the skipped iterations' slots to kSlotEmpty, since a
// value left there would carry the tag of the iteration 2^kPartTagBits later.
constexpr int kPartSlots = 8;
constexpr int kResidentLag = 2;
constexpr int kResidentCopies = kResidentLag + 2;
static_assert(kPartSlots > kResidentLag + 1 && (1 << kPartTagBits) > kPartSlots, "partial-sum ring");

// Control block of one slab problem, in the workspace.  Written by the step
// kernels only; the host reads `done` to learn that a step has stopped.
struct Ctl {
    int32_t base;          // ping-pong index holding the first iterate of the step
    int32_t iter;          // iterations performed in the current step
    int32_t done;          // 1 once the current step has stopped
    int32_t status;        // OCI_OK / OCI_NOT_CONVERGED / OCI_NONFINITE
    int32_t err;           // device guard tripped (OCI_ERR_DEVICE)
    int32_t singular;      // setup found a zero pivot
    uint32_t bar_count;    // grid barrier: arrivals in the current generation
    uint32_t bar_gen;      // grid barrier: generation
    double e_prev;         // e_{l-1}
    double e_last;         // e_l
    double rho;            // e_l / e_{l-1}
    int32_t bcast;         // batched steps: start the next step from psi_prev on both levels
    int32_t pad0;
    uint64_t t_begin;      // structured solve: device clock (wall_clock64) at the step's start and
    uint64_t t_end;        // at its stopping decision, for the batch's workgroup allocation
};
static_assert(sizeof(Ctl) == 80, "Ctl layout");

// Device-side view of one slab problem (all pointers into the workspace or
// caller memory).  Passed by value to every kernel.
struct Slab {
    int32_t J, N, G, n;          // n = 4 N G
    int32_t np;                  // n padded to a power of two >= 8 (factor block size)
    double dt;
    const double *mu, *w;        // [N] ascending Gauss-Legendre nodes / weights
    const double *dx;            // [J]
    const double *sigma_t;       // [J][G]
    const double *sigma_s;       // [J][G][G], [j][g][gp] = gp -> g
    const double *speed;         // [G]
    void *X;                     // [J][np][np] inverse of A_j (identity-padded), tiled (see xoff)
    double *psi[2];              // [J][G][N][4] ping-pong iterates
    double *phi[2];              // [J][G][4]   scalar flux of each iterate
    double *psi_prev;            // [J][G][N][2] state psi_{k-1/2}
    double *crhs;                // [J][G][N][4] constant part of b for the current step
    double *exch;                // [2][max workgroups][2][2][G][N/2][2 words] boundary edges between workgroups
    double *si_linv;             // [J][G][N][16] inverse of the 4x4 SI cell matrix
    double *si_resp;             // [J][G][N][8] response of the cell to its two incident edges
    double *si_msw;              // [J][NG][4] 2x2 edge-to-edge map, in sweep order
    double *si_alpha;            // [J][NG][2] outgoing edges of the uncoupled solution, sweep order
    double *si_ein;              // [J][NG][2] incident edges met by the sweep, sweep order
    double *partials;            // [kPartSlots][max workgroups] per-workgroup sums (by iteration mod 2, or mod kPartSlots)
    int32_t zero_cell;           // test hook: the setup zeroes column 0 of this cell's matrix (-1: none)
    int32_t ordering;            // 0: Jacobi over cells, 1: red-black (structured solve)
    int32_t periodic;            // 1: periodic mesh instead of incident fluxes (structured solve)
    int32_t hist_cap;            // entries of hist
    double *hist;                // e_l of every iteration of the last step, or null
    double *edge;                // structured solve: [2][J][G][N][2] outgoing corners of each (g, m) at
                                 // levels k and k+1/2, by iteration parity
    double *wb;                  // structured cell solve: [J][4G][2G] complex, the rows of (I - W C)^-1 then of
                                 // C (I - W C)^-1 (see oci_wb.hip); null for the dense solve
    Ctl *ctl;
    // grid barrier words, 256 bytes apart: [0] arrivals of group leaders,
    // [kBarStride] release flag, [(2 + k) * kBarStride] arrivals in group k
    uint64_t *bar;
    int32_t bar_groups;          // group counters present in `bar`
    int32_t bar_gsz;             // workgroups per arrival group
    // step controls
    double tol;
    int32_t max_iters, fixed_iters, norm, refined;
};

// Per-step inputs (caller memory).
struct StepIO {
    const double *q;             // [J][G][4] or null
    const double *inc_l;         // [2][G][N/2] or null
    const double *inc_r;         // [2][G][N/2] or null
    double *phi_out;             // [J][G][4]
    double *psi_out;             // [J][G][N][4] or null
    void *info;                  // oci_step_info*
    int32_t nsteps;              // time steps in one launch (register-resident kernel; <= 1: one);
                                 // phi_out and info then hold one record per step
    int32_t pad;
    int64_t q_stride;            // elements between consecutive steps' q (0: the same q every step)
    int64_t inc_stride;          // elements between consecutive steps' inc_l / inc_r (0: the same)
};

// One slab of a batch: its view, its step inputs/outputs, and the block of
// workgroups [wg0, wg0 + nwg) of the batched launch that serves it.
struct BatchEntry {
    Slab S;
    StepIO io;
    int32_t ntiles, wg0, nwg, pad;
};

// Element (r, c) of a cell's n x n factor block, stored as 16-byte vectors
// along rows: block [c / V][r][c % V], V = 16 / sizeof(T).  The thread that
// owns row r reads columns c .. c+V-1 with one 16-byte load, and the threads
// of consecutive rows read consecutive 16-byte words.
template <typename T>
__host__ __device__ inline size_t xoff(int n, int r, int c) {
    constexpr int V = 16 / sizeof(T);
    return ((size_t)(c / V) * n + r) * V + (c % V);
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace oci
