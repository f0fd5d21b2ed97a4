// oci_setup.hip -- per-cell assembly and inversion of the one-cell-inversion
// systems on gfx950.
//
// One workgroup per cell.  The cell matrix (paper eqs. Aj, scatter_mg,
// fullOCIlhs) is assembled on the device and replaced by its inverse, which
// every later iteration applies as one matrix-vector product per cell: that
// keeps all lanes busy where the two triangular substitutions of getrs would
// be a dependent chain of n steps.  Pivoting is partial, by rows, as in the
// gesv factorisation of the paper's batched solver (largest |a_ik| among the
// candidate rows, the lowest row winning ties).
//  * Small cells (n <= 64) work in LDS: right-looking LU, then inversion from
//    the factors the way LAPACK's getri does (invert U, solve X L = U^-1,
//    undo the row exchanges as column exchanges).
//  * Larger cells use blocked Gauss-Jordan elimination in place in the
//    cell's slot of the factor buffer: a panel of NB columns is eliminated in
//    LDS, and the rest of the matrix receives the panel's rank-NB update as a
//    matrix product on the matrix cores (MFMA).  Both routes perform the same
//    2 n^3 flops; Gauss-Jordan puts nearly all of them into those uniform
//    rank-NB products.
// Work precision T is float for the refined path and double for the FP64
// path; assembly arithmetic is double and rounded once to T.
#include "oci_internal.hpp"

namespace oci {

template <typename T>
struct LdsMat {
    T *a;
    int ld;
    __device__ T &operator()(int r, int c) const { return a[r * ld + c]; }
};

template <typename T>
struct TiledMat {
    T *a;
    int n;
    __device__ T &operator()(int r, int c) const { return a[xoff<T>(n, r, c)]; }
};

// Value of A_j at (r, c) (double precision).  Unknown index (g*N + m)*4 + u.
__device__ inline double cell_entry(const Slab &S, int j, int r, int c) {
    if (r >= S.n || c >= S.n) return r == c ? 1.0 : 0.0;  // padding block: identity
    if (j == S.zero_cell && c == 0) return 0.0;            // test hook: a zero pivot
    const int N = S.N, G = S.G;
    const int gr = r / (4 * N), mr = (r / 4) % N, ur = r & 3;
    const int gc = c / (4 * N), mc = (c / 4) % N, uc = c & 3;
    const double dx = S.dx[j];
    double v = 0.0;
    if (gr == gc && mr == mc) {
        // within-cell operator L_{c,j,g,m} (eq. Aj) with this group's sigma and v
        const double sig = S.sigma_t[(size_t)j * G + gr];
        const double a = dx / (S.speed[gr] * S.dt);
        const double mu = S.mu[mr];
        const double d = 0.5 * (fabs(mu) + dx * sig);
        const double h = 0.5 * mu;
        // L = [[d, h, a/2, 0], [-h, d, 0, a/2], [-a, 0, a+d, h], [0, -a, -h, a+d]]
        const bool top = ur < 2, left = uc < 2;
        if (top == left)
            v = ur == uc ? (top ? d : a + d) : ((ur & 1) ? -h : h);
        else if (top)
            v = uc - 2 == ur ? 0.5 * a : 0.0;
        else
            v = uc == ur - 2 ? -a : 0.0;
    }
    if (ur == uc) {
        // minus the scattering block S_{gc -> gr}: same corner and time level
        v -= 0.25 * dx * S.sigma_s[((size_t)j * G + gr) * G + gc] * S.w[mc];
    }
    return v;
}

// Workgroup argmax of |a(i,k)| over i in [k, n): largest value, lowest index
// winning ties.  Returns -1 when the column is zero from row k down.
template <typename T, typename M>
__device__ int pivot_row(const M &A, int n, int k, T *s_best, int *s_idx) {
    const int tid = threadIdx.x;
    T best = T(-1);
    int bi = n;
    for (int i = k + tid; i < n; i += kBlock) {
        const T v = fabs(A(i, k));
        if (v > best) { best = v; bi = i; }  // rows visited in increasing order
    }
    for (int off = 32; off > 0; off >>= 1) {
        const T ov = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    const int wave = tid >> 6, lane = tid & 63;
    if (lane == 0) { s_best[wave] = best; s_idx[wave] = bi; }
    __syncthreads();
    if (tid == 0) {
        T b = s_best[0];
        int i0 = s_idx[0];
        for (int w = 1; w < kBlock / 64; ++w)
            if (s_best[w] > b || (s_best[w] == b && s_idx[w] < i0)) { b = s_best[w]; i0 = s_idx[w]; }
        s_idx[kBlock / 64] = (b > T(0)) ? i0 : -1;
    }
    __syncthreads();
    const int p = s_idx[kBlock / 64];
    __syncthreads();
    return p;
}

// LU with partial pivoting then in-place inversion.  Returns false (in all
// threads) if a pivot was zero; the matrix content is then unspecified.
template <typename T, typename M>
__device__ bool factor_invert(const M &A, int n, int *s_piv, T *s_work) {
    __shared__ T s_best[kBlock / 64];
    __shared__ int s_idx[kBlock / 64 + 1];
    const int tid = threadIdx.x;

    // ---- getrf: right-looking, one column at a time
    for (int k = 0; k < n; ++k) {
        const int p = pivot_row<T>(A, n, k, s_best, s_idx);
        if (p < 0) return false;
        if (tid == 0) s_piv[k] = p;
        if (p != k)
            for (int c = tid; c < n; c += kBlock) {
                T t = A(k, c);
                A(k, c) = A(p, c);
                A(p, c) = t;
            }
        __syncthreads();
        const T inv = T(1) / A(k, k);
        for (int i = k + 1 + tid; i < n; i += kBlock) A(i, k) *= inv;
        __syncthreads();
        const int m = n - k - 1;
        for (int e = tid; e < m * m; e += kBlock) {
            const int i = k + 1 + e / m, c = k + 1 + e % m;
            A(i, c) -= A(i, k) * A(k, c);
        }
        __syncthreads();
    }

    // ---- invert U in place (upper triangle, diagonal included)
    for (int j = 0; j < n; ++j) {
        const T ujj = T(1) / A(j, j);
        // column j above the diagonal: x = -ujj * Uinv[0:j,0:j] * U[0:j, j]
        for (int i = tid; i < j; i += kBlock) s_work[i] = A(i, j);
        __syncthreads();
        T acc[2] = {T(0), T(0)};
        for (int r = 0; r < 2; ++r) {
            const int i = tid + r * kBlock;
            if (i < j) {
                T s = T(0);
                for (int k = i; k < j; ++k) s += A(i, k) * s_work[k];
                acc[r] = -ujj * s;
            }
        }
        __syncthreads();
        for (int r = 0; r < 2; ++r) {
            const int i = tid + r * kBlock;
            if (i < j) A(i, j) = acc[r];
        }
        if (tid == 0) A(j, j) = ujj;
        __syncthreads();
    }

    // ---- solve X L = U^-1 for X, columns right to left (L unit lower)
    for (int j = n - 2; j >= 0; --j) {
        for (int i = j + 1 + tid; i < n; i += kBlock) {
            s_work[i] = A(i, j);
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < n; i += kBlock) A(i, j) = T(0);
        __syncthreads();
        for (int r = tid; r < n; r += kBlock) {
            T s = A(r, j);
            for (int k = j + 1; k < n; ++k) s -= A(r, k) * s_work[k];
            A(r, j) = s;
        }
        __syncthreads();
    }

    // ---- undo the row exchanges as column exchanges, last first
    for (int j = n - 2; j >= 0; --j) {
        const int p = s_piv[j];
        if (p != j)
            for (int r = tid; r < n; r += kBlock) {
                T t = A(r, j);
                A(r, j) = A(r, p);
                A(r, p) = t;
            }
        __syncthreads();
    }
    return true;
}

// Assemble, factor and invert the matrix of one small cell per workgroup,
// in LDS (dynamic shared, n x (n+1) of T), then store it tiled.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_assemble_factor(Slab S, int j0) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_piv[kMaxN];
    __shared__ T s_work[kMaxN];
    const int j = j0 + blockIdx.x;
    if (j >= S.J) return;
    const int n = S.np;
    T *Xj = reinterpret_cast<T *>(S.X) + (size_t)j * n * n;
    LdsMat<T> A{reinterpret_cast<T *>(smem), n + 1};
    for (int e = threadIdx.x; e < n * n; e += kBlock) {
        const int r = e / n, c = e % n;
        A(r, c) = (T)cell_entry(S, j, r, c);
    }
    __syncthreads();
    const bool ok = factor_invert<T>(A, n, s_piv, s_work);
    if (ok) {
        TiledMat<T> X{Xj, n};
        for (int e = threadIdx.x; e < n * n; e += kBlock) {
            const int r = e / n, c = e % n;
            X(r, c) = A(r, c);
        }
    }
    if (!ok && threadIdx.x == 0) atomicOr(&S.ctl->singular, 1);
}

// ------------------------------------------------- blocked Gauss-Jordan (MFMA)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename T> struct Quad;
template <> struct Quad<float> { using type = f32x4; };
template <> struct Quad<double> { using type = f64x4; };

// 16x16x4 matrix-core product D = A B + C.  Lane l supplies A[l%16][l/16]
// and B[l/16][l%16].  Element q of lane l's result is D[4 (l/16) + q][l%16]
// for float and D[l/16 + 4 q][l%16] for double (both checked on gfx950).
// Used with A row i standing for D row mfma_row(i), lane l's four results
// are D rows 4 (l/16) .. 4 (l/16) + 3 in order for both types.
__device__ inline int mfma_row(float, int li) { return li; }
__device__ inline int mfma_row(double, int li) { return 4 * (li & 3) + (li >> 2); }
__device__ inline f32x4 mfma16(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f64x4 mfma16(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Four consecutive columns c .. c+3 (c a multiple of 4) of row r of a tiled
// n x n block: one 16-byte word for float, two for double.
__device__ inline f32x4 load_quad(const float *X, int n, int r, int c) {
    return *reinterpret_cast<const f32x4 *>(X + xoff<float>(n, r, c));
}
__device__ inline f64x4 load_quad(const double *X, int n, int r, int c) {
    const double2 a = *reinterpret_cast<const double2 *>(X + xoff<double>(n, r, c));
    const double2 b = *reinterpret_cast<const double2 *>(X + xoff<double>(n, r, c + 2));
    return f64x4{a.x, a.y, b.x, b.y};
}
__device__ inline void store_quad(float *X, int n, int r, int c, f32x4 v) {
    *reinterpret_cast<f32x4 *>(X + xoff<float>(n, r, c)) = v;
}
__device__ inline void store_quad(double *X, int n, int r, int c, f64x4 v) {
    *reinterpret_cast<double2 *>(X + xoff<double>(n, r, c)) = double2{v.x, v.y};
    *reinterpret_cast<double2 *>(X + xoff<double>(n, r, c + 2)) = double2{v.z, v.w};
}

__device__ inline void copy16(void *dst, const void *src) {
    *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(src);
}

// Lane moves inside rows of 16 lanes (DPP, no LDS round trip) for the pivot
// search; called with every lane of the wave active.
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <- 7 - i within 8
constexpr int kDppMirror = 0x140;      // lane i <- 15 - i within 16
template <int CTRL>
__device__ inline unsigned dpp_u32(unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
__device__ inline unsigned lane_u32(unsigned v, int lane) {
    return (unsigned)__builtin_amdgcn_readlane((int)v, lane);
}
// Maximum and minimum over the 64 lanes of the wave; every lane gets them.
__device__ inline unsigned wave_max_u32(unsigned v) {
    v = max(v, dpp_u32<kDppXor1>(v));
    v = max(v, dpp_u32<kDppXor2>(v));
    v = max(v, dpp_u32<kDppHalfMirror>(v));
    v = max(v, dpp_u32<kDppMirror>(v));
    return max(max(lane_u32(v, 0), lane_u32(v, 16)), max(lane_u32(v, 32), lane_u32(v, 48)));
}
__device__ inline unsigned wave_min_u32(unsigned v) {
    v = min(v, dpp_u32<kDppXor1>(v));
    v = min(v, dpp_u32<kDppXor2>(v));
    v = min(v, dpp_u32<kDppHalfMirror>(v));
    v = min(v, dpp_u32<kDppMirror>(v));
    return min(min(lane_u32(v, 0), lane_u32(v, 16)), min(lane_u32(v, 32), lane_u32(v, 48)));
}

// Elements q .. q+V-1 of a register vector from / to one 16-byte word.
template <typename R>
__device__ inline void get16(R &v, int q, const float *s) {
    const f32x4 w = *reinterpret_cast<const f32x4 *>(s);
    v[q] = w.x;
    v[q + 1] = w.y;
    v[q + 2] = w.z;
    v[q + 3] = w.w;
}
template <typename R>
__device__ inline void get16(R &v, int q, const double *s) {
    const double2 w = *reinterpret_cast<const double2 *>(s);
    v[q] = w.x;
    v[q + 1] = w.y;
}
template <typename R>
__device__ inline void put16(float *d, const R &v, int q) {
    *reinterpret_cast<f32x4 *>(d) = f32x4{v[q], v[q + 1], v[q + 2], v[q + 3]};
}
template <typename R>
__device__ inline void put16(double *d, const R &v, int q) {
    *reinterpret_cast<double2 *>(d) = double2{v[q], v[q + 1]};
}

// |v| as an unsigned key in two words (ordered like the magnitude).
__device__ inline void mag_key(float v, unsigned &hi, unsigned &lo) {
    hi = __float_as_uint(v) & 0x7fffffffu;
    lo = 0;
}
__device__ inline void mag_key(double v, unsigned &hi, unsigned &lo) {
    hi = (unsigned)__double2hiint(v) & 0x7fffffffu;
    lo = (unsigned)__double2loint(v);
}

// The cell matrix (the same entries as cell_entry) written row by row into
// its tiled np x np block X: one thread per row with the row's constants
// computed once, and the cell's weights w_m and scattering coefficients
// dx Sigma_s / 4 staged in LDS (`cw`, N + G^2 doubles).  Columns come in
// blocks of the four unknowns of one (group, angle).
template <typename T, int BS>
__device__ void assemble_tiled(const Slab &S, int j, T *X, double *cw) {
    constexpr int V = 16 / (int)sizeof(T);
    const int N = S.N, G = S.G, n = S.n, np = S.np;
    const double dx = S.dx[j];
    double *css = cw + N;
    for (int i = threadIdx.x; i < N; i += BS) cw[i] = S.w[i];
    for (int i = threadIdx.x; i < G * G; i += BS) css[i] = 0.25 * dx * S.sigma_s[(size_t)j * G * G + i];
    __syncthreads();
    for (int r = threadIdx.x; r < np; r += BS) {
        double Lr[4] = {0.0, 0.0, 0.0, 0.0};
        int g = 0, m = 0, u = 0;
        if (r < n) {
            g = r / (4 * N);
            m = (r >> 2) % N;
            u = r & 3;
            const double sig = S.sigma_t[(size_t)j * G + g];
            const double a = dx / (S.speed[g] * S.dt);
            const double mu = S.mu[m];
            const double d = 0.5 * (fabs(mu) + dx * sig), h = 0.5 * mu;
            // row u of L = [[d, h, a/2, 0], [-h, d, 0, a/2], [-a, 0, a+d, h], [0, -a, -h, a+d]]
            if (u == 0) { Lr[0] = d; Lr[1] = h; Lr[2] = 0.5 * a; }
            else if (u == 1) { Lr[0] = -h; Lr[1] = d; Lr[3] = 0.5 * a; }
            else if (u == 2) { Lr[0] = -a; Lr[2] = a + d; Lr[3] = h; }
            else { Lr[1] = -a; Lr[2] = -h; Lr[3] = a + d; }
        }
        const double *ssr = css + g * G;
        int gc = 0, mc = 0;
        for (int blk = 0; blk < np / 4; ++blk) {
            T v[4];
            if (r >= n || 4 * blk >= n) {  // padding: identity
                for (int uc = 0; uc < 4; ++uc) v[uc] = 4 * blk + uc == r ? T(1) : T(0);
            } else {
                const double sc = ssr[gc] * cw[mc];
                const bool diag = gc == g && mc == m;
                for (int uc = 0; uc < 4; ++uc) {
                    double x = uc == u ? -sc : 0.0;
                    if (diag) x += Lr[uc];
                    v[uc] = (T)x;
                }
                if (blk == 0 && j == S.zero_cell) v[0] = T(0);   // test hook: a zero pivot
            }
            for (int w = 0; w < 4 / V; ++w) copy16(X + ((size_t)(blk * (4 / V) + w) * np + r) * V, v + w * V);
            if (++mc == N) { mc = 0; ++gc; }
        }
    }
}

// Assemble the cell matrix into the cell's tiled slot of the factor buffer
// and replace it by its inverse (np >= 128, a multiple of NB and of 16, and
// np <= BS: thread r owns row r of the panel).
//
// Gauss-Jordan: eliminating column k with pivot row p scales row p by 1/a_pk
// (storing 1/a_pk in place of a_pk) and subtracts a_ik times that row from
// every other row i (storing -a_ik/a_pk in place of a_ik).  Rows are moved as
// the elimination goes so that the pivot of column k ends in row k; the
// result T then holds A^-1 with its columns permuted: X[:, c] = T[:, sigma(c)]
// where sigma(c) is the final position of the row that started as row c.
//
// Blocking: the NB columns [k0, k0+NB) are eliminated with each thread's
// panel row in registers.  The pivot of each column is the largest magnitude
// among the rows not yet used as pivots, the lowest row winning ties: a DPP
// reduction per wave and one workgroup barrier per column, each wave
// publishing its best row beside its key so the winner's row needs no second
// round.  Then the pivot rows move to rows k0 .. k0+NB-1 and the rows they
// displace from that block take the vacated places.  The panel's effect on
// any other column x is x <- (x with those moves applied and rows
// k0..k0+NB-1 zeroed) + P x_piv, where x_piv holds that column's entries in
// the NB pivot rows before the panel.  The product runs as 16x16x4 MFMAs, one
// wave per 16-column stripe, each wave reading the pivot rows' entries of its
// stripe before it overwrites the stripe.  A row outside the block whose
// content moved can only have come from inside the block, and each stripe
// writes the block's row tiles last, so every read of a moved row precedes
// its overwrite in the same wave.  In the MFMA the output tile is transposed
// (A operand = pivot rows, B operand = P), which leaves each lane holding
// four consecutive columns of one row: one 16-byte word of the tiled layout
// for float, two for double.  The contraction index is split as
// k = (lane / 16) * NB/4 + step, so each lane reads its P operands as
// consecutive words.
template <typename T, int NB, int BS>
__global__ __launch_bounds__(BS) void k_gj_invert(Slab S, int j0) {
    using Q = typename Quad<T>::type;
    constexpr int V = 16 / (int)sizeof(T);  // elements per 16-byte word
    constexpr int LDP = NB + V;             // panel row stride (elements)
    constexpr int W = BS / 64;
    constexpr int KQ = NB / 4;              // MFMA steps per rank-NB update
    constexpr int SC = (kMaxN + BS - 1) / BS;
    constexpr int U = 2 * V;                // row tiles per MFMA group (loads in flight)
    static_assert(NB % 16 == 0 && NB <= 64 && KQ % V == 0 && BS % 64 == 0, "shape");
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_src[kMaxN];  // physical row -> its row at the start of the panel
    __shared__ int s_np[kMaxN];   // row at the start of the panel -> physical row after it
    __shared__ int s_sig[kMaxN];
    __shared__ int s_pl[NB];      // pivot row of each panel column
    __shared__ int s_mark[NB];
    __shared__ int s_out[NB];
    __shared__ uint4 s_key[2][W];  // each wave's best candidate: magnitude words, row
    __shared__ __align__(16) T s_wr[2][W][NB];
    const int j = j0 + blockIdx.x;
    if (j >= S.J) return;
    const int n = S.np, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nvb = n / V;
    const bool own = tid < n;
    T *P = reinterpret_cast<T *>(smem);  // [n][LDP]
    T *X = reinterpret_cast<T *>(S.X) + (size_t)j * n * n;

    assemble_tiled<T, BS>(S, j, X, reinterpret_cast<double *>(smem));
    int sig[SC];
    for (int t = 0; t < SC; ++t) sig[t] = tid + t * BS;
    if (tid < NB) s_mark[tid] = 0;
    __syncthreads();

    const int g = lane >> 4, li = lane & 15;
    const int nrt = n / 16, nstripe = (n - NB) / 16;
    for (int k0 = 0; k0 < n; k0 += NB) {
        // this thread's panel row, a register vector indexed by the
        // wave-uniform column (dynamic register indexing, no memory)
        typedef T Row __attribute__((ext_vector_type(NB)));
        Row pr{};
        if (own)
#pragma unroll
            for (int q = 0; q < NB; q += V) get16(pr, q, X + ((size_t)((k0 + q) / V) * n + tid) * V);
        for (int r = tid; r < n; r += BS) {
            s_src[r] = r;
            s_np[r] = r;
        }
        bool cand = own && tid >= k0;
        for (int kk = 0; kk < NB; ++kk) {
            const int par = kk & 1;
            unsigned mh = 0, ml = 0;
            if (cand) mag_key(pr[kk], mh, ml);
            const unsigned wh = wave_max_u32(mh);
            if (mh != wh) ml = 0;
            const unsigned wl = sizeof(T) == 8 ? wave_max_u32(ml) : 0u;
            const unsigned mine = cand && mh == wh && ml == wl ? (unsigned)tid : ~0u;
            const unsigned wr = wave_min_u32(mine);
            if (lane == 0) s_key[par][wave] = uint4{wh, wl, wr, 0u};
            if ((unsigned)tid == wr)
#pragma unroll
                for (int q = 0; q < NB; q += V) put16(&s_wr[par][wave][q], pr, q);
            __syncthreads();
            uint4 key[W];
#pragma unroll
            for (int w = 0; w < W; ++w) key[w] = s_key[par][w];
            unsigned bh = 0, bl = 0, br = ~0u;
            int bw = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const unsigned h = key[w].x, l = key[w].y, rw = key[w].z;
                const bool better = rw != ~0u && (h > bh || (h == bh && (l > bl || (l == bl && rw < br))));
                bh = better ? h : bh;
                bl = better ? l : bl;
                br = better ? rw : br;
                bw = better ? w : bw;
            }
            if ((bh | bl) == 0) {  // every candidate is zero
                if (tid == 0) atomicOr(&S.ctl->singular, 1);
                return;
            }
            const int p = (int)br;
            Row pn;
#pragma unroll
            for (int q = 0; q < NB; q += V) get16(pn, q, &s_wr[par][bw][q]);
            const T inv = T(1) / pn[kk];
            // one branch-free update for every row: the pivot row (equal to
            // pn) is scaled by 1/a, every other row loses fi times it; rows a
            // thread does not own are never stored
            const bool isp = tid == p;
            const T fi = isp ? T(0) : pr[kk] * inv;
            pr = (isp ? inv : T(1)) * pr - fi * pn;
            pr[kk] = isp ? inv : -fi;
            cand = cand && !isp;
            if (tid == 0) s_pl[kk] = p;
        }

        // pivot rows to k0 .. k0+NB-1, displaced block rows to the vacated rows
        __syncthreads();
        const int stamp = k0 + 1;
        int pk = -1;
        if (tid < NB) {
            pk = s_pl[tid];
            if (pk < k0 + NB) s_mark[pk - k0] = stamp;
        }
        __syncthreads();
        const bool outside = tid < NB && pk >= k0 + NB;
        const bool unchosen = tid < NB && s_mark[tid] != stamp;
        int rank_u = 0;
        if (wave == 0) {
            const unsigned long long below = (1ull << lane) - 1;
            const unsigned long long bo = __ballot(outside), bu = __ballot(unchosen);
            rank_u = __popcll(bu & below);
            if (outside) s_out[__popcll(bo & below)] = pk;
            if (tid < NB) {
                s_src[k0 + tid] = pk;
                s_np[pk] = k0 + tid;
            }
        }
        __syncthreads();
        if (unchosen) {
            const int q = s_out[rank_u];
            s_src[q] = k0 + tid;
            s_np[k0 + tid] = q;
        }
        __syncthreads();
        if (own) {
            T *dst = P + s_np[tid] * LDP;
#pragma unroll
            for (int q = 0; q < NB; q += V) put16(dst + q, pr, q);
        }
        for (int t = 0; t < SC; ++t)
            if (tid + t * BS < n) sig[t] = s_np[sig[t]];
        __syncthreads();

        // the panel is final
        for (int e = tid; e < n * (NB / V); e += BS) {
            const int r = e % n, q = e / n;
            copy16(X + ((size_t)(k0 / V + q) * n + r) * V, P + r * LDP + q * V);
        }

        // rank-NB update of every other column, one 16-column stripe per wave
        const int rt0 = ((k0 + NB) / 16) % nrt;
        for (int s = wave; s < nstripe; s += W) {
            const int c0 = (s < k0 / 16 ? s : s + NB / 16) * 16;
            // the stripe's entries of the pivot rows, read before the stripe
            // is overwritten
            T aop[KQ];
#pragma unroll
            for (int kc = 0; kc < KQ; ++kc)
                aop[kc] = X[xoff<T>(n, s_src[k0 + g * KQ + kc], c0 + mfma_row(T(), li))];
            for (int i = 0; i < nrt; i += U) {
                Q acc[U];
                int row[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int rt = (rt0 + i + u) % nrt;
                    row[u] = rt * 16 + li;
                    const bool in_block = rt * 16 >= k0 && rt * 16 < k0 + NB;
                    acc[u] = in_block ? Q{} : load_quad(X, n, s_src[row[u]], c0 + 4 * g);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    T bop[KQ];
                    const T *pr2 = P + row[u] * LDP + g * KQ;
#pragma unroll
                    for (int kc = 0; kc < KQ; kc += V) copy16(bop + kc, pr2 + kc);
#pragma unroll
                    for (int kc = 0; kc < KQ; ++kc) acc[u] = mfma16(aop[kc], bop[kc], acc[u]);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) store_quad(X, n, row[u], c0 + 4 * g, acc[u]);
            }
        }
        __syncthreads();
    }

    // X[:, c] = T[:, sigma(c)], a block of rows at a time through LDS
    for (int t = 0; t < SC; ++t)
        if (tid + t * BS < n) s_sig[tid + t * BS] = sig[t];
    const int ldl = n + 1;
    const int rb = n * LDP / ldl;
    T *L = P;
    __syncthreads();
    for (int r0 = 0; r0 < n; r0 += rb) {
        const int nr = rb < n - r0 ? rb : n - r0;
        for (int e = tid; e < nr * nvb; e += BS) {
            const int rr = e % nr, cb = e / nr;
            T v[V];
            copy16(v, X + ((size_t)cb * n + r0 + rr) * V);
            for (int u = 0; u < V; ++u) L[rr * ldl + cb * V + u] = v[u];
        }
        __syncthreads();
        for (int e = tid; e < nr * nvb; e += BS) {
            const int rr = e % nr, cb = e / nr;
            T v[V];
            for (int u = 0; u < V; ++u) v[u] = L[rr * ldl + s_sig[cb * V + u]];
            copy16(X + ((size_t)cb * n + r0 + rr) * V, v);
        }
        __syncthreads();
    }
}

// Dynamic LDS of k_gj_invert: the panel.
template <typename T, int NB>
static size_t gj_lds_bytes(int n) {
    constexpr int V = 16 / (int)sizeof(T);
    return (size_t)n * (NB + V) * sizeof(T);
}

template <typename T, int NB, int BS>
static hipError_t launch_gj(const Slab &S, int j0, int nb, hipStream_t st) {
    const void *f = reinterpret_cast<const void *>(&k_gj_invert<T, NB, BS>);
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, f);
    if (e != hipSuccess) return e;
    const size_t dyn = gj_lds_bytes<T, NB>(S.np);
    if (dyn + a.sharedSizeBytes > 160 * 1024) return hipErrorInvalidValue;
    if ((size_t)(S.N + S.G * S.G) * sizeof(double) > dyn) return hipErrorInvalidValue;  // assembly staging
    if (S.np > BS) return hipErrorInvalidValue;                                         // a row per thread
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_gj_invert<T, NB, BS>), dim3(nb), dim3(BS), dyn, st, S, j0);
    return hipGetLastError();
}

// Inverse of every 4x4 SI cell matrix L_{c,j,g,m} (eq. Aj), one thread each,
// Gauss-Jordan with partial pivoting in double.
__global__ __launch_bounds__(kBlock) void k_si_invert(Slab S) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const size_t total = (size_t)S.J * S.G * S.N;
    if (t >= total) return;
    const int m = t % S.N, g = (t / S.N) % S.G, j = t / ((size_t)S.N * S.G);
    const double dx = S.dx[j];
    const double sig = S.sigma_t[(size_t)j * S.G + g];
    const double a = dx / (S.speed[g] * S.dt);
    const double mu = S.mu[m];
    const double d = 0.5 * (fabs(mu) + dx * sig), h = 0.5 * mu;
    double M[4][8] = {{d, h, 0.5 * a, 0.0, 1, 0, 0, 0},
                      {-h, d, 0.0, 0.5 * a, 0, 1, 0, 0},
                      {-a, 0.0, a + d, h, 0, 0, 1, 0},
                      {0.0, -a, -h, a + d, 0, 0, 0, 1}};
    for (int k = 0; k < 4; ++k) {
        int p = k;
        for (int i = k + 1; i < 4; ++i)
            if (fabs(M[i][k]) > fabs(M[p][k])) p = i;
        if (M[p][k] == 0.0) { atomicOr(&S.ctl->singular, 2); return; }
        if (p != k)
            for (int c = 0; c < 8; ++c) { double tmp = M[k][c]; M[k][c] = M[p][c]; M[p][c] = tmp; }
        const double inv = 1.0 / M[k][k];
        for (int c = 0; c < 8; ++c) M[k][c] *= inv;
        for (int i = 0; i < 4; ++i)
            if (i != k) {
                const double f = M[i][k];
                for (int c = 0; c < 8; ++c) M[i][c] -= f * M[k][c];
            }
    }
    double *out = S.si_linv + t * 16;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) out[r * 4 + c] = M[r][4 + c];
    // response to the incident edges (levels k, k+1/2): mu > 0 enters rows 0
    // and 2 with +mu, mu < 0 enters rows 1 and 3 with -mu (eq. si_rhs)
    const bool pos = mu > 0.0;
    const int ca = pos ? 0 : 1, cb = pos ? 2 : 3;
    const double f = pos ? mu : -mu;
    double *rs = S.si_resp + t * 8;
    for (int r = 0; r < 4; ++r) {
        rs[r] = M[r][4 + ca] * f;
        rs[4 + r] = M[r][4 + cb] * f;
    }
    // the 2x2 map from incident to outgoing edges, stored in sweep order
    const int o0 = pos ? 1 : 0, o1 = pos ? 3 : 2;
    const int NG = S.N * S.G;
    const int step = pos ? j : S.J - 1 - j;
    double *mw = S.si_msw + ((size_t)step * NG + g * S.N + m) * 4;
    mw[0] = rs[o0];
    mw[1] = rs[4 + o0];
    mw[2] = rs[o1];
    mw[3] = rs[4 + o1];
}

// ---------------------------------------------------------------- launchers
hipError_t launch_setup(const Slab &S, bool fp32, hipStream_t st) {
    const int n = S.np;
    const int chunk = 65535;
    for (int j0 = 0; j0 < (S.wb ? 0 : S.J); j0 += chunk) {   // no n x n factors for the structured solve
        const int nb = (S.J - j0) < chunk ? (S.J - j0) : chunk;
        hipError_t e;
        if (n <= 64) {
            const size_t lds = (size_t)n * (n + 1) * (fp32 ? sizeof(float) : sizeof(double));
            if (fp32)
                hipLaunchKernelGGL((k_assemble_factor<float>), dim3(nb), dim3(kBlock), lds, st, S, j0);
            else
                hipLaunchKernelGGL((k_assemble_factor<double>), dim3(nb), dim3(kBlock), lds, st, S, j0);
            e = hipGetLastError();
        } else if (n % 32 != 0 || n > kMaxN) {
            e = hipErrorInvalidValue;
        } else if (fp32) {
            e = n >= 512 ? launch_gj<float, 32, 512>(S, j0, nb, st) : launch_gj<float, 32, 256>(S, j0, nb, st);
        } else {
            e = n >= 512 ? launch_gj<double, 16, 512>(S, j0, nb, st) : launch_gj<double, 16, 256>(S, j0, nb, st);
        }
        if (e != hipSuccess) return e;
    }
    const size_t total = (size_t)S.J * S.G * S.N;
    hipLaunchKernelGGL(k_si_invert, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S);
    return hipGetLastError();
}

}  // namespace oci
