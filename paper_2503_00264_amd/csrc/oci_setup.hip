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

// Workgroup choice of the pivot from each thread's candidate (magnitude
// `best` < 0 when it has none, row `bi`, signed value `bv`): the largest
// magnitude, the lowest row on ties.  Returns the row and sets *pa to the
// signed pivot, or returns -1 when every candidate is zero.
template <typename T, int BS>
__device__ int gj_pick(T best, int bi, T bv, T *s_wv, int *s_wi, T *pa) {
    constexpr int W = BS / 64;
    for (int off = 32; off > 0; off >>= 1) {
        const T ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        const T ov = __shfl_xor(bv, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; bv = ov; }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        s_wv[wave] = bv;
        s_wi[wave] = best < T(0) ? -1 : bi;
    }
    __syncthreads();
    T b = T(-1), v = T(0);
    int i0 = -1;
    for (int w = 0; w < W; ++w) {
        const int iw = s_wi[w];
        if (iw < 0) continue;
        const T m = fabs(s_wv[w]);
        if (m > b || (m == b && iw < i0)) { b = m; i0 = iw; v = s_wv[w]; }
    }
    *pa = v;
    return b > T(0) ? i0 : -1;
}

// Assemble the cell matrix into the cell's tiled slot of the factor buffer
// and replace it by its inverse (np >= 128, a multiple of NB and of 16).
//
// Gauss-Jordan with row exchanges: eliminating column k with pivot row p
// first swaps rows k and p, scales row k by 1/a_kk (storing 1/a_kk in place
// of a_kk) and subtracts a_ik times row k from every other row i (storing
// -a_ik/a_kk in place of a_ik).  After all n columns the matrix holds
// A^-1 with its columns permuted: X[:, c] = T[:, sigma(c)], where sigma
// applies the exchanges (k, p_k) to the column index in order k = 0, 1, ...
//
// Blocking: the NB columns [k0, k0+NB) are eliminated in LDS (panel P, all
// n rows, exchanges applied there).  Their combined effect on any other
// column x is x <- (x with its rows exchanged and rows k0..k0+NB-1 zeroed)
// + P x_piv, where x_piv holds that column's entries in the NB pivot rows
// before the panel; these rows are gathered into LDS (Bp) and the product
// runs as 16x16x4 MFMAs, one wave per 16-column stripe.  A row outside the
// pivot block whose content moved there by an exchange can only have come
// from inside the block, and each stripe writes the block's own row tiles
// last, so every read of a moved row precedes its overwrite in the same
// wave.  In the MFMA the output tile is transposed (A operand = Bp, B operand
// = P), which leaves each lane holding four consecutive columns of one row:
// one 16-byte word of the tiled layout.  The contraction index is split as
// k = (lane / 16) * NB/4 + step, so each lane reads its P operands as
// consecutive words.
template <typename T, int NB, int BS>
__global__ __launch_bounds__(BS) void k_gj_invert(Slab S, int j0) {
    using Q = typename Quad<T>::type;
    constexpr int V = 16 / (int)sizeof(T);  // elements per 16-byte word
    constexpr int LDP = NB + V;             // panel row stride (elements)
    constexpr int PADB = 16;                // Bp row padding (elements)
    constexpr int W = BS / 64;
    constexpr int KQ = NB / 4;              // MFMA steps per rank-NB update
    constexpr int SC = (kMaxN + BS - 1) / BS;
    constexpr int U = 2;                    // row tiles per MFMA group
    static_assert(NB % 16 == 0 && KQ % V == 0 && BS % 64 == 0, "shape");
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_src[kMaxN];
    __shared__ int s_sig[kMaxN];
    __shared__ T s_wv[W];
    __shared__ int s_wi[W];
    const int j = j0 + blockIdx.x;
    if (j >= S.J) return;
    const int n = S.np, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ldb = n + PADB, nvb = n / V;
    T *P = reinterpret_cast<T *>(smem);  // [n][LDP]
    T *Bp = P + (size_t)n * LDP;         // [NB][ldb]
    T *X = reinterpret_cast<T *>(S.X) + (size_t)j * n * n;

    for (int e = tid; e < n * nvb; e += BS) {
        const int r = e % n, cb = e / n;
        T v[V];
        for (int u = 0; u < V; ++u) v[u] = (T)cell_entry(S, j, r, cb * V + u);
        copy16(X + ((size_t)cb * n + r) * V, v);
    }
    int sig[SC];
    for (int t = 0; t < SC; ++t) sig[t] = tid + t * BS;
    __syncthreads();

    const int g = lane >> 4, li = lane & 15;
    const int nrt = n / 16, nstripe = (n - NB) / 16;
    for (int k0 = 0; k0 < n; k0 += NB) {
        for (int e = tid; e < n * (NB / V); e += BS) {
            const int r = e % n, q = e / n;
            copy16(P + r * LDP + q * V, X + ((size_t)(k0 / V + q) * n + r) * V);
        }
        for (int r = tid; r < n; r += BS) s_src[r] = r;
        __syncthreads();
        T pa;
        int p;
        {
            T best = T(-1), bv = T(0);
            int bi = n;
            for (int r = k0 + tid; r < n; r += BS) {
                const T v = P[r * LDP];
                if (fabs(v) > best) { best = fabs(v); bi = r; bv = v; }
            }
            p = gj_pick<T, BS>(best, bi, bv, s_wv, s_wi, &pa);
        }
        for (int kk = 0; kk < NB; ++kk) {
            const int k = k0 + kk;
            if (p < 0) {
                if (tid == 0) atomicOr(&S.ctl->singular, 1);
                return;
            }
            const T inv = T(1) / pa;
            if (tid < NB) {
                const T vk = P[k * LDP + tid], vp = P[p * LDP + tid];
                P[k * LDP + tid] = tid == kk ? inv : vp * inv;
                if (p != k) P[p * LDP + tid] = vk;
            }
            if (tid == 0 && p != k) {
                const int t = s_src[k];
                s_src[k] = s_src[p];
                s_src[p] = t;
            }
            for (int t = 0; t < SC; ++t) {
                if (sig[t] == k) sig[t] = p;
                else if (sig[t] == p) sig[t] = k;
            }
            __syncthreads();
            T best = T(-1), bv = T(0);
            int bi = n;
            const T *prow = P + k * LDP;
            for (int r = tid; r < n; r += BS) {
                T *row = P + r * LDP;
                if (r != k) {
                    const T f = row[kk];
#pragma unroll
                    for (int c = 0; c < NB; c += V) {
                        T a[V], b[V];
                        copy16(a, row + c);
                        copy16(b, prow + c);
                        for (int u = 0; u < V; ++u) a[u] -= f * b[u];
                        copy16(row + c, a);
                    }
                    row[kk] = -f * inv;
                }
                if (kk + 1 < NB && r > k) {
                    const T v = row[kk + 1];
                    if (fabs(v) > best) { best = fabs(v); bi = r; bv = v; }
                }
            }
            if (kk + 1 < NB) p = gj_pick<T, BS>(best, bi, bv, s_wv, s_wi, &pa);
            else __syncthreads();
        }

        // the panel is final: store it, and gather the pivot rows of the rest
        for (int e = tid; e < n * (NB / V); e += BS) {
            const int r = e % n, q = e / n;
            copy16(X + ((size_t)(k0 / V + q) * n + r) * V, P + r * LDP + q * V);
        }
        for (int e = tid; e < NB * nvb; e += BS) {
            const int kk = e % NB, cb = e / NB;
            if (cb >= k0 / V && cb < (k0 + NB) / V) continue;
            copy16(Bp + kk * ldb + cb * V, X + ((size_t)cb * n + s_src[k0 + kk]) * V);
        }
        __syncthreads();

        // rank-NB update of every other column, one 16-column stripe per wave
        const int rt0 = ((k0 + NB) / 16) % nrt;
        for (int s = wave; s < nstripe; s += W) {
            const int c0 = (s < k0 / 16 ? s : s + NB / 16) * 16;
            T aop[KQ];
#pragma unroll
            for (int kc = 0; kc < KQ; ++kc) aop[kc] = Bp[(g * KQ + kc) * ldb + c0 + mfma_row(T(), li)];
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
                    const T *pr = P + row[u] * LDP + g * KQ;
#pragma unroll
                    for (int kc = 0; kc < KQ; kc += V) copy16(bop + kc, pr + kc);
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
    const int rb = (n * LDP + NB * ldb) / ldl;
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

// Dynamic LDS of k_gj_invert: the panel and the gathered pivot rows.
template <typename T, int NB>
static size_t gj_lds_bytes(int n) {
    constexpr int V = 16 / (int)sizeof(T);
    return ((size_t)n * (NB + V) + (size_t)NB * (n + 16)) * sizeof(T);
}

template <typename T, int NB, int BS>
static hipError_t launch_gj(const Slab &S, int j0, int nb, hipStream_t st) {
    const void *f = reinterpret_cast<const void *>(&k_gj_invert<T, NB, BS>);
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, f);
    if (e != hipSuccess) return e;
    const size_t dyn = gj_lds_bytes<T, NB>(S.np);
    if (dyn + a.sharedSizeBytes > 160 * 1024) return hipErrorInvalidValue;
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
    for (int j0 = 0; j0 < S.J; j0 += chunk) {
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
