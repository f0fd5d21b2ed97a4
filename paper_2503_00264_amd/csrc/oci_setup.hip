// oci_setup.hip -- per-cell assembly, LU factorisation with partial pivoting
// and inversion of the one-cell-inversion systems on gfx950.
//
// One workgroup per cell.  The cell matrix (paper eqs. Aj, scatter_mg,
// fullOCIlhs) is built directly in on-chip memory (LDS) when it fits, else in
// the cell's slot of the factor buffer.  It is factored by right-looking LU
// with partial pivoting (the gesv factorisation of the paper's batched
// solver; largest |a_ik| is the pivot, the lowest row winning ties) and then
// inverted in place from its factors the way LAPACK's getri does: invert U,
// solve X L = U^-1, undo the row exchanges as column exchanges.  Every later
// iteration applies the result as one matrix-vector product per cell, which
// keeps all lanes busy where the two triangular substitutions of getrs would
// be a dependent chain of n steps.  Work precision T is float for the
// refined path and double for the FP64 path; assembly arithmetic is double
// and rounded once to T.
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
        const double L[16] = {d, h, 0.5 * a, 0.0,
                              -h, d, 0.0, 0.5 * a,
                              -a, 0.0, a + d, h,
                              0.0, -a, -h, a + d};
        v = L[ur * 4 + uc];
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

// Assemble, factor and invert the matrix of one cell per workgroup.
// USE_LDS: work in LDS (dynamic shared, n x (n+1) of T), then store tiled.
template <typename T, bool USE_LDS>
__global__ __launch_bounds__(kBlock) void k_assemble_factor(Slab S, int j0) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_piv[kMaxN];
    __shared__ T s_work[kMaxN];
    const int j = j0 + blockIdx.x;
    if (j >= S.J) return;
    const int n = S.np;
    T *Xj = reinterpret_cast<T *>(S.X) + (size_t)j * n * n;
    bool ok;
    if (USE_LDS) {
        LdsMat<T> A{reinterpret_cast<T *>(smem), n + 1};
        for (int e = threadIdx.x; e < n * n; e += kBlock) {
            const int r = e / n, c = e % n;
            A(r, c) = (T)cell_entry(S, j, r, c);
        }
        __syncthreads();
        ok = factor_invert<T>(A, n, s_piv, s_work);
        if (ok) {
            TiledMat<T> X{Xj, n};
            for (int e = threadIdx.x; e < n * n; e += kBlock) {
                const int r = e / n, c = e % n;
                X(r, c) = A(r, c);
            }
        }
    } else {
        TiledMat<T> A{Xj, n};
        for (int e = threadIdx.x; e < n * n; e += kBlock) {
            const int r = e / n, c = e % n;
            A(r, c) = (T)cell_entry(S, j, r, c);
        }
        __syncthreads();
        ok = factor_invert<T>(A, n, s_piv, s_work);
    }
    if (!ok && threadIdx.x == 0) atomicOr(&S.ctl->singular, 1);
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
    const size_t lds64 = (size_t)n * (n + 1) * sizeof(double);
    const size_t lds32 = (size_t)n * (n + 1) * sizeof(float);
    const int chunk = 65535;
    for (int j0 = 0; j0 < S.J; j0 += chunk) {
        const int nb = (S.J - j0) < chunk ? (S.J - j0) : chunk;
        if (fp32) {
            if (lds32 <= 64 * 1024)
                hipLaunchKernelGGL((k_assemble_factor<float, true>), dim3(nb), dim3(kBlock), lds32, st, S, j0);
            else
                hipLaunchKernelGGL((k_assemble_factor<float, false>), dim3(nb), dim3(kBlock), 0, st, S, j0);
        } else {
            if (lds64 <= 64 * 1024)
                hipLaunchKernelGGL((k_assemble_factor<double, true>), dim3(nb), dim3(kBlock), lds64, st, S, j0);
            else
                hipLaunchKernelGGL((k_assemble_factor<double, false>), dim3(nb), dim3(kBlock), 0, st, S, j0);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const size_t total = (size_t)S.J * S.G * S.N;
    hipLaunchKernelGGL(k_si_invert, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S);
    return hipGetLastError();
}

}  // namespace oci
