// FP64 truncated split of the two-site tensor through the Gram matrix, a
// Householder tridiagonal reduction and a divide-and-conquer eigensolver.
//
// The split of Sec. 2.3 needs, for the side the isometry centre leaves, an
// orthonormal basis of the leading singular subspace of the rows X (nv x n)
// and the singular values (for the truncation rule and the discarded weight).
// Those are the eigenvectors of H = X^T X (n x n).  Here:
//   1. H = X^T X by the FP64 MFMA product (a separate launch);
//   2. gtd_eig_kernel, one workgroup with H in LDS (n <= GTD_MAX_N):
//      Householder reduction H = P T P^T (T tridiagonal), the eigenpairs of T
//      by Cuppen's divide and conquer with the deflation rules of Dongarra and
//      Sorensen, secular roots by the rational two-pole iteration of Li's
//      "middle way", eigenvectors from the Loewner form of Gu and Eisenstat (so
//      they are orthogonal to working precision), and the back-transformation
//      V = P Z; V^T is written out (row i = eigenvector i);
//   3. W = V^T X^T by the FP64 MFMA product: row i is (X v_i)^T, whose norm is
//      the singular value s_i computed without squaring the rounding of H;
//   4. gtd_select_kernel: descending order, the truncation rule and the
//      discarded weight (tail summed from the smallest value up), and the kept
//      rows Q_i = v_i^T (orthonormal by construction, also for tiny s_i).
// The singular subspaces come from an exact eigendecomposition of a matrix
// within eps * ||X||^2 of X^T X: a backward perturbation of X of order
// eps * ||X||, far below what the truncation tolerances resolve.

#include <cfloat>

#include "common.h"
#include "select.h"

namespace smps {

constexpr int GTD_NT = 1024;  // threads of the eigensolver workgroup
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int GTD_MAX_N = 128;

// rows of the 16-lane DPP groups
template <int CTRL>
__device__ __forceinline__ double gtd_dpp(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double sum16(double x) {
    x += gtd_dpp<0xB1>(x);
    x += gtd_dpp<0x4E>(x);
    x += gtd_dpp<0x141>(x);
    x += gtd_dpp<0x140>(x);
    return x;
}
__device__ __forceinline__ double prod16(double x) {
    x *= gtd_dpp<0xB1>(x);
    x *= gtd_dpp<0x4E>(x);
    x *= gtd_dpp<0x141>(x);
    x *= gtd_dpp<0x140>(x);
    return x;
}
__device__ __forceinline__ double sum64(double x) {
    x = sum16(x);
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
}

// Sums and products over a group of G lanes (G = 16: a DPP row; 4: a quad; 1: one lane).
template <int G>
__device__ __forceinline__ double gsum(double x) {
    if constexpr (G == 16) return sum16(x);
    else if constexpr (G == 4) {
        x += gtd_dpp<0xB1>(x);
        x += gtd_dpp<0x4E>(x);
        return x;
    } else return x;
}
template <int G>
__device__ __forceinline__ double gprod(double x) {
    if constexpr (G == 16) return prod16(x);
    else if constexpr (G == 4) {
        x *= gtd_dpp<0xB1>(x);
        x *= gtd_dpp<0x4E>(x);
        return x;
    } else return x;
}

// Root j of 1/rho + sum_i z2_i / (dl_i - lambda) = 0 (dl ascending, z2 > 0)
// on a group of G lanes (terms strided over the lanes; every lane ends with
// the same result).  The root is returned as an origin pole o and an offset
// tau (lambda = dl[o] + tau) so that dl_i - lambda = (dl_i - dl_o) - tau keeps
// full relative accuracy near the pole.  Iteration: the two nearest poles are
// kept exactly and the rest of each side is fitted by a constant plus one pole
// (value and slope), the resulting quadratic is solved for the step, and any
// step leaving the bracket is replaced by bisection.
template <int G>
__device__ void gtd_secular(const double* dl, const double* z2, int K, double rho, int j, int gl, int* o_out,
                            double* tau_out) {
    const double irho = 1.0 / rho;
    int o;
    double lo, hi, tau;
    if (j < K - 1) {
        const double gap = dl[j + 1] - dl[j];
        const double h = 0.5 * gap;
        double part = 0.0;
        for (int i = gl; i < K; i += G) part += z2[i] / ((dl[i] - dl[j]) - h);
        double fm = irho + gsum<G>(part);
        if (fm >= 0.0) {
            o = j;
            lo = 0.0;
            hi = h;
        } else {
            o = j + 1;
            lo = -h;
            hi = 0.0;
        }
        tau = 0.5 * (lo + hi);
    } else {
        o = K - 1;
        double part = 0.0;
        for (int i = gl; i < K; i += G) part += z2[i];
        const double zz = gsum<G>(part);
        lo = 0.0;
        hi = rho * zz;
        tau = 0.5 * hi;
    }
    const double dlo = dl[o];
    for (int it = 0; it < 64; ++it) {
        double ps = 0.0, dps = 0.0, ph = 0.0, dph = 0.0, ab = 0.0;
        for (int i = gl; i < K; i += G) {
            const double del = (dl[i] - dlo) - tau;
            const double r = 1.0 / del;
            const double t = z2[i] * r;
            const double td = t * r;
            if (i <= j) {
                ps += t;
                dps += td;
            } else {
                ph += t;
                dph += td;
            }
            ab += fabs(t);
        }
        ps = gsum<G>(ps);
        dps = gsum<G>(dps);
        ph = gsum<G>(ph);
        dph = gsum<G>(dph);
        ab = gsum<G>(ab);
        const double f = irho + ps + ph;
        if (fabs(f) <= 8.0 * DBL_EPSILON * (irho + ab) * (double)K) break;
        if (f < 0.0)
            lo = tau;
        else
            hi = tau;
        const double Da = (dl[j] - dlo) - tau;
        double eta;
        if (j < K - 1) {
            const double Db = (dl[j + 1] - dlo) - tau;
            const double C = f - Da * dps - Db * dph;
            const double A = (Da + Db) * f - Da * Db * (dps + dph);
            const double B = Da * Db * f;
            const double disc = sqrt(fabs(A * A - 4.0 * B * C));
            if (A > 0.0)
                eta = 2.0 * B / (A + disc);
            else
                eta = C != 0.0 ? (A - disc) / (2.0 * C) : -f / (dps + dph);
        } else {
            const double C = f - Da * dps;
            eta = C != 0.0 ? Da + Da * Da * dps / C : -f / dps;
        }
        double nt = tau + eta;
        if (!(nt > lo && nt < hi)) nt = 0.5 * (lo + hi);
        const bool stop = nt == tau || hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi));
        tau = nt;
        if (stop) break;
    }
    *o_out = o;
    *tau_out = tau;
}

// LDS layout of gtd_eig_kernel (n = live order):
//   A   n (n + 1) doubles: H during the reduction (row stride n + 1); the
//       per-node coefficient blocks Y of one divide-and-conquer depth (node
//       [a, b) at A + a S, S the largest node at that depth); the eigenvector
//       rows during the back-transformation (row stride n + 1)
//   16 arrays of n doubles and 8 of n ints (reflector, split and merge data)
//   3 arrays of 130 ints (per-node counts of one depth)
struct GtdLds {
    double *A, *d, *e, *tau, *pp, *vv, *ds, *zs, *dl, *zl, *zh, *rt, *lv, *rc, *rs;
    int *idx, *ip, *ndf, *dfl, *ro, *fp, *rp, *rn, *nk, *nr, *nd;
};

__host__ __device__ inline size_t gtd_lds_bytes(int n) {
    return sizeof(double) * ((size_t)n * (n + 1) + 16 * (size_t)n) + sizeof(int) * (8 * (size_t)n + 3 * 130) + 64;
}

__device__ GtdLds gtd_carve(double* sm, int n) {
    GtdLds s;
    double* p = sm;
    s.A = p;
    p += (size_t)n * (n + 1);
    double** arr[] = {&s.d, &s.e, &s.tau, &s.pp, &s.vv, &s.ds, &s.zs, &s.dl,
                      &s.zl, &s.zh, &s.rt, &s.lv, &s.rc, &s.rs};
    for (double** a : arr) {
        *a = p;
        p += n;
    }
    p += 2 * (size_t)n;  // spare (16 arrays reserved)
    int* q = (int*)p;
    int** iarr[] = {&s.idx, &s.ip, &s.ndf, &s.dfl, &s.ro, &s.fp, &s.rp, &s.rn};
    for (int** a : iarr) {
        *a = q;
        q += n;
    }
    int** narr[] = {&s.nk, &s.nr, &s.nd};
    for (int** a : narr) {
        *a = q;
        q += 130;
    }
    return s;
}

struct GtdDesc {
    const double* H;    // n x n Gram matrix (row-major, symmetric)
    const int* dims;    // live sizes
    DimExpr n;          // matrix order
    double* Vt;         // n x n out: row i = unit eigenvector of the i-th smallest eigenvalue
    double* refl;       // n x n scratch: Householder vectors (row k: v_k at columns k+1..n-1)
    double* Qa;         // n x n scratch (divide and conquer, ping): row c = eigenvector c
    double* Qb;         // n x n scratch (pong)
    int* status;        // bit 0: non-finite input
};

// Node at depth t containing row x (the split tree of [0, n), splits at
// a + (b - a) / 2): its interval and index.
__device__ __forceinline__ void gtd_locate(int n, int t, int x, int* a_out, int* b_out, int* q_out) {
    int a = 0, b = n, q = 0;
    for (int l = 0; l < t; ++l) {
        const int mid = a + (b - a) / 2;
        q <<= 1;
        if (x >= mid) {
            a = mid;
            q |= 1;
        } else {
            b = mid;
        }
    }
    *a_out = a;
    *b_out = b;
    *q_out = q;
}

// Secular roots, Loewner weights and the coefficient columns of one depth,
// G lanes per root / weight / column.
template <int G>
__device__ void gtd_roots_and_columns(const GtdLds& s, int n, int t, int S) {
    const int tid = threadIdx.x, gl = tid & (G - 1), grp = tid / G;
    constexpr int NG = GTD_NT / G;
    // roots
    for (int x = grp; x < n; x += NG) {
        int a, b, q;
        gtd_locate(n, t, x, &a, &b, &q);
        if (b - a < 2) continue;
        const int j = x - a, K = s.nk[q];
        if (j >= K) continue;
        const int mid = a + (b - a) / 2;
        const double rho = 2.0 * fabs(s.e[mid - 1]);
        int o;
        double tu;
        gtd_secular<G>(s.dl + a, s.zh + a, K, rho, j, gl, &o, &tu);
        if (gl == 0) {
            s.ro[a + j] = o;
            s.rt[a + j] = tu;
        }
    }
    __syncthreads();
    // Loewner weights zhat_i^2 = (-delta_ii / rho) prod_{j != i} (-delta_ij) / (dl_j - dl_i)
    for (int x = grp; x < n; x += NG) {
        int a, b, q;
        gtd_locate(n, t, x, &a, &b, &q);
        if (b - a < 2) continue;
        const int i = x - a, K = s.nk[q];
        if (i >= K) continue;
        const int mid = a + (b - a) / 2;
        const double rho = 2.0 * fabs(s.e[mid - 1]);
        const double di = s.dl[a + i];
        double pr = 1.0;
        for (int j = gl; j < K; j += G) {
            const double del = (di - s.dl[a + s.ro[a + j]]) - s.rt[a + j];
            pr *= j == i ? -del / rho : -del / (s.dl[a + j] - di);
        }
        pr = gprod<G>(pr);
        if (gl == 0) s.pp[a + i] = copysign(sqrt(fmax(pr, 0.0)), s.zl[a + i]);
    }
    __syncthreads();
    // final ascending order (roots merged with the deflated values); zero Y
    for (int x = tid; x < n; x += GTD_NT) {
        int a, b, q;
        gtd_locate(n, t, x, &a, &b, &q);
        const int sz = b - a;
        if (sz < 2) continue;
        const int c = x - a, K = s.nk[q], nd = s.nd[q];
        if (c < K) {
            const double lam = s.dl[a + s.ro[a + c]] + s.rt[a + c];
            int lo = 0, hi = nd;
            while (lo < hi) {
                const int md = (lo + hi) >> 1;
                if (s.ds[a + s.dfl[a + md]] < lam)
                    lo = md + 1;
                else
                    hi = md;
            }
            s.fp[a + c] = c + lo;
            s.vv[a + c] = lam;
        } else {
            const int u = c - K;
            const double dv = s.ds[a + s.dfl[a + u]];
            int lo = 0, hi = K;
            while (lo < hi) {
                const int md = (lo + hi) >> 1;
                if (s.dl[a + s.ro[a + md]] + s.rt[a + md] <= dv)
                    lo = md + 1;
                else
                    hi = md;
            }
            s.fp[a + c] = u + lo;
            s.vv[a + c] = dv;
        }
        double* Y = s.A + (size_t)a * S + (size_t)c * sz;
        for (int k = 0; k < sz; ++k) Y[k] = 0.0;
    }
    __syncthreads();
    // coefficient columns: c < K the normalised Loewner vector at the
    // non-deflated positions; K + u the unit vector of deflated position u
    for (int x = grp; x < n; x += NG) {
        int a, b, q;
        gtd_locate(n, t, x, &a, &b, &q);
        const int sz = b - a;
        if (sz < 2) continue;
        const int c = x - a, K = s.nk[q];
        double* Y = s.A + (size_t)a * S;
        if (c < K) {
            const int o = s.ro[a + c];
            const double tu = s.rt[a + c], dlo = s.dl[a + o];
            double nn = 0.0;
            for (int i = gl; i < K; i += G) {
                const double w = s.pp[a + i] / ((s.dl[a + i] - dlo) - tu);
                nn = fma(w, w, nn);
            }
            nn = gsum<G>(nn);
            const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
            for (int i = gl; i < K; i += G) {
                const double w = nn > 0.0 ? s.pp[a + i] / ((s.dl[a + i] - dlo) - tu) * inv : (i == c ? 1.0 : 0.0);
                Y[(size_t)s.ndf[a + i] * sz + c] = w;
            }
        } else if (gl == 0) {
            Y[(size_t)s.dfl[a + (c - K)] * sz + c] = 1.0;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(GTD_NT) void gtd_eig_kernel(GtdDesc g) {
    extern __shared__ double sm[];
    const int n = eval_dim(g.dims, g.n);
    const int tid = threadIdx.x, lane = tid & 63, gl = tid & 15, grp = tid >> 4;
    const int ld = n + 1;
    GtdLds s = gtd_carve(sm, n);
    double* A = s.A;
    __shared__ int s_bad;
    __shared__ double s_tau[2], s_kc;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int i = grp; i < n; i += GTD_NT / 16)
        for (int j = gl; j < n; j += 16) {
            const double v = g.H[(size_t)i * n + j];
            if (!isfinite(v)) s_bad = 1;
            A[i * ld + j] = v;
        }
    __syncthreads();
    if (s_bad) {
        for (int i = grp; i < n; i += GTD_NT / 16)
            for (int j = gl; j < n; j += 16) g.Vt[(size_t)i * n + j] = i == j ? 1.0 : 0.0;
        if (tid == 0 && g.status) atomicOr(g.status, 1);
        return;
    }
    // ---- 1. Householder reduction to tridiagonal form, H in LDS (row stride
    // n + 1).  The update keeps H exactly symmetric, so column r below the
    // diagonal is read as row r right of it.  The 16-lane group that owns row
    // r once it is final forms its reflector (beta, tau and v, the last stored
    // over row r right of the diagonal for the back-transformation) and hands
    // v to the next step through vbuf[r & 1]; K = tau/2 p^T v and w = p - K v
    // are formed by wave 0.
    double* vbuf[2] = {s.vv, s.zl};
    double* wv = s.dl;
    // reflector of row r (called by one whole 16-lane group)
    auto reflector = [&](int r) {
        double* row = A + r * ld;
        if (gl == 0) s.d[r] = row[r];
        if (r + 1 >= n) return;
        double part = 0.0;
        for (int j = r + 2 + gl; j < n; j += 16) part = fma(row[j], row[j], part);
        const double xn2 = sum16(part), x0 = row[r + 1];
        double beta, tau, scale;
        if (xn2 == 0.0 || r + 2 >= n) {
            beta = x0;
            tau = 0.0;
            scale = 0.0;
        } else {
            beta = -copysign(sqrt(fma(x0, x0, xn2)), x0);
            tau = (beta - x0) / beta;
            scale = 1.0 / (x0 - beta);
        }
        double* vout = vbuf[r & 1];
        for (int j = r + 1 + gl; j < n; j += 16) {
            const double v = j == r + 1 ? 1.0 : (tau != 0.0 ? row[j] * scale : 0.0);
            vout[j - r - 1] = v;
            row[j] = v;
        }
        if (gl == 0) {
            s.e[r] = beta;
            s.tau[r] = tau;
            s_tau[r & 1] = tau;
        }
    };
    if (grp == 0) reflector(0);
    __syncthreads();
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        const double tau = s_tau[k & 1];
        const double* vv = vbuf[k & 1];
        if (tau != 0.0) {
            // p = tau S v, S the trailing block; one 16-lane group per row
            for (int i = grp; i < m; i += GTD_NT / 16) {
                const double* row = A + (k + 1 + i) * ld + (k + 1);
                double acc = 0.0;
                for (int j = gl; j < m; j += 16) acc = fma(row[j], vv[j], acc);
                acc = sum16(acc);
                if (gl == 0) s.pp[i] = tau * acc;
            }
            __syncthreads();
            if (tid < 64) {
                double pk = 0.0;
                for (int i = lane; i < m; i += 64) pk = fma(s.pp[i], vv[i], pk);
                const double Kc = 0.5 * tau * sum64(pk);
                for (int i = lane; i < m; i += 64) wv[i] = s.pp[i] - Kc * vv[i];
            }
            __syncthreads();
            // S -= (v_i w_j) + (w_i v_j): the same two products in either order,
            // so the block stays exactly symmetric
            for (int i = grp; i < m; i += GTD_NT / 16) {
                const double vi = vv[i], wi = wv[i];
                double* row = A + (k + 1 + i) * ld + (k + 1);
                for (int j = gl; j < m; j += 16) row[j] -= (vi * wv[j]) + (wi * vv[j]);
                if (i == 0) reflector(k + 1);  // row k + 1 is final: the next step's reflector
            }
        } else if (grp == 0) {
            reflector(k + 1);
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (n >= 2) {
            s.d[n - 2] = A[(n - 2) * ld + (n - 2)];
            s.e[n - 2] = A[(n - 1) * ld + (n - 2)];
            s.tau[n - 2] = 0.0;
        }
        s.d[n - 1] = A[(n - 1) * ld + (n - 1)];
        s.tau[n - 1] = 0.0;
    }
    __syncthreads();
    // reflector k sits in row k right of the diagonal; zero elsewhere
    for (int k = grp; k + 2 < n; k += GTD_NT / 16)
        if (s.tau[k] != 0.0)
            for (int j = gl; j < n; j += 16) g.refl[(size_t)k * n + j] = j > k ? A[k * ld + j] : 0.0;
    // ---- 2. divide and conquer on (d, e), leaves of one row.  Every e_i
    // couples one split, so a leaf carries d_i - |e_{i-1}| - |e_i|.  Qc row c
    // is eigenvector c of its node (entries at the node's rows).
    double* Qc = g.Qa;
    double* Qn = g.Qb;
    for (int i = tid; i < n; i += GTD_NT) {
        const double el = i > 0 ? fabs(s.e[i - 1]) : 0.0, er = i + 1 < n ? fabs(s.e[i]) : 0.0;
        s.lv[i] = s.d[i] - el - er;
        Qc[(size_t)i * n + i] = 1.0;
    }
    int depth = 0;
    while ((1 << depth) < n) ++depth;
    __syncthreads();
    for (int t = depth - 1; t >= 0; --t) {
        int S;
        {
            int a, b, q;
            gtd_locate(n, t, n - 1, &a, &b, &q);
            S = b - a;  // the rightmost node is the largest at its depth
        }
        // z (last row of the left child's vectors, sign-adjusted first row of
        // the right child's) in the merged ascending order of the eigenvalues
        for (int x = tid; x < n; x += GTD_NT) {
            int a, b, q;
            gtd_locate(n, t, x, &a, &b, &q);
            const int sz = b - a;
            if (sz < 2) continue;
            const int mid = a + sz / 2, m = mid - a, c = x - a;
            const double dv = s.lv[x];
            double zv;
            int pos;
            if (c < m) {
                zv = Qc[(size_t)x * n + (mid - 1)];
                int lo = 0, hi = sz - m;  // right-child values below dv
                while (lo < hi) {
                    const int md = (lo + hi) >> 1;
                    if (s.lv[mid + md] < dv)
                        lo = md + 1;
                    else
                        hi = md;
                }
                pos = c + lo;
            } else {
                zv = (s.e[mid - 1] >= 0.0 ? 1.0 : -1.0) * Qc[(size_t)x * n + mid];
                int lo = 0, hi = m;  // left-child values not above dv
                while (lo < hi) {
                    const int md = (lo + hi) >> 1;
                    if (s.lv[a + md] <= dv)
                        lo = md + 1;
                    else
                        hi = md;
                }
                pos = (c - m) + lo;
            }
            s.ds[a + pos] = dv;
            s.zs[a + pos] = zv * 0.70710678118654752440;  // z / sqrt(2): unit norm, rho -> 2 rho
            s.idx[a + pos] = c;
            s.ip[x] = pos;
        }
        __syncthreads();
        // deflation, one thread per node: negligible z components, and close
        // neighbours whose z pair a rotation moves onto one member
        for (int q = tid; q < (1 << t); q += GTD_NT) {
            int a, b;
            {
                int lo = 0, hi = n;
                for (int l = t - 1; l >= 0; --l) {
                    const int mid = lo + (hi - lo) / 2;
                    if ((q >> l) & 1)
                        lo = mid;
                    else
                        hi = mid;
                }
                a = lo;
                b = hi;
            }
            const int sz = b - a;
            if (sz < 2) continue;
            const int mid = a + sz / 2;
            const double rho = 2.0 * fabs(s.e[mid - 1]);
            const double tol = 8.0 * DBL_EPSILON * fmax(fmax(fabs(s.ds[a]), fabs(s.ds[b - 1])), rho);
            int K = 0, nd = 0, nr = 0, pj = -1;
            auto defl_insert = [&](int x) {  // deflated list kept in ascending value order
                const double v = s.ds[a + x];
                int u = nd - 1;
                while (u >= 0 && s.ds[a + s.dfl[a + u]] > v) {
                    s.dfl[a + u + 1] = s.dfl[a + u];
                    --u;
                }
                s.dfl[a + u + 1] = x;
                ++nd;
            };
            for (int nj = 0; nj < sz; ++nj) {
                const double zn = s.zs[a + nj];
                if (rho * fabs(zn) <= tol) {
                    defl_insert(nj);
                    continue;
                }
                if (pj < 0) {
                    pj = nj;
                    continue;
                }
                const double gap = s.ds[a + nj] - s.ds[a + pj];
                if (gap > 2.0 * tol) {  // |c s| <= 1/2: no rotation can deflate
                    s.ndf[a + K++] = pj;
                    pj = nj;
                    continue;
                }
                const double zp = s.zs[a + pj];
                const double tt = hypot(zn, zp);
                const double c = zn / tt, sn = -zp / tt;
                if (fabs(gap * c * sn) <= tol) {
                    s.zs[a + nj] = tt;
                    s.zs[a + pj] = 0.0;
                    s.rp[a + nr] = pj;
                    s.rn[a + nr] = nj;
                    s.rc[a + nr] = c;
                    s.rs[a + nr] = sn;
                    ++nr;
                    const double dp = s.ds[a + pj], dn = s.ds[a + nj];
                    s.ds[a + pj] = dp * c * c + dn * sn * sn;
                    s.ds[a + nj] = dp * sn * sn + dn * c * c;
                    defl_insert(pj);
                    pj = nj;
                } else {
                    s.ndf[a + K++] = pj;
                    pj = nj;
                }
            }
            if (pj >= 0) s.ndf[a + K++] = pj;
            s.nk[q] = K;
            s.nr[q] = nr;
            s.nd[q] = nd;
        }
        __syncthreads();
        // the non-deflated values and weights in ascending order
        for (int x = tid; x < n; x += GTD_NT) {
            int a, b, q;
            gtd_locate(n, t, x, &a, &b, &q);
            if (b - a < 2 || x - a >= s.nk[q]) continue;
            const int p = s.ndf[x];
            s.dl[x] = s.ds[a + p];
            s.zl[x] = s.zs[a + p];
            s.zh[x] = s.zs[a + p] * s.zs[a + p];
        }
        __syncthreads();
        if (S > 32)
            gtd_roots_and_columns<16>(s, n, t, S);
        else if (S > 8)
            gtd_roots_and_columns<4>(s, n, t, S);
        else
            gtd_roots_and_columns<1>(s, n, t, S);
        // the deflation rotations act on the rows of Y (last rotation first)
        for (int x = tid; x < n; x += GTD_NT) {
            int a, b, q;
            gtd_locate(n, t, x, &a, &b, &q);
            const int sz = b - a;
            if (sz < 2) continue;
            const int c = x - a, nr = s.nr[q];
            double* Y = s.A + (size_t)a * S;
            for (int r = nr - 1; r >= 0; --r) {
                const int pj = s.rp[a + r], nj = s.rn[a + r];
                const double cc = s.rc[a + r], sn = s.rs[a + r];
                const double yp = Y[(size_t)pj * sz + c], yn = Y[(size_t)nj * sz + c];
                Y[(size_t)pj * sz + c] = cc * yp - sn * yn;
                Y[(size_t)nj * sz + c] = sn * yp + cc * yn;
            }
        }
        __syncthreads();
        // new vectors: eigenvector c of the node (row a + fp(c) of Qn) at node
        // row r is sum over the block's columns col of Qc[a + col][a + r] Y[ip(col)][c],
        // where only columns of the child that owns row r contribute
        if (S >= 32) {
            // FP64 MFMA 16 x 16 x 4 tiles (c, r) over the owning child's columns;
            // each wave takes whole tiles
            const int wave = tid >> 6, li = lane & 15, lk = lane >> 4;
            for (int q = 0; q < (1 << t); ++q) {
                int a = 0, b = n;
                for (int l = t - 1; l >= 0; --l) {
                    const int mid = a + (b - a) / 2;
                    if ((q >> l) & 1)
                        a = mid;
                    else
                        b = mid;
                }
                const int sz = b - a;
                if (sz < 2) continue;
                const int m = sz / 2, ct = (sz + 15) / 16, rt0 = (m + 15) / 16, rt1 = (sz - m + 15) / 16;
                const double* Y = s.A + (size_t)a * S;
                for (int tl = wave; tl < ct * (rt0 + rt1); tl += GTD_NT / 64) {
                    const int ci = tl / (rt0 + rt1), ri = tl - ci * (rt0 + rt1);
                    const bool top = ri < rt0;
                    const int r0 = top ? 16 * ri : m + 16 * (ri - rt0), rend = top ? m : sz;
                    const int k0 = top ? 0 : m, k1 = top ? m : sz, c0 = 16 * ci;
                    v4d acc = {0.0, 0.0, 0.0, 0.0};
                    for (int kk = k0; kk < k1; kk += 4) {
                        const int col = kk + lk, c = c0 + li, r = r0 + li;
                        const double av = (col < k1 && c < sz) ? Y[(size_t)s.ip[a + col] * sz + c] : 0.0;
                        const double bv = (col < k1 && r < rend) ? Qc[(size_t)(a + col) * n + a + r] : 0.0;
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                    }
                    // v_mfma_f64_16x16x4 returns rows lk + 4 v, column li
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int c = c0 + lk + 4 * v, r = r0 + li;
                        if (c < sz && r < rend) Qn[(size_t)(a + s.fp[a + c]) * n + a + r] = acc[v];
                    }
                }
            }
        } else {
            for (int x = tid; x < n * ((S + 3) / 4); x += GTD_NT) {
                const int xr = x / ((S + 3) / 4), tile = x - xr * ((S + 3) / 4);
                int a, b, q;
                gtd_locate(n, t, xr, &a, &b, &q);
                const int sz = b - a;
                const int r0 = 4 * tile;
                if (sz < 2 || r0 >= sz) continue;
                const int m = sz / 2, c = xr - a;
                const double* Y = s.A + (size_t)a * S;
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                const int r1 = min(r0 + 4, sz);
                for (int u = 0; u < r1 - r0; ++u) {
                    const int r = r0 + u;
                    const int c0 = r >= m ? m : 0, c1 = r >= m ? sz : m;
                    for (int col = c0; col < c1; ++col)
                        acc[u] = fma(Qc[(size_t)(a + col) * n + a + r], Y[(size_t)s.ip[a + col] * sz + c], acc[u]);
                }
                double* out = Qn + (size_t)(a + s.fp[a + c]) * n + a;
                for (int u = 0; u < r1 - r0; ++u) out[r0 + u] = acc[u];
            }
        }
        __syncthreads();
        for (int x = tid; x < n; x += GTD_NT) {
            int a, b, q;
            gtd_locate(n, t, x, &a, &b, &q);
            if (b - a >= 2)
                s.lv[a + s.fp[x]] = s.vv[x];
            else if (b - a == 1)
                Qn[(size_t)x * n + x] = Qc[(size_t)x * n + x];  // a leaf reached at this depth
        }
        __syncthreads();
        double* sw = Qc;
        Qc = Qn;
        Qn = sw;
    }
    // ---- 3. back-transformation: V^T = Z^T P^T.  Each row of Z^T (= Qc, an
    // eigenvector in the tridiagonal basis) takes the reflectors from the
    // right, last first, independently of the other rows: a 16-lane group
    // keeps two rows in registers (8 elements per lane) and reads the
    // reflectors from LDS, so no barrier is needed between reflectors.
    // the reflectors of the reduction: saved to global memory before divide
    // and conquer took the LDS (rows with tau = 0 are never read)
    for (int k = grp; k + 2 < n; k += GTD_NT / 16)
        if (s.tau[k] != 0.0)
            for (int j = gl; j < n; j += 16) A[k * ld + j] = g.refl[(size_t)k * n + j];
    __syncthreads();
    constexpr int BE = GTD_MAX_N / 16;
    for (int c0 = 2 * grp; c0 < n; c0 += 2 * (GTD_NT / 16)) {
        const int c1 = c0 + 1;
        double x0[BE], x1[BE];
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int j = gl + 16 * e;
            x0[e] = j < n ? Qc[(size_t)c0 * n + j] : 0.0;
            x1[e] = (j < n && c1 < n) ? Qc[(size_t)c1 * n + j] : 0.0;
        }
        for (int k = n - 3; k >= 0; --k) {
            const double tk = s.tau[k];
            if (tk == 0.0) continue;  // uniform
            const double* v = A + k * ld;  // zero at columns <= k
            const int e0 = (k + 1) >> 4;   // elements below e0 are at columns <= k for every lane
            double vr[BE];
#pragma unroll
            for (int e = 0; e < BE; ++e) vr[e] = (e >= e0 && gl + 16 * e < n) ? v[gl + 16 * e] : 0.0;
            double d0 = 0.0, d1 = 0.0;
#pragma unroll
            for (int e = 0; e < BE; ++e)
                if (e >= e0) {
                    d0 = fma(x0[e], vr[e], d0);
                    d1 = fma(x1[e], vr[e], d1);
                }
            d0 = sum16(d0) * tk;
            d1 = sum16(d1) * tk;
#pragma unroll
            for (int e = 0; e < BE; ++e)
                if (e >= e0) {
                    x0[e] = fma(-d0, vr[e], x0[e]);
                    x1[e] = fma(-d1, vr[e], x1[e]);
                }
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int j = gl + 16 * e;
            if (j < n) {
                g.Vt[(size_t)c0 * n + j] = x0[e];
                if (c1 < n) g.Vt[(size_t)c1 * n + j] = x1[e];
            }
        }
    }
}

// select + write: rows of W = V^T X^T (norm = s_i), descending order, the
// truncation rule (shared with the Jacobi path), kept rows of V^T, the basis.

constexpr int GTD_SEL_MAX = 1024;

__global__ __launch_bounds__(1024) void gtd_select_kernel(JacobiDesc d, const double* W, const double* Vt) {
    __shared__ double sig_raw[GTD_SEL_MAX];
    __shared__ double sig_sorted[GTD_SEL_MAX];
    __shared__ int perm[GTD_SEL_MAX];
    __shared__ double s_delta;
    const int n = eval_dim(d.dims_in, d.len), nv = eval_dim(d.dims_in, d.nvec);
    const int r = jacobi_select(W, n, nv, nv, sig_raw, sig_sorted, perm, d, &s_delta);
    if (threadIdx.x == 0 && d.log_sweeps) *d.log_sweeps = 0;
    for (int e = threadIdx.x; e < r * n; e += blockDim.x) {
        const int i = e / n, l = e - i * n;
        d.Q[e] = Vt[(size_t)perm[i] * n + l];
    }
    if (d.basis)
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
            const int i = e / n, l = e - i * n;
            d.basis[e] = Vt[(size_t)perm[i] * n + l];
        }
}

static int g_gtd_ok = 0;

hipError_t gtd_init() {
    const size_t need = gtd_lds_bytes(GTD_MAX_N);
    hipError_t e = hipFuncSetAttribute((const void*)gtd_eig_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)need);
    g_gtd_ok = e == hipSuccess;
    if (e != hipSuccess) (void)hipGetLastError();
    return hipSuccess;
}

bool gtd_supported(int nvec_cap, int len_cap) {
    return g_gtd_ok && len_cap >= 1 && len_cap <= GTD_MAX_N && nvec_cap >= 1 && nvec_cap <= GTD_SEL_MAX;
}

size_t gtd_work_doubles(int nvec_cap, int len_cap) {
    const size_t n = (size_t)len_cap;
    return 5 * n * n + n * (size_t)nvec_cap + 64;
}

// H = X^T X, eigensolver, W = V^T X^T, select.  X (nv x n) is d.X; work holds
// gtd_work_doubles(nvec_cap, len_cap) doubles.
hipError_t launch_gtd(const JacobiDesc& d, int nvec_cap, int len_cap, double* work, hipStream_t s) {
    const size_t n = (size_t)len_cap;
    double* H = work;
    double* Vt = H + n * n;
    double* refl = Vt + n * n;
    double* Qa = refl + n * n;
    double* Qb = Qa + n * n;
    double* W = Qb + n * n;
    GemmDesc h{};
    h.A = d.X;
    h.B = d.X;
    h.C = H;
    h.dims = d.dims_in;
    h.M = d.len;
    h.N = d.len;
    h.K = d.nvec;
    h.ta = 1;
    h.alpha = 1.0;
    hipError_t e = launch_gemm(h, len_cap, len_cap, 1, s, P_F64);
    if (e != hipSuccess) return e;
    GtdDesc g{};
    g.H = H;
    g.dims = d.dims_in;
    g.n = d.len;
    g.Vt = Vt;
    g.refl = refl;
    g.Qa = Qa;
    g.Qb = Qb;
    g.status = d.status;
    hipLaunchKernelGGL(gtd_eig_kernel, dim3(1), dim3(GTD_NT), gtd_lds_bytes(len_cap), s, g);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    GemmDesc w{};
    w.A = Vt;
    w.B = d.X;
    w.C = W;
    w.dims = d.dims_in;
    w.M = d.len;
    w.N = d.nvec;
    w.K = d.len;
    w.tb = 1;
    w.alpha = 1.0;
    e = launch_gemm(w, len_cap, nvec_cap, 1, s, P_F64);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gtd_select_kernel, dim3(1), dim3(1024), 0, s, d, W, Vt);
    return hipGetLastError();
}

}  // namespace smps
