// FP64 factorization of the two-site tensor and the truncation step.
//
// The split of Sec. 2.3 needs, for the side the isometry centre leaves, an
// orthonormal basis of the leading singular subspace, the singular values
// (for the truncation rule and the discarded weight) and nothing else: the
// other factor is recomputed as an exact projection by a matrix product.
// One-sided (Hestenes) Jacobi gives exactly that without accumulating a
// rotation matrix: rotating pairs of vectors until all are mutually
// orthogonal leaves W = Q diag(s), so the kept rows of Q are W_j / s_j.
//
// * jacobi_lds_kernel: the whole matrix resides in LDS (up to ~19k doubles on
//   gfx950's 160 KB); one workgroup; a group of 16 lanes (one DPP row) rotates
//   a pair, reducing its dot product with DPP row moves, and the disjoint
//   pairs of a round run concurrently (home/away or round-robin ordering).
// * jacobi_round_kernel (single problem, larger matrices): the rows stay in
//   global memory; one launch per round of the round-robin tournament, one
//   wave per pair; the host reads the rotation flag after each sweep.
// * jacobi_panel_kernel (batched, larger matrices): the vectors are cut into
//   blocks; in each round every workgroup takes one pair of blocks into LDS
//   and gives their union one inner sweep; a fixed sweep budget with per-
//   problem early exit keeps the launch sequence capturable.
// * select / write: norms, descending order, the truncation rule and the
//   discarded weight in FP64 (tail summed from the smallest value up), then
//   the kept rows normalised.

#include <cfloat>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>

#include "common.h"
#include "select.h"

namespace smps {

constexpr int JT = 1024;               // threads per Jacobi workgroup (blocked path, select)
// threads of the LDS-resident kernel for length class 16 E: 1024, except the
// widest class, whose two register-held rows would not fit 128 VGPRs per lane
__host__ __device__ constexpr int lds_threads(int E) { return E >= 16 ? 512 : 1024; }
constexpr int LDS_BYTES = 160 * 1024;  // gfx950 LDS per workgroup
constexpr int JAC_MAX_SWEEPS = 40;
// cold starts of large, strongly graded matrices need many round-robin sweeps
// (two-site tensors with singular values spread over 13 decades take ~40)
constexpr int ROUND_MAX_SWEEPS = 120;
constexpr int SEL_MAX = 2048;          // vectors handled by the select kernel

__device__ __forceinline__ int tourney(int pos, int rd, int n2) {
    // player at position pos in round rd of a round-robin over n2 (even) players
    if (pos == 0) return 0;
    int x = pos - 1 + rd;  // < 2 (n2 - 1)
    if (x >= n2 - 1) x -= n2 - 1;
    return x + 1;
}

// Sum over the 8 lanes of a half row (quad pairs, then the half-row mirror).
__device__ __forceinline__ double row_sum8(double x) {
    x += dpp_mov<0xB1>(x);
    x += dpp_mov<0x4E>(x);
    x += dpp_mov<0x141>(x);
    return x;
}
__device__ __forceinline__ double row_sum4(double x) {
    x += dpp_mov<0xB1>(x);
    x += dpp_mov<0x4E>(x);
    return x;
}
// Sum over a whole wave: the rows' sums, then the other rows' by lane swaps
// (each step again adds equal partners in either order, so every lane ends
// with the identical value).
__device__ __forceinline__ double wave_sum(double x) {
    x = row_sum16(x);
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
}
// Sum over a half wave (two DPP rows): the rows' sums, then the partner row's.
__device__ __forceinline__ double half_wave_sum(double x) {
    x = row_sum16(x);
    x += __shfl_xor(x, 16, 64);
    return x;
}
template <int G>
__device__ __forceinline__ double group_sum(double x) {
    if constexpr (G == 64) return wave_sum(x);
    else if constexpr (G == 32) return half_wave_sum(x);
    else if constexpr (G == 16) return row_sum16(x);
    else if constexpr (G == 8) return row_sum8(x);
    else return row_sum4(x);
}

// Rutishauser's rotation for a pair with squared norms a, b and dot product c:
// t = sgn(z) / (|z| + sqrt(1 + z^2)), z = (b - a) / 2c, written as
// t = sgn(b - a) 2c / (|b - a| + sqrt((b - a)^2 + 4c^2)).  That form is
// homogeneous of degree 0: it is evaluated as it stands when (b - a)^2 + 4c^2
// lies between 2^-900 and 2^900, and otherwise (a rare branch) after scaling
// both terms by an approximate 1 / max(|b - a|, |2c|), so nothing under- or
// overflows; the square root and the quotient use the hardware
// approximations with one Newton step each.  cs = 1 / sqrt(1 + t^2) gets its
// own Newton step so that cs^2 + sn^2 = 1 to rounding: that, not the exact
// angle, keeps the transformation orthogonal.
__device__ __forceinline__ void jacobi_rotation(double a, double b, double c, double& cs, double& sn, double& t) {
    double dn = b - a, cn = c + c;
    double hh = fma(dn, dn, cn * cn);
    if (!(hh > 0x1p-900 && hh < 0x1p900)) {
        asm volatile("");  // keeps the rare branch a branch (not evaluated on every pair)
        const double r = __builtin_amdgcn_rcp(fmax(fabs(dn), fabs(cn)));
        dn *= r;
        cn *= r;
        hh = fma(dn, dn, cn * cn);
    }
    double rs = __builtin_amdgcn_rsq(hh);
    rs = rs * fma(-0.5 * hh * rs, rs, 1.5);
    const double den = fma(hh, rs, fabs(dn));
    double rc = __builtin_amdgcn_rcp(den);
    rc = rc * fma(-den, rc, 2.0);
    t = (dn >= 0.0 ? cn : -cn) * rc;
    const double h = fma(t, t, 1.0);
    cs = __builtin_amdgcn_rsq(h);
    cs = cs * fma(-0.5 * h * cs, cs, 1.5);
    sn = cs * t;
}

// |c| > tol sqrt(a b), compared squared: c^2 > (tol a)(tol b), three products
// instead of two square roots (a, b are positive; c^2 overflowing to inf still
// answers correctly, and tol <= 2^-52 * 2048 keeps tol a finite).
__device__ __forceinline__ bool jacobi_needs_rotation(double a, double b, double c, double tol) {
    return c * c > (tol * a) * (tol * b);
}

// Copy nrows rows of len doubles from global memory (row j starts at
// row_src(j)) into LDS rows of stride ld >= len, zero padded.  Each thread
// issues LOADS independent loads before it stores any of them: the LDS stores
// could alias a generic pointer's loads, so a plain copy loop would wait for
// every load in turn.  Returns nonzero if a loaded value is not finite.
template <int LOADS = 8, typename RowSrc>
__device__ __forceinline__ int load_rows_to_lds(double* W, int nrows, int len, int ld, RowSrc row_src, int tid,
                                                int nt) {
    const int total = nrows * ld;
    int bad = 0;
    for (int base = 0; base < total; base += LOADS * nt) {
        double v[LOADS];
#pragma unroll
        for (int u = 0; u < LOADS; ++u) {
            const int e = base + u * nt + tid;
            v[u] = 0.0;
            if (e < total) {
                const int j = e / ld, i = e - j * ld;
                if (i < len) v[u] = row_src(j)[i];
            }
        }
#pragma unroll
        for (int u = 0; u < LOADS; ++u) {
            const int e = base + u * nt + tid;
            if (e < total) {
                bad |= !isfinite(v[u]);
                W[e] = v[u];
            }
        }
    }
    return bad;
}

__device__ __forceinline__ int pow2_ceil(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Orthogonalise nv vectors (row j at W + j*ld, length len) held in LDS; nrm
// (nv doubles of LDS) holds their squared norms, recomputed exactly at the
// start of every sweep and updated in between by the exact 2x2 relations
// (a' = a - t c, b' = b + t c), so a pair needs one dot product only.
// A group of G lanes (G = 4, 8 or 16 inside one DPP row, two rows, or a whole wave) handles a pair;
// the pairs of a round are disjoint and run concurrently.  E > 0: each lane
// keeps its E elements of both vectors in registers between the dot product
// and the rotation (rows zero padded to ld = G E); E = 0: generic strided loop.
//
// Pair orderings (every pair once per sweep):
// * home/away (E > 0, P = pairs padded to a power of two, all P groups
//   resident): stage h = P, P/2, ..., 1 cuts the rows into sets of 2h; in a
//   set, group i keeps row i of the lower half in registers for the whole
//   stage and meets row (i + r) mod h of the upper half in round r.  Only the
//   visiting row goes through LDS, half the traffic of moving both rows.
// * round-robin tournament (otherwise).
// Returns (block-uniform) the number of sweeps that applied a rotation.
// Jw (nullable): an nv x nj matrix (row stride nj) receiving every rotation
// applied to the vectors, so that it accumulates the product of the rotations.
__device__ __forceinline__ void rotate_acc(double* Jw, int nj, int p, int q, int gl, int G, double cs, double sn) {
    double* jp = Jw + (size_t)p * nj;
    double* jq = Jw + (size_t)q * nj;
    for (int i = gl; i < nj; i += G) {
        const double a = jp[i], b = jq[i];
        jp[i] = cs * a - sn * b;
        jq[i] = sn * a + cs * b;
    }
}

template <int E, int G = 16, bool ACC = false>
__device__ int jacobi_orth_t(double* W, int nv, int len, int ld, double* nrm, int* s_flag, double floor2,
                             int true_len, int max_sweeps = JAC_MAX_SWEEPS, double* Jw = nullptr, int nj = 0) {
    static_assert(G == 4 || G == 8 || G == 16 || G == 32 || G == 64, "group width");
    static_assert(E > 0 || G == 16, "generic path uses 16-lane groups");
    const int tid = threadIdx.x;
    if (nv < 2) return 0;
    // cosine threshold: rounding in a length-n dot product is ~eps*sqrt(n); eps*n leaves margin
    const double tol = DBL_EPSILON * (double)(true_len > 16 ? true_len : 16);
    const double tiny = fmax(DBL_MIN * 1.0e4, floor2);
    const int P = (nv + 1) / 2, n2 = 2 * P;
    const int nt = blockDim.x;
    const int gl = tid & (G - 1), gi = tid / G, ngroups = nt / G;
    const int P2 = pow2_ceil(P);
    const bool home_away = E > 0 && P2 <= ngroups && 4 * P2 <= 5 * P;
    int any = 0;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        {
            constexpr int g = 16;
            const int hl = tid & (g - 1), hi = tid / g;
            for (int j = hi; j < nv; j += nt / g) {
                const double* w = W + j * ld;
                double a0 = 0.0, a1 = 0.0;
                int i = hl;
                for (; i + g < len; i += 2 * g) {
                    a0 = fma(w[i], w[i], a0);
                    a1 = fma(w[i + g], w[i + g], a1);
                }
                if (i < len) a0 = fma(w[i], w[i], a0);
                const double a = row_sum16(a0 + a1);
                if (hl == 0) nrm[j] = a;
            }
        }
        if (tid == 0) *s_flag = 0;
        __syncthreads();
        if constexpr (E > 0) {
            if (home_away) {
                for (int h = P2; h >= 1; h >>= 1) {
                    const int set = gi / h, i = gi - set * h;
                    const int home = set * 2 * h + i;
                    const bool act = gi < P2 && home < nv;
                    double x[E];
                    double a = 0.0;
                    if (act) {
#pragma unroll
                        for (int e = 0; e < E; ++e) x[e] = W[home * ld + gl + G * e];
                        a = nrm[home];
                    }
                    for (int r = 0; r < h; ++r) {
                        const int q = set * 2 * h + h + ((i + r) & (h - 1));
                        if (act && q < nv) {
                            const double b = nrm[q];
                            if (a > tiny && b > tiny) {  // uniform in the group
                                double* wq = W + q * ld;
                                double y[E];
                                double cc[2] = {0.0, 0.0};
#pragma unroll
                                for (int e = 0; e < E; ++e) y[e] = wq[gl + G * e];
#pragma unroll
                                for (int e = 0; e < E; ++e) cc[e & 1] = fma(x[e], y[e], cc[e & 1]);
                                const double c = group_sum<G>(cc[0] + cc[1]);
                                if (jacobi_needs_rotation(a, b, c, tol)) {
                                    double cs, sn, t;
                                    jacobi_rotation(a, b, c, cs, sn, t);
#pragma unroll
                                    for (int e = 0; e < E; ++e) {
                                        const double xe = x[e];
                                        x[e] = cs * xe - sn * y[e];
                                        wq[gl + G * e] = sn * xe + cs * y[e];
                                    }
                                    if constexpr (ACC) rotate_acc(Jw, nj, home, q, gl, G, cs, sn);
                                    a = fmax(a - t * c, 0.0);
                                    if (gl == 0) {
                                        nrm[q] = b + t * c;
                                        *s_flag = 1;
                                    }
                                }
                            }
                        }
                        __syncthreads();
                    }
                    if (act) {
#pragma unroll
                        for (int e = 0; e < E; ++e) W[home * ld + gl + G * e] = x[e];
                        if (gl == 0) nrm[home] = a;
                    }
                    __syncthreads();
                }
                const int rot = *s_flag;
                __syncthreads();
                if (!rot) break;
                ++any;
                continue;
            }
        }
        for (int rd = 0; rd < n2 - 1; ++rd) {
            for (int pi = gi; pi < P; pi += ngroups) {
                const int p = tourney(pi, rd, n2), q = tourney(n2 - 1 - pi, rd, n2);
                if (p >= nv || q >= nv) continue;
                const double a = nrm[p], b = nrm[q];
                if (!(a > tiny && b > tiny)) continue;  // uniform in the group
                double* wp = W + p * ld;
                double* wq = W + q * ld;
                double x[E > 0 ? E : 1], y[E > 0 ? E : 1];
                double c;
                if constexpr (E > 0) {
                    double cc[2] = {0.0, 0.0};
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int i = gl + G * e;  // len == G E here (zero padded)
                        x[e] = wp[i];
                        y[e] = wq[i];
                    }
#pragma unroll
                    for (int e = 0; e < E; ++e) cc[e & 1] = fma(x[e], y[e], cc[e & 1]);
                    c = group_sum<G>(cc[0] + cc[1]);
                } else {
                    double c0 = 0.0, c1 = 0.0;
                    int i = gl;
                    for (; i + G < len; i += 2 * G) {
                        c0 = fma(wp[i], wq[i], c0);
                        c1 = fma(wp[i + G], wq[i + G], c1);
                    }
                    if (i < len) c0 = fma(wp[i], wq[i], c0);
                    c = group_sum<G>(c0 + c1);
                }
                if (jacobi_needs_rotation(a, b, c, tol)) {
                    double cs, sn, t;
                    jacobi_rotation(a, b, c, cs, sn, t);
                    if constexpr (E > 0) {
#pragma unroll
                        for (int e = 0; e < E; ++e) {
                            const int i = gl + G * e;
                            wp[i] = cs * x[e] - sn * y[e];
                            wq[i] = sn * x[e] + cs * y[e];
                        }
                    } else {
                        for (int i = gl; i < len; i += G) {
                            const double xv = wp[i], yv = wq[i];
                            wp[i] = cs * xv - sn * yv;
                            wq[i] = sn * xv + cs * yv;
                        }
                    }
                    if constexpr (ACC) rotate_acc(Jw, nj, p, q, gl, G, cs, sn);
                    if (gl == 0) {
                        nrm[p] = fmax(a - t * c, 0.0);
                        nrm[q] = b + t * c;
                        *s_flag = 1;
                    }
                }
            }
            __syncthreads();
        }
        const int rot = *s_flag;
        __syncthreads();
        if (!rot) break;
        ++any;
    }
    return any;
}

// register-held elements per lane for a vector length cap (0: strided loop)
static int elems_for(int len_cap) {
    if (len_cap <= 16) return 1;
    if (len_cap <= 32) return 2;
    if (len_cap <= 64) return 4;
    if (len_cap <= 128) return 8;
    if (len_cap <= 256) return 16;
    return 0;
}

// ---- completion of a rank-deficient warm-start basis -----------------------
// The basis handed to the next visit of a bond must be a complete orthogonal
// matrix (it pre-rotates that visit's vectors).  When the split's vectors do
// not span the whole space (numerically rank-deficient two-site tensors, or
// fewer vectors than their length), the normalised vectors of the nonzero
// values fill rows 0..m-1 and rows m..len-1 are completed here: pivoted
// Gram-Schmidt on the unit vectors, each step taking the unit vector with the
// largest squared component p_j outside the current span (at least
// (len - k)/len at step k, since the p_j sum to len - k), with a second pass
// whenever the first leaves less than half of it.  B is len x len in global
// memory, read and written by this workgroup only.

__device__ double block_sum(double x, double* redv) {
    x = wave_sum(x);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) redv[w] = x;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += redv[i];
    __syncthreads();
    return t;
}

__device__ int block_argmax(const double* p, int n, double* redv, int* redi) {
    double best = -2.0;
    int bi = 0;
    for (int j = threadIdx.x; j < n; j += blockDim.x)
        if (p[j] > best) {
            best = p[j];
            bi = j;
        }
    for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) {
        redv[w] = best;
        redi[w] = bi;
    }
    __syncthreads();
    double b = redv[0];
    int r = redi[0];
    for (int i = 1; i < nw; ++i)
        if (redv[i] > b || (redv[i] == b && redi[i] < r)) {
            b = redv[i];
            r = redi[i];
        }
    __syncthreads();
    return r;
}

// A basis is completed when the split has at least as many vectors as their
// length (it would be complete at full rank: rank-deficient two-site tensors)
// and the rows have at least COMPLETE_MIN_LEN elements; otherwise it stays the
// identity.  Below that length the completion (a few barriers per vector)
// costs more than the cold sweeps it saves (measured on the 512-chain batch:
// 64-element rows 100 -> 600 us per split, 256-element rows 7.8 -> 3.7 ms);
// with fewer vectors than their length the bond's next visit takes its warm
// start from accumulated rotations instead (n=20 chi=64: 8 ms per apply spent
// on completions nobody read).
constexpr int COMPLETE_MIN_LEN = 128;
__device__ __forceinline__ bool completes_basis(int nv, int len) { return nv >= len && len >= COMPLETE_MIN_LEN; }

// LDS doubles complete_basis needs: p, coefficients, reductions and the
// sliced partial sums (at most one per thread of a 1024-thread workgroup).
__host__ __device__ constexpr size_t complete_lds_doubles(int len) {
    return (size_t)len * 2 + 64 + 1024;
}

// r[l] = base[l] - sum_{i<k} coef[i] B[i][l] for all l, the k-sum split over
// the threads beyond len (slices of i, combined through LDS in slice order, so
// the result does not depend on timing); returns this thread's part of |r|^2.
__device__ double project_out(const double* B, int len, int k, const double* coef, double* r, int piv,
                              bool from_unit, double* part) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int ns = nt >= 2 * len ? min(nt / len, 16) : 1;  // slices of the i range
    const int sl = tid / len, l0 = tid - sl * len;
    double acc = 0.0;
    if (ns > 1) {
        if (sl < ns) {
            const int i0 = (int)((long long)k * sl / ns), i1 = (int)((long long)k * (sl + 1) / ns);
            for (int i = i0; i < i1; ++i) acc = fma(coef[i], B[(size_t)i * len + l0], acc);
            part[sl * len + l0] = acc;
        }
        __syncthreads();
        double nrm = 0.0;
        if (tid < len) {
            double a = 0.0;
            for (int x = 0; x < ns; ++x) a += part[x * len + tid];
            const double v = (from_unit ? (tid == piv ? 1.0 : 0.0) : r[tid]) - a;
            r[tid] = v;
            nrm = v * v;
        }
        __syncthreads();
        return nrm;
    }
    double nrm = 0.0;
    for (int l = tid; l < len; l += nt) {
        double v = from_unit ? (l == piv ? 1.0 : 0.0) : r[l];
        for (int i = 0; i < k; ++i) v = fma(-coef[i], B[(size_t)i * len + l], v);
        r[l] = v;
        nrm = fma(v, v, nrm);
    }
    return nrm;
}

__device__ void complete_basis(double* B, int len, int m, double* scratch) {
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, w = tid >> 6, nw = (nt + 63) >> 6;
    double* p = scratch;          // len
    double* coef = p + len;       // len
    double* redv = coef + len;    // 32
    int* redi = (int*)(redv + 32);
    double* part = redv + 64;     // slices x len <= blockDim.x doubles
    for (int j = tid; j < len; j += nt) {
        double a = 0.0;
        for (int i = 0; i < m; ++i) {
            const double b = B[(size_t)i * len + j];
            a = fma(b, b, a);
        }
        p[j] = 1.0 - a;
    }
    __syncthreads();
    for (int k = m; k < len; ++k) {
        const int piv = block_argmax(p, len, redv, redi);
        const double pk = p[piv];
        for (int i = tid; i < k; i += nt) coef[i] = B[(size_t)i * len + piv];
        __syncthreads();
        double* r = B + (size_t)k * len;
        double n2 = block_sum(project_out(B, len, k, coef, r, piv, true, part), redv);
        __threadfence_block();
        if (n2 < 0.5 * pk) {
            // second pass: coefficients against the same rows
            for (int i = w; i < k; i += nw) {
                double a = 0.0;
                for (int l = lane; l < len; l += 64) a = fma(B[(size_t)i * len + l], r[l], a);
                a = wave_sum(a);
                if (lane == 0) coef[i] = a;
            }
            __syncthreads();
            n2 = block_sum(project_out(B, len, k, coef, r, piv, false, part), redv);
            __threadfence_block();
        }
        const double inv = 1.0 / sqrt(n2);
        for (int l = tid; l < len; l += nt) {
            const double v = r[l] * inv;
            r[l] = v;
            p[l] -= v * v;
        }
        __threadfence_block();
        __syncthreads();
        if (tid == 0) p[piv] = -1.0;
        __syncthreads();
    }
}

// Kept rows: Q[i] = W[perm[i]] / s_i (a zero vector only occurs when the
// whole matrix is zero and one row is kept: it becomes the first unit vector).
__device__ void jacobi_write_rows(const double* W, int nv, int len, int ld, const double* sig_sorted,
                                  const int* perm, int r, double* Q, double* basis, int gram,
                                  const double* Jw = nullptr) {
    if (Jw) {
        // accumulated rotations: row perm[i] of J is the nvec-side singular
        // vector of the i-th value (orthonormal also for zero values)
        for (size_t e = threadIdx.x; e < (size_t)r * nv; e += blockDim.x) {
            const int i = (int)(e / nv), l = (int)(e % nv);
            Q[e] = Jw[(size_t)perm[i] * nv + l];
        }
        if (basis)
            for (size_t e = threadIdx.x; e < (size_t)nv * nv; e += blockDim.x) basis[e] = Jw[e];
        return;
    }
    for (size_t e = threadIdx.x; e < (size_t)r * len; e += blockDim.x) {
        const int i = (int)(e / len), l = (int)(e % len);
        const double s = gram ? sig_sorted[i] * sig_sorted[i] : sig_sorted[i];
        Q[e] = s > 0.0 ? W[(size_t)perm[i] * ld + l] / s : (l == i ? 1.0 : 0.0);
    }
    if (!basis) return;
    // len x len basis for the next visit of this bond: the normalised vectors
    // of the nonzero values (rows of zero values are completed afterwards by
    // complete_basis)
    const int nz = nv < len ? nv : len;
    for (size_t e = threadIdx.x; e < (size_t)len * len; e += blockDim.x) {
        const int i = (int)(e / len), l = (int)(e % len);
        const bool live = i < nz && sig_sorted[i] > 0.0;
        basis[e] = live ? W[(size_t)perm[i] * ld + l] / sig_sorted[i] : 0.0;
    }
}

// Rows of the basis that jacobi_write_rows filled (the nonzero values among
// the first min(nv, len) sorted ones).
__device__ int basis_rows(const double* sig_sorted, int nv, int len) {
    const int nz = nv < len ? nv : len;
    int m = 0;
    while (m < nz && sig_sorted[m] > 0.0) ++m;
    return m;
}

template <int E, bool ACC>
__global__ __launch_bounds__(lds_threads(E)) void jacobi_lds_kernel(JacobiDesc d0, const JacobiDesc* arr) {
    const int LDS_NT = blockDim.x;  // at most lds_threads(E); fewer for few vectors
    extern __shared__ double sm[];
    const JacobiDesc d = arr ? arr[blockIdx.x] : d0;  // batched: one factorization per workgroup
    __shared__ int s_flag, s_bad;
    __shared__ double s_delta;
    const int nv = eval_dim(d.dims_in, d.nvec), len = eval_dim(d.dims_in, d.len);
    // rows padded with zeros to 16 E so the register path needs no bounds tests
    const int ld = E > 0 ? 16 * E : len;
    const int tid = threadIdx.x;
    double* W = sm;
    double* Jw = ACC ? sm + (size_t)nv * ld : nullptr;  // nv x nv, starts as the identity
    double* sig_raw = sm + (size_t)nv * ld + (ACC ? (size_t)nv * nv : 0);
    double* sig_sorted = sig_raw + nv;
    int* perm = (int*)(sig_sorted + nv);
    if (tid == 0) s_bad = 0;
    // warm start of an accumulated factorization: X = J0 (raw vectors), J = J0
    // (X == X_raw: the vectors were not pre-rotated, so J starts from the identity)
    const bool warm = ACC && d.acc_tag && d.X != d.X_raw && *d.acc_tag == 2 * nv + d.acc_dir + 1;
    if (Jw)
        for (int e = tid; e < nv * nv; e += LDS_NT) Jw[e] = warm ? d.acc_basis[e] : (e / nv == e % nv) ? 1.0 : 0.0;
    __syncthreads();
    const double* X = (ACC && d.acc_tag && !warm) ? d.X_raw : d.X;
    const int bad = load_rows_to_lds(W, nv, len, ld, [=](int j) { return X + (size_t)j * len; }, tid, LDS_NT);
    if (bad) s_bad = 1;
    __syncthreads();
    if (s_bad) {
        for (int e = tid; e < nv * ld; e += LDS_NT) W[e] = 0.0;
        if (tid == 0 && d.status) *d.status = 1;
        __syncthreads();
    }
    // ||X||_F^2 (summed in vector order, deterministic) for the rank floor
    __shared__ double s_total2;
    {
        const int gl = tid & 15, gi = tid >> 4;
        for (int j = gi; j < nv; j += LDS_NT / 16) {
            double a = 0.0;
            for (int i = gl; i < len; i += 16) a = fma(W[j * ld + i], W[j * ld + i], a);
            a = row_sum16(a);
            if (gl == 0) sig_raw[j] = a;
        }
        __syncthreads();
        if (tid == 0) {
            double t2 = 0.0;
            for (int j = 0; j < nv; ++j) t2 += sig_raw[j];
            s_total2 = t2;
        }
        __syncthreads();
    }
    const int nsw = jacobi_orth_t<E, 16, ACC>(W, nv, E > 0 ? ld : len, ld, sig_raw, &s_flag,
                                           zero_floor2(s_total2, nv, len, d.floor_eps), len, JAC_MAX_SWEEPS, Jw,
                                           nv);
    if (tid == 0 && d.log_sweeps) *d.log_sweeps = nsw;
    // still rotating when the sweep budget ran out: reported like the blocked paths
    if (tid == 0 && d.status && jacobi_unconverged(nsw, JAC_MAX_SWEEPS)) atomicOr(d.status, 2);
    const int r = jacobi_select(W, nv, len, ld, sig_raw, sig_sorted, perm, d, &s_delta);
    jacobi_write_rows(W, nv, len, ld, sig_sorted, perm, r, d.Q, d.basis, d.gram, Jw);
    if (ACC && d.acc_tag) {
        for (int e = tid; e < nv * nv; e += LDS_NT) d.acc_basis[e] = Jw[e];
        if (tid == 0) *d.acc_tag = 2 * nv + d.acc_dir + 1;
    }
    if (!ACC && d.basis) {
        // complete a rank-deficient basis; W is free now and holds the scratch
        const int m = basis_rows(sig_sorted, nv, len);
        __threadfence_block();
        __syncthreads();
        if (m < len && completes_basis(nv, len) && (size_t)nv * ld >= complete_lds_doubles(len))
            complete_basis(d.basis, len, m, W);
        else if (m < len)
            for (int e = tid; e < len * len; e += LDS_NT) d.basis[e] = (e / len == e % len) ? 1.0 : 0.0;
    }
}

// Threads of a blocked-path workgroup: G = 16 as the LDS kernel of class E;
// wider groups (rows of 257..1024 elements) one group per pair of a 32-row
// block pair (16 pairs) or of a 16-row one (8 pairs).
__host__ __device__ constexpr int panel_threads(int E, int G) {
    return G == 64 ? 1024 : G == 32 ? 512 : lds_threads(E);
}

// One block pair of round rd of the blocked path: position `pos` of the
// tournament over blocks, the union orthogonalised in LDS (one inner sweep)
// and written back when it rotated.  Rows are zero padded to G E elements
// (E > 0), E held per lane by groups of G lanes; E = 0 is the strided generic
// loop.  Returns 1 when a rotation was applied, 0 otherwise, -1 on
// non-finite input (status bit 1 set).  Uniform over the workgroup.
template <int E, int G>
__device__ int panel_pair_round(const JacobiDesc& d, int rd, int pos, double* sm, int* s_flag, int* s_bad,
                                double* s_nrm) {
    constexpr int NT = panel_threads(E, G);
    const int bs = d.bs, nblk2 = d.nblk;
    if (rd >= nblk2 - 1 || pos >= nblk2 / 2) return 0;
    const int nv = eval_dim(d.dims_in, d.nvec), len = eval_dim(d.dims_in, d.len);
    // rows zero padded to G E in LDS for the register path (E > 0)
    const int ld = E > 0 ? G * E : len;
    const int bp = tourney(pos, rd, nblk2), bq = tourney(nblk2 - 1 - pos, rd, nblk2);
    // vectors of the two blocks that exist
    int idx[2], cnt[2];
    idx[0] = bp * bs;
    idx[1] = bq * bs;
    cnt[0] = min(bs, max(0, nv - idx[0]));
    cnt[1] = min(bs, max(0, nv - idx[1]));
    const int nloc = cnt[0] + cnt[1];
    if (nloc < 2) return 0;
    const int tid = threadIdx.x;
    if (tid == 0) *s_bad = 0;
    __syncthreads();
    const double* X = d.X;
    const int i0 = idx[0], i1 = idx[1], c0 = cnt[0];
    const int bad = load_rows_to_lds(
        sm, nloc, len, ld, [=](int j) { return X + (size_t)(j < c0 ? i0 + j : i1 + (j - c0)) * len; }, tid, NT);
    if (bad) *s_bad = 1;
    __syncthreads();
    if (*s_bad) {
        if (tid == 0 && d.status) atomicOr(d.status, 1);
        return -1;
    }
    // one inner sweep per round: the outer tournament then acts as one cyclic ordering
    const bool any = jacobi_orth_t<E, G>(sm, nloc, E > 0 ? ld : len, ld, s_nrm, s_flag,
                                         zero_floor2(*d.fro2, nv, len, d.floor_eps), len, 1) > 0;
    if (!any) return 0;
    for (int e = tid; e < nloc * ld; e += NT) {
        const int j = e / ld, l = e - j * ld;
        if (l >= len) continue;
        const int gj = j < c0 ? i0 + j : i1 + (j - c0);
        d.X[(size_t)gj * len + l] = sm[e];
    }
    return 1;
}

// One round of the single-problem blocked path: workgroup i takes the block
// pair of tournament position i.
template <int E, int G = 16>
__global__ __launch_bounds__(panel_threads(E, G)) void jacobi_panel_kernel(JacobiDesc d, int rd) {
    extern __shared__ double sm[];
    __shared__ int s_flag, s_bad;
    __shared__ double s_nrm[64];
    if (panel_pair_round<E, G>(d, rd, (int)blockIdx.x, sm, &s_flag, &s_bad, s_nrm) > 0 && threadIdx.x == 0 &&
        d.conv)
        atomicOr(d.conv, 1);
}

// ---- persistent batched blocked path ----------------------------------------
// One launch runs every sweep of every factorization of a batched step.
// Workgroups form teams of P (the largest block-pair count of the launch);
// a team takes factorizations from a device queue (the descriptor array,
// ordered longest first on the host) and runs the tournament over blocks,
// member m taking the pair of position m in every round, with a team barrier
// between rounds, until a sweep rotates nothing (or the sweep budget runs
// out, status bit 2).  The grid is at most one workgroup per compute unit,
// so every team is resident; every wait is bounded all the same (status bit
// 4 and the team stops when a barrier times out).

__device__ __forceinline__ int ld_agent(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr long long PANEL_SPIN_LIMIT = 1LL << 22;

// Team barrier number `phase` (1, 2, ... in every member).  Every wave first
// waits for its own memory operations (so this workgroup's stores have
// reached its L2 and no load is left in flight); one thread then counts the
// arrival with a release at agent scope (the L2 write-back that makes the
// stores visible to the other XCDs), waits for phase * P arrivals and
// acquires at agent scope (invalidating the caches the whole workgroup
// reads through).  Returns false when the team has given up (a wait ran out).
__device__ bool team_barrier(PanelTeamState* T, int P, int phase, int* s_ok) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __hip_atomic_fetch_add(&T->bar, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const int target = phase * P;
        long long spins = 0;
        while (ld_agent(&T->bar) < target) {
            if (ld_agent(&T->abort) || ++spins > PANEL_SPIN_LIMIT) {
                st_agent(&T->abort, 1);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_ok = ok && !ld_agent(&T->abort);
    }
    __syncthreads();
    return *s_ok != 0;
}

template <int E, int G = 16>
__global__ __launch_bounds__(panel_threads(E, G)) void jacobi_panel_persistent_kernel(JacobiDesc d0,
                                                                                     const JacobiDesc* arr,
                                                                                     int count, int P,
                                                                                     PanelQueueState* q,
                                                                                     int max_sweeps) {
    extern __shared__ double sm[];
    __shared__ int s_flag, s_bad, s_ok, s_prob, s_rot;
    __shared__ double s_nrm[64];
    // team and member of this workgroup: with a team count divisible by 8 the
    // members of a team share blockIdx mod 8, i.e. one XCD and its L2
    const int b = (int)blockIdx.x, nteam = (int)gridDim.x / P;
    int team, member;
    if (nteam % 8 == 0) {
        team = (b % 8) + 8 * ((b / 8) / P);
        member = (b / 8) % P;
    } else {
        team = b / P;
        member = b % P;
    }
    PanelTeamState* T = &q->team[team];
    const int tid = threadIdx.x;
    int phase = 0;
    for (;;) {
        // the leader takes the next factorization and clears the flags
        int taken = -1;
        if (member == 0 && tid == 0) {
            const int p = __hip_atomic_fetch_add(&q->head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            taken = p < count ? p : -1;
            st_agent(&T->prob, taken);
            for (int k = 0; k < 3; ++k) st_agent(&T->rot[k], 0);
        }
        if (!team_barrier(T, P, ++phase, &s_ok)) {
            int* st = taken < 0 ? nullptr : arr ? arr[taken].status : d0.status;
            if (st) atomicOr(st, 4);
            return;
        }
        if (tid == 0) s_prob = ld_agent(&T->prob);
        __syncthreads();
        const int pi = s_prob;
        if (pi < 0) return;
        const JacobiDesc d = arr ? arr[pi] : d0;
        const int rounds = d.nblk - 1;
        int sw = 0;
        bool converged = false, alive = true;
        for (; sw < max_sweeps && alive; ++sw) {
            // slot (sw + 1) mod 3 was last read two sweeps ago: free for the next sweep
            if (member == 0 && tid == 0) st_agent(&T->rot[(sw + 1) % 3], 0);
            for (int rd = 0; rd < rounds && alive; ++rd) {
                const int r = panel_pair_round<E, G>(d, rd, member, sm, &s_flag, &s_bad, s_nrm);
                if (r > 0 && tid == 0)
                    __hip_atomic_fetch_or(&T->rot[sw % 3], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                alive = team_barrier(T, P, ++phase, &s_ok);
            }
            if (!alive) break;
            if (tid == 0) s_rot = ld_agent(&T->rot[sw % 3]);
            __syncthreads();
            if (!s_rot) {
                converged = true;
                break;
            }
        }
        if (member == 0 && tid == 0) {
            if (!alive && d.status) atomicOr(d.status, 4);
            else if (!converged && d.status) atomicOr(d.status, 2);
            if (d.log_sweeps) *d.log_sweeps = sw;  // sweeps that rotated
        }
        if (!alive) return;
        // every member has read this factorization's flags before the leader moves on
        if (!team_barrier(T, P, ++phase, &s_ok)) return;
    }
}


// One round of the global-memory path for matrices too large for LDS: wave w
// of workgroup b takes pair 4 b + w of round rd of the round-robin tournament,
// reads both rows (EW elements per lane, len <= 64 EW), forms the three dot
// products, rotates and writes the rows back.  A launch per round is the
// only synchronisation; the host reads the rotation flag after each sweep.
template <int EW>
__global__ __launch_bounds__(256) void jacobi_round_kernel(JacobiDesc d, int rd) {
    const int nv = eval_dim(d.dims_in, d.nvec), len = eval_dim(d.dims_in, d.len);
    const int P = (nv + 1) / 2, n2 = 2 * P;
    const int lane = threadIdx.x & 63;
    const int pi = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pi >= P || rd >= n2 - 1) return;  // wave-uniform
    const int p = tourney(pi, rd, n2), q = tourney(n2 - 1 - pi, rd, n2);
    if (p >= nv || q >= nv) return;
    double* wp = d.X + (size_t)p * len;
    double* wq = d.X + (size_t)q * len;
    double x[EW], y[EW];
    double a0 = 0.0, b0 = 0.0, c0 = 0.0;
#pragma unroll
    for (int e = 0; e < EW; ++e) {
        const int i = lane + 64 * e;
        x[e] = i < len ? wp[i] : 0.0;
        y[e] = i < len ? wq[i] : 0.0;
        a0 = fma(x[e], x[e], a0);
        b0 = fma(y[e], y[e], b0);
        c0 = fma(x[e], y[e], c0);
    }
    a0 = row_sum16(a0);
    b0 = row_sum16(b0);
    c0 = row_sum16(c0);
    a0 += __shfl_xor(a0, 16, 64);
    b0 += __shfl_xor(b0, 16, 64);
    c0 += __shfl_xor(c0, 16, 64);
    a0 += __shfl_xor(a0, 32, 64);
    b0 += __shfl_xor(b0, 32, 64);
    c0 += __shfl_xor(c0, 32, 64);
    if (!isfinite(a0) || !isfinite(b0)) {
        if (lane == 0 && d.status) atomicOr(d.status, 1);
        return;
    }
    const double tiny = fmax(DBL_MIN * 1.0e4, zero_floor2(*d.fro2, nv, len, d.floor_eps));
    if (!(a0 > tiny && b0 > tiny)) return;
    const double tol = DBL_EPSILON * (double)(len > 16 ? len : 16);
    if (!jacobi_needs_rotation(a0, b0, c0, tol)) return;
    double cs, sn, t;
    jacobi_rotation(a0, b0, c0, cs, sn, t);
#pragma unroll
    for (int e = 0; e < EW; ++e) {
        const int i = lane + 64 * e;
        if (i < len) {
            wp[i] = cs * x[e] - sn * y[e];
            wq[i] = sn * x[e] + cs * y[e];
        }
    }
    if (lane == 0) atomicOr(d.conv, 1);
}

__global__ void or_int_kernel(int* p, int v) { atomicOr(p, v); }

// Blocked path finish: select on the vectors in global memory.
__global__ __launch_bounds__(JT) void jacobi_select_kernel(JacobiDesc d0, const JacobiDesc* arr) {
    const JacobiDesc d = arr ? arr[blockIdx.x] : d0;
    __shared__ double sig_raw[SEL_MAX];
    __shared__ double sig_sorted[SEL_MAX];
    __shared__ int perm_s[SEL_MAX];
    __shared__ double s_delta;
    const int nv = eval_dim(d.dims_in, d.nvec), len = eval_dim(d.dims_in, d.len);
    jacobi_select(d.X, nv, len, len, sig_raw, sig_sorted, perm_s, d, &s_delta);
    for (int j = threadIdx.x; j < nv; j += JT) d.perm[j] = perm_s[j];
}

__global__ __launch_bounds__(256) void jacobi_write_kernel(JacobiDesc d0, const JacobiDesc* arr) {
    const JacobiDesc d = arr ? arr[blockIdx.z] : d0;
    const int nv = eval_dim(d.dims_in, d.nvec), len = eval_dim(d.dims_in, d.len);
    const int r = d.dims_out[d.rank_idx];
    const int i = blockIdx.y;
    if (i < r) {
        const double s = d.gram ? d.sigma[i] * d.sigma[i] : d.sigma[i];
        const double* w = d.X + (size_t)d.perm[i] * len;
        for (int l = blockIdx.x * 256 + threadIdx.x; l < len; l += gridDim.x * 256)
            d.Q[(size_t)i * len + l] = s > 0.0 ? w[l] / s : (l == i ? 1.0 : 0.0);
    }
    if (d.basis && i < len) {
        // normalised vectors of the nonzero values; jacobi_complete_kernel fills the rest
        const bool live = i < nv && d.sigma[i] > 0.0;
        const double s = live ? d.sigma[i] : 1.0;
        const double* w = d.X + (size_t)(live ? d.perm[i] : 0) * len;
        for (int l = blockIdx.x * 256 + threadIdx.x; l < len; l += gridDim.x * 256)
            d.basis[(size_t)i * len + l] = live ? w[l] / s : 0.0;
    }
}

// Completion of the blocked paths' warm-start basis (one workgroup per
// factorization; dynamic LDS: complete_lds_doubles(len) doubles).
__global__ __launch_bounds__(1024) void jacobi_complete_kernel(JacobiDesc d0, const JacobiDesc* arr) {
    extern __shared__ double sm[];
    const JacobiDesc d = arr ? arr[blockIdx.x] : d0;
    if (!d.basis) return;
    const int nv = eval_dim(d.dims_in, d.nvec), len = eval_dim(d.dims_in, d.len);
    const int m = basis_rows(d.sigma, nv, len);
    if (m >= len) return;
    if (completes_basis(nv, len)) {
        complete_basis(d.basis, len, m, sm);
        return;
    }
    for (int e = threadIdx.x; e < len * len; e += blockDim.x) d.basis[e] = (e / len == e % len) ? 1.0 : 0.0;
}

__global__ void zero_int_kernel(int* p) { *p = 0; }
__global__ void set_int_kernel(int* p, int v) { *p = v; }

// ||X||_F^2 for the blocked path's rank floor: per-vector sums in vector order.
__global__ __launch_bounds__(JT) void fro2_kernel(JacobiDesc d0, const JacobiDesc* arr) {
    const JacobiDesc d = arr ? arr[blockIdx.x] : d0;
    __shared__ double part[SEL_MAX];
    const int nv = eval_dim(d.dims_in, d.nvec), len = eval_dim(d.dims_in, d.len);
    const int tid = threadIdx.x, gl = tid & 15, gi = tid >> 4;
    for (int j = gi; j < nv; j += JT / 16) {
        const double* w = d.X + (size_t)j * len;
        double a = 0.0;
        for (int i = gl; i < len; i += 16) a = fma(w[i], w[i], a);
        a = row_sum16(a);
        if (gl == 0) part[j] = a;
    }
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int j = 0; j < nv; ++j) t += part[j];
        *d.fro2 = t;
    }
}

// Dynamic LDS a Jacobi workgroup may use: the device limit, capped at the
// gfx950 160 KB, less a fixed reserve for the kernels' static LDS (a few
// scalars and at most SEL_MAX-sized arrays in the selection kernels, checked
// at initialisation).  The value does not depend on anything but the limit,
// so that a planning context (no device) takes the same path decisions as a
// gfx950 device.
constexpr int LDS_STATIC_RESERVE = 1024;
static int g_lds_bytes = LDS_BYTES - LDS_STATIC_RESERVE;
// Compute units of the device (gfx950: 256), the bound of a persistent grid.
static int g_num_cu = 256;

hipError_t jacobi_init(int device) {
    int lim = 0;
    hipError_t e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (e != hipSuccess) return e;
    int ncu = 0;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    if (ncu > 0) g_num_cu = ncu;
    lim = lim < LDS_BYTES ? lim : LDS_BYTES;
    // the dynamic part may use what the kernels' static LDS leaves free
    size_t stat = 0;
    const void* kernels[] = {(const void*)jacobi_lds_kernel<0, false>, (const void*)jacobi_lds_kernel<1, false>,
                             (const void*)jacobi_lds_kernel<2, false>, (const void*)jacobi_lds_kernel<4, false>,
                             (const void*)jacobi_lds_kernel<8, false>, (const void*)jacobi_lds_kernel<16, false>,
                             (const void*)jacobi_lds_kernel<0, true>,  (const void*)jacobi_lds_kernel<1, true>,
                             (const void*)jacobi_lds_kernel<2, true>,  (const void*)jacobi_lds_kernel<4, true>,
                             (const void*)jacobi_lds_kernel<8, true>,  (const void*)jacobi_lds_kernel<16, true>,
                             (const void*)jacobi_panel_kernel<0>, (const void*)jacobi_panel_kernel<1>,
                             (const void*)jacobi_panel_kernel<2>, (const void*)jacobi_panel_kernel<4>,
                             (const void*)jacobi_panel_kernel<8>, (const void*)jacobi_panel_kernel<16>,
                             (const void*)jacobi_panel_kernel<16, 32>, (const void*)jacobi_panel_kernel<16, 64>,
                             (const void*)jacobi_panel_persistent_kernel<0>,
                             (const void*)jacobi_panel_persistent_kernel<1>,
                             (const void*)jacobi_panel_persistent_kernel<2>,
                             (const void*)jacobi_panel_persistent_kernel<4>,
                             (const void*)jacobi_panel_persistent_kernel<8>,
                             (const void*)jacobi_panel_persistent_kernel<16>,
                             (const void*)jacobi_panel_persistent_kernel<16, 32>,
                             (const void*)jacobi_panel_persistent_kernel<16, 64>,
                             (const void*)jacobi_complete_kernel};
    for (const void* f : kernels) {
        hipFuncAttributes a{};
        if (hipFuncGetAttributes(&a, f) == hipSuccess && a.sharedSizeBytes > stat) stat = a.sharedSizeBytes;
    }
    int dyn = lim - std::max(LDS_STATIC_RESERVE, (int)((stat + 255) / 256 * 256));
    bool ok = true;
    for (const void* f : kernels)
        ok = ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();  // keep the default limit
        dyn = 64 * 1024 - (int)((stat + 255) / 256 * 256);
    }
    g_lds_bytes = dyn;
    return hipSuccess;
}

int jacobi_lds_limit() { return g_lds_bytes; }

static size_t lds_need(int nvec, int len, bool acc = false) {
    const int e = elems_for(len);
    const size_t ld = e > 0 ? 16 * (size_t)e : (size_t)len;
    return sizeof(double) * ((size_t)nvec * ld + (acc ? (size_t)nvec * nvec : 0) + 2 * (size_t)nvec) +
           sizeof(int) * (size_t)nvec + 64;
}

bool jacobi_fits_lds(int nvec_cap, int len_cap, bool acc) {
    return nvec_cap <= SEL_MAX && lds_need(nvec_cap, len_cap, acc) <= (size_t)g_lds_bytes - 1024;
}

int jacobi_lds_class(int len_cap) { return elems_for(len_cap); }
size_t jacobi_lds_bytes(int nvec_cap, int len_cap, bool acc) { return lds_need(nvec_cap, len_cap, acc); }

// Shape of the blocked path for rows of at most len_cap elements: E elements
// per lane held by groups of G lanes, rows zero padded to ld = G E (E = 0:
// unpadded, strided loop), bs rows per block (a workgroup takes two blocks in
// LDS).  Rows of 257..1024 elements keep 16 elements per lane in half-wave or
// whole-wave groups (the per-pair reduction and rotation cost the same
// instructions whatever the row length, so long rows per lane amortise them),
// with a power-of-two block so that the home/away ordering applies.
struct PanelShape {
    int E, G, ld, threads, bs;
};

static PanelShape panel_shape(int len_cap) {
    PanelShape p{};
    const size_t room = (size_t)std::max(0, g_lds_bytes - 4096);
    if (len_cap > 256 && len_cap <= 1024) {
        p.G = len_cap <= 512 ? 32 : 64;
        p.E = 16;
        p.ld = p.G * p.E;
        p.threads = panel_threads(p.E, p.G);
        int bs = (int)std::min<size_t>(p.threads / p.G, room / (2 * sizeof(double) * (size_t)p.ld));
        int b2 = 1;
        while (2 * b2 <= bs) b2 <<= 1;
        p.bs = bs >= 1 ? b2 : 0;
    } else {
        p.G = 16;
        p.E = elems_for(len_cap);
        p.ld = p.E > 0 ? 16 * p.E : len_cap;
        p.threads = panel_threads(p.E, p.G);
        p.bs = (int)std::min<size_t>(32, room / (2 * sizeof(double) * (size_t)p.ld));
    }
    return p;
}

size_t jacobi_panel_bytes(int len_cap, int bs) {
    return sizeof(double) * 2 * (size_t)bs * (size_t)panel_shape(len_cap).ld;
}

void jacobi_panel_params(int nvec_cap, int len_cap, int* bs_out, int* nblk_out) {
    const int bs = std::max(1, panel_shape(len_cap).bs);
    int nblk = (nvec_cap + bs - 1) / bs;
    if (nblk & 1) ++nblk;
    if (nblk < 2) nblk = 2;
    *bs_out = bs;
    *nblk_out = nblk;
}

// One launch of the blocked path's round rd for the shape of len_cap.
static void launch_panel_round(const PanelShape& ps, dim3 grid, size_t shm, hipStream_t s, const JacobiDesc& d,
                               int rd) {
    const dim3 block(ps.threads);
    if (ps.G == 64) {
        hipLaunchKernelGGL((jacobi_panel_kernel<16, 64>), grid, block, shm, s, d, rd);
        return;
    }
    if (ps.G == 32) {
        hipLaunchKernelGGL((jacobi_panel_kernel<16, 32>), grid, block, shm, s, d, rd);
        return;
    }
    switch (ps.E) {
        case 1: hipLaunchKernelGGL(jacobi_panel_kernel<1>, grid, block, shm, s, d, rd); break;
        case 2: hipLaunchKernelGGL(jacobi_panel_kernel<2>, grid, block, shm, s, d, rd); break;
        case 4: hipLaunchKernelGGL(jacobi_panel_kernel<4>, grid, block, shm, s, d, rd); break;
        case 8: hipLaunchKernelGGL(jacobi_panel_kernel<8>, grid, block, shm, s, d, rd); break;
        case 16: hipLaunchKernelGGL(jacobi_panel_kernel<16>, grid, block, shm, s, d, rd); break;
        default: hipLaunchKernelGGL(jacobi_panel_kernel<0>, grid, block, shm, s, d, rd); break;
    }
}

// The persistent launch for the shape of len_cap: the factorizations of arr
// (count of them), or d0 alone when arr is NULL.
static void launch_panel_persistent(const PanelShape& ps, int grid, size_t shm, hipStream_t s, const JacobiDesc& d0,
                                    const JacobiDesc* arr, int count, int P, PanelQueueState* q, int max_sweeps) {
    const dim3 g(grid), block(ps.threads);
#define SMPS_PANEL_PERSISTENT(...)                                                                                  \
    hipLaunchKernelGGL((jacobi_panel_persistent_kernel<__VA_ARGS__>), g, block, shm, s, d0, arr, count, P, q, \
                       max_sweeps)
    if (ps.G == 64) {
        SMPS_PANEL_PERSISTENT(16, 64);
    } else if (ps.G == 32) {
        SMPS_PANEL_PERSISTENT(16, 32);
    } else {
        switch (ps.E) {
            case 1: SMPS_PANEL_PERSISTENT(1); break;
            case 2: SMPS_PANEL_PERSISTENT(2); break;
            case 4: SMPS_PANEL_PERSISTENT(4); break;
            case 8: SMPS_PANEL_PERSISTENT(8); break;
            case 16: SMPS_PANEL_PERSISTENT(16); break;
            default: SMPS_PANEL_PERSISTENT(0); break;
        }
    }
#undef SMPS_PANEL_PERSISTENT
}

size_t jacobi_work_doubles(int, int) { return 0; }

template <bool ACC>
static void launch_lds_t(const JacobiDesc& d, const JacobiDesc* arr, int count, int E, size_t shm, hipStream_t s,
                         int threads) {
    const dim3 g(count), b(threads);
    switch (E) {
        case 1: hipLaunchKernelGGL((jacobi_lds_kernel<1, ACC>), g, b, shm, s, d, arr); break;
        case 2: hipLaunchKernelGGL((jacobi_lds_kernel<2, ACC>), g, b, shm, s, d, arr); break;
        case 4: hipLaunchKernelGGL((jacobi_lds_kernel<4, ACC>), g, b, shm, s, d, arr); break;
        case 8: hipLaunchKernelGGL((jacobi_lds_kernel<8, ACC>), g, b, shm, s, d, arr); break;
        case 16: hipLaunchKernelGGL((jacobi_lds_kernel<16, ACC>), g, b, shm, s, d, arr); break;
        default: hipLaunchKernelGGL((jacobi_lds_kernel<0, ACC>), g, b, shm, s, d, arr); break;
    }
}

// nvec_cap > 0: a workgroup just large enough for the pairs of nvec_cap
// vectors (16 lanes per pair, the pair count rounded up to a power of two as
// the home/away ordering needs, at least one wave); 0: the class maximum.
static int lds_launch_threads(int E, int nvec_cap) {
    const int full = lds_threads(E);
    if (nvec_cap <= 0) return full;
    int p2 = 1;
    while (p2 < (nvec_cap + 1) / 2) p2 <<= 1;
    return std::max(64, std::min(full, 16 * p2));
}

static void launch_lds(const JacobiDesc& d, const JacobiDesc* arr, int count, int E, size_t shm, hipStream_t s,
                       bool acc, int nvec_cap = 0) {
    const int threads = lds_launch_threads(E, nvec_cap);
    if (acc)
        launch_lds_t<true>(d, arr, count, E, shm, s, threads);
    else
        launch_lds_t<false>(d, arr, count, E, shm, s, threads);
}

// One sweep of the global-memory path (flag reset + one launch per round) as
// a HIP graph, captured once per (device, operands, sizes) and replayed: the
// sweep is hundreds of tiny launches, and replaying them from a graph costs a
// fraction of issuing them one by one.
namespace {
struct SweepGraphs {
    std::mutex m;
    std::unordered_map<std::string, hipGraphExec_t> exec;
};
SweepGraphs& sweep_graphs() {
    static SweepGraphs g;
    return g;
}
template <typename T>
void key_add(std::string& k, const T& v) {
    k.append(reinterpret_cast<const char*>(&v), sizeof(T));
}
}  // namespace

static void enqueue_round_sweep(const JacobiDesc& dd, int rounds, int ew, dim3 grid, int* flags, hipStream_t s) {
    const dim3 block(256);
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, s, flags);
    for (int rd = 0; rd < rounds; ++rd) {
        switch (ew) {
            case 2: hipLaunchKernelGGL(jacobi_round_kernel<2>, grid, block, 0, s, dd, rd); break;
            case 4: hipLaunchKernelGGL(jacobi_round_kernel<4>, grid, block, 0, s, dd, rd); break;
            case 8: hipLaunchKernelGGL(jacobi_round_kernel<8>, grid, block, 0, s, dd, rd); break;
            case 16: hipLaunchKernelGGL(jacobi_round_kernel<16>, grid, block, 0, s, dd, rd); break;
            default: hipLaunchKernelGGL(jacobi_round_kernel<32>, grid, block, 0, s, dd, rd); break;
        }
    }
}

// One sweep of the single-problem blocked path: flag reset + one launch per
// round of the tournament over blocks.
static void enqueue_panel_sweep(const JacobiDesc& dd, const PanelShape& ps, size_t shm, int* flags, hipStream_t s) {
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, s, flags);
    for (int rd = 0; rd < dd.nblk - 1; ++rd) launch_panel_round(ps, dim3(dd.nblk / 2), shm, s, dd, rd);
}

// ew > 0: a sweep of the round kernel with ew elements per lane; ew == 0: a
// sweep of the blocked path (ps, shm).
static hipError_t round_sweep_graph(const JacobiDesc& dd, int rounds, int ew, dim3 grid, int* flags,
                                    hipGraphExec_t* out, const PanelShape* ps = nullptr, size_t shm = 0) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::string key;
    key_add(key, dev);
    key_add(key, dd.bs);
    key_add(key, dd.nblk);
    key_add(key, shm);
    if (ps) {
        key_add(key, ps->E);
        key_add(key, ps->G);
    }
    key_add(key, dd.X);
    key_add(key, dd.dims_in);
    key_add(key, dd.nvec);
    key_add(key, dd.len);
    key_add(key, dd.status);
    key_add(key, dd.fro2);
    key_add(key, dd.floor_eps);
    key_add(key, flags);
    key_add(key, rounds);
    key_add(key, ew);
    key_add(key, grid.x);
    SweepGraphs& sg = sweep_graphs();
    std::lock_guard<std::mutex> lock(sg.m);
    auto it = sg.exec.find(key);
    if (it != sg.exec.end()) {
        *out = it->second;
        return hipSuccess;
    }
    if (sg.exec.size() >= 4096) {  // bounded: drop everything and start again
        for (auto& kv : sg.exec) hipGraphExecDestroy(kv.second);
        sg.exec.clear();
    }
    hipStream_t cs;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        if (ew > 0)
            enqueue_round_sweep(dd, rounds, ew, grid, flags, cs);
        else
            enqueue_panel_sweep(dd, *ps, shm, flags, cs);
        e = hipGetLastError();
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
    }
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    hipStreamDestroy(cs);
    if (e != hipSuccess) return e;
    sg.exec.emplace(std::move(key), exec);
    *out = exec;
    return hipSuccess;
}

hipError_t launch_jacobi(const JacobiDesc& d, int nvec_cap, int len_cap, double* work, int* flags, hipStream_t s) {
    if (nvec_cap <= 0 || len_cap <= 0) return hipSuccess;
    // exact splits of short rows: the Gram / tridiagonal / divide-and-conquer
    // path when the caller provides its workspace
    if (work && !d.gram && !d.accumulate && !d.total_ext && gtd_supported(nvec_cap, len_cap))
        return launch_gtd(d, nvec_cap, len_cap, work, s);
    if (jacobi_fits_lds(nvec_cap, len_cap, d.accumulate != 0)) {
        launch_lds(d, nullptr, 1, elems_for(len_cap), lds_need(nvec_cap, len_cap, d.accumulate != 0), s,
                   d.accumulate != 0, nvec_cap);
        return hipGetLastError();
    }
    if (d.accumulate) return hipErrorInvalidValue;  // accumulation is an LDS-kernel feature
    if (nvec_cap > SEL_MAX) return hipErrorInvalidValue;
    if (len_cap > 64 * 32) return hipErrorInvalidValue;
    // `flags` is one device int used as the "rotated" flag, read by the host after every sweep
    JacobiDesc dd = d;
    dd.conv = flags;
    dd.done = nullptr;
    if (!dd.fro2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fro2_kernel, dim3(1), dim3(JT), 0, s, dd, nullptr);
    hipGraphExec_t exec = nullptr;
    const PanelShape ps = panel_shape(len_cap);
    if (len_cap <= 1024 && ps.bs >= 1) {
        // blocked path: a tournament over blocks of rows, each block pair
        // orthogonalised in LDS (one inner sweep), one launch per round
        jacobi_panel_params(nvec_cap, len_cap, &dd.bs, &dd.nblk);
        const size_t shm = jacobi_panel_bytes(len_cap, dd.bs);
        hipError_t ge = round_sweep_graph(dd, dd.nblk - 1, 0, dim3(dd.nblk / 2), flags, &exec, &ps, shm);
        if (ge != hipSuccess) return ge;
    } else {
        // rows beyond 1024 elements: one wave per pair from global memory, one
        // launch per round of the tournament over single rows
        const int P = (nvec_cap + 1) / 2, rounds = 2 * P - 1;
        const dim3 grid((P + 3) / 4);
        const int ew = len_cap <= 128 ? 2 : len_cap <= 256 ? 4 : len_cap <= 512 ? 8 : len_cap <= 1024 ? 16 : 32;
        hipError_t ge = round_sweep_graph(dd, rounds, ew, grid, flags, &exec);
        if (ge != hipSuccess) return ge;
    }
    int sweep = 0;
    bool converged = false;
    for (; sweep < ROUND_MAX_SWEEPS; ++sweep) {
        hipError_t e = hipGraphLaunch(exec, s);
        if (e != hipSuccess) return e;
        int h = 0;
        e = hipMemcpyAsync(&h, flags, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (!h) {
            converged = true;
            break;
        }
    }
    if (!converged && dd.status) hipLaunchKernelGGL(or_int_kernel, dim3(1), dim3(1), 0, s, dd.status, 2);
    hipLaunchKernelGGL(jacobi_select_kernel, dim3(1), dim3(JT), 0, s, dd, nullptr);
    // sweeps that rotated (the last, converged one did not)
    if (dd.log_sweeps) hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, s, dd.log_sweeps, sweep);
    const int rows = d.basis ? (nvec_cap > len_cap ? nvec_cap : len_cap) : nvec_cap;
    hipLaunchKernelGGL(jacobi_write_kernel, dim3((len_cap + 255) / 256, rows, 1), dim3(256), 0, s, dd, nullptr);
    if (dd.basis)
        hipLaunchKernelGGL(jacobi_complete_kernel, dim3(1), dim3(1024), sizeof(double) * complete_lds_doubles(len_cap),
                           s, dd, nullptr);
    return hipGetLastError();
}

// ---- batched forms (descriptor arrays on the device) -----------------------

hipError_t launch_jacobi_lds_batched(const JacobiDesc* arr, int count, int E, size_t shm, hipStream_t s, bool acc) {
    if (count <= 0) return hipSuccess;
    JacobiDesc none{};
    launch_lds(none, arr, count, E, shm, s, acc);
    return hipGetLastError();
}

int jacobi_panel_teams(int count, int max_pairs) {
    int teams = std::max(1, std::min(count, g_num_cu / std::max(1, max_pairs)));
    teams = std::min(teams, PANEL_MAX_TEAMS);
    if (teams >= 8) teams -= teams % 8;
    return teams;
}

// Every descriptor carries bs / nblk / fro2; q is the launch's queue state
// (PANEL_QUEUE_BYTES).  Six kernels whatever the sweep count: queue reset,
// norms, the persistent sweeps, selection, write-back, basis completion.
hipError_t launch_jacobi_panel_batched(const JacobiDesc* arr, int count, int max_pairs, int max_rows, int len_cap,
                                       size_t shm, PanelQueueState* q, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    // a team must fit on the device at one workgroup per compute unit
    if (max_pairs < 1 || max_pairs > g_num_cu) return hipErrorInvalidValue;
    JacobiDesc none{};
    hipError_t e = launch_zero_ints((int*)q, (int)(PANEL_QUEUE_BYTES / sizeof(int)), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fro2_kernel, dim3(count), dim3(JT), 0, s, none, arr);
    const PanelShape ps = panel_shape(len_cap);
    const int teams = jacobi_panel_teams(count, max_pairs);
    launch_panel_persistent(ps, teams * max_pairs, shm, s, none, arr, count, max_pairs, q, ROUND_MAX_SWEEPS);
    hipLaunchKernelGGL(jacobi_select_kernel, dim3(count), dim3(JT), 0, s, none, arr);
    hipLaunchKernelGGL(jacobi_write_kernel, dim3((len_cap + 255) / 256, max_rows, count), dim3(256), 0, s, none,
                       arr);
    hipLaunchKernelGGL(jacobi_complete_kernel, dim3(count), dim3(1024), sizeof(double) * complete_lds_doubles(len_cap),
                       s, none, arr);
    return hipGetLastError();
}

}  // namespace smps
