// Step (3) of Fig. 1 (ELSI paper, Sec. 3.1): eigenvalues and eigenvectors of
// the symmetric tridiagonal T by divide and conquer (Cuppen 1981).
//
//   * T is torn at the leaf boundaries: for a boundary coupling rho between
//     rows r and r+1, T = diag(T1', T2') + |rho| u u^T with u = e_r +
//     sign(rho) e_{r+1}, T1' and T2' having |rho| removed from their diagonal
//     ends.  Leaves (<= 64 rows) are solved by implicit QL in one workgroup.
//   * Two neighbouring solved blocks T1' = Q1 D1 Q1^T, T2' = Q2 D2 Q2^T merge
//     through the rank-one problem D + rho z z^T, z = diag(Q1, Q2)^T u:
//       - deflation (Dongarra-Sorensen): a component with rho |z_i| <= tol
//         keeps (d_i, e_i); two poles closer than tol (after a Givens rotation
//         that moves the weight of one onto the other) deflate one of them;
//       - the remaining K eigenvalues solve 1 + rho sum z_i^2 / (d_i - lam)
//         = 0, one root per interval; each root is found relative to its
//         nearer pole with a two-pole rational model (Bunch-Nielsen-Sorensen)
//         safeguarded by bisection;
//       - z is recomputed from the computed roots by the Loewner formula
//         (Gu & Eisenstat 1995) so that the eigenvectors
//         u_j = (zhat_i / (d_i - lam_j))_i are numerically orthogonal;
//       - the merged eigenvector block is diag(Q1, Q2) G U, G the deflation
//         rotations, formed by two FP64 matrix-core products.
//   * Every merge level is processed by level-wide kernels; the eigenvalues
//     of each solved block are kept sorted ascending.
#include "common.h"

#include <algorithm>
#include <vector>

namespace eg {

void dgemm(hipStream_t st, char ta, char tb, int m, int n, int k, double alpha, const double* A, int lda,
           const double* B, int ldb, double beta, double* C, int ldc, int uplo);

namespace {

constexpr int LEAF = 64;
constexpr double kEps = 2.220446049250313e-16;

// ---------------------------------------------------------------------------
// leaves: implicit QL with the shift taken from the leading 2x2 (the
// eigenvalue nearer to d_l); rotations of one sweep are recorded by thread 0
// and applied to the rows of the leaf eigenvector block by all threads.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void dc_leaf_kernel(int n, const double* __restrict__ d,
                                                     const double* __restrict__ e, double* Z, int ldz,
                                                     double* w, int* err)
{
    __shared__ double dd[LEAF], ee[LEAF];
    __shared__ double Q[LEAF][LEAF + 1];
    __shared__ double rc[LEAF], rs[LEAF];
    __shared__ int rp[LEAF];
    __shared__ int sh_l, sh_nrot, sh_fail;
    const int tid = threadIdx.x;
    const int a = blockIdx.x * LEAF;
    const int L = min(LEAF, n - a);
    if (tid < L) {
        dd[tid] = d[a + tid];
        ee[tid] = (tid + 1 < L) ? e[a + tid] : 0.0;
        for (int c = 0; c < L; ++c) Q[tid][c] = (c == tid) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        if (a > 0) dd[0] -= fabs(e[a - 1]);
        if (a + L < n) dd[L - 1] -= fabs(e[a + L - 1]);
        sh_l = 0;
        sh_fail = 0;
    }
    __syncthreads();
    int iters = 0;
    for (;;) {
        __syncthreads();
        const int l_now = sh_l;
        __syncthreads();   // every thread has read sh_l before thread 0 may change it
        if (l_now >= L) break;
        if (tid == 0) {
            int l = sh_l;
            int m = l;
            while (m < L - 1) {
                if (fabs(ee[m]) <= kEps * (fabs(dd[m]) + fabs(dd[m + 1]))) break;
                ++m;
            }
            sh_nrot = 0;
            if (m == l) {
                sh_l = l + 1;
            } else if (++iters > 30 * LEAF) {
                sh_fail = 1;
                sh_l = L;
            } else {
                if (m < L - 1) ee[m] = 0.0;
                double g = (dd[l + 1] - dd[l]) / (2.0 * ee[l]);
                double r = sqrt(g * g + 1.0);
                double mu = dd[l] - ee[l] / (g + (g >= 0.0 ? r : -r));
                double bulge = 0.0;
                int nr = 0;
                for (int pp = m - 1; pp >= l; --pp) {
                    const int qq = pp + 1;
                    double xp, xq;
                    if (pp == m - 1) { xp = ee[pp]; xq = dd[qq] - mu; }
                    else { xp = bulge; xq = ee[qq]; }
                    double rr = sqrt(xp * xp + xq * xq);
                    double c = 1.0, s = 0.0;
                    if (rr != 0.0) { c = xq / rr; s = xp / rr; }
                    if (pp != m - 1) ee[qq] = rr;
                    double a0 = dd[pp], b0 = ee[pp], c0 = dd[qq];
                    dd[pp] = c * c * a0 - 2.0 * c * s * b0 + s * s * c0;
                    ee[pp] = c * s * (a0 - c0) + (c * c - s * s) * b0;
                    dd[qq] = s * s * a0 + 2.0 * c * s * b0 + c * c * c0;
                    if (pp > l) {
                        double ep = ee[pp - 1];
                        ee[pp - 1] = c * ep;
                        bulge = s * ep;
                    }
                    rp[nr] = pp; rc[nr] = c; rs[nr] = s; ++nr;
                }
                sh_nrot = nr;
            }
        }
        __syncthreads();
        const int nr = sh_nrot;
        if (tid < L) {
            for (int t = 0; t < nr; ++t) {
                const int pp = rp[t];
                double x = Q[tid][pp], y = Q[tid][pp + 1];
                Q[tid][pp] = rc[t] * x - rs[t] * y;
                Q[tid][pp + 1] = rs[t] * x + rc[t] * y;
            }
        }
        __syncthreads();
    }
    if (tid == 0 && sh_fail) atomicOr(err, 1);
    // ascending order: rank of each eigenvalue (ties by index)
    if (tid < L) {
        double v = dd[tid];
        int rank = 0;
        for (int j = 0; j < L; ++j) rank += (dd[j] < v || (dd[j] == v && j < tid)) ? 1 : 0;
        w[a + rank] = v;
        for (int r = 0; r < L; ++r) Z[cm(a + r, a + rank, ldz)] = Q[r][tid];
    }
}

// ---------------------------------------------------------------------------
// merge bookkeeping (per merge, offset o, halves n1 + n2 = ns):
//   K[m], rho[m], zs2[m] (sum of the non-deflated z^2), nrot[m]
//   arrays indexed o + q:
//     ds, zs     non-deflated poles (ascending) and weights
//     ndrow      local row of the q-th non-deflated pole
//     rowpos     for each local row: its non-deflated position q, or -1 - (deflated slot)
//     dfv, dfrow deflated values and their local rows (slot order)
//     rot_p, rot_q, rot_c, rot_s   deflation rotations (local rows)
//     org, tau   root j = ds[org_j] + tau_j
//     zh         Loewner weights
//     colpos     final column of entry: roots at o + j, deflated at o + K + slot
// ---------------------------------------------------------------------------
struct MergeArrays {
    int *K, *nrot, *ndrow, *rowpos, *dfrow, *rot_p, *rot_q, *org, *colroot, *coldef, *perm;
    double *rho, *zs2, *ds, *zs, *dfv, *rot_c, *rot_s, *tau, *zh, *zfull, *dfull, *skey;
    int* stag;
};

typedef MergeDescH MergeDesc;

__device__ double block_reduce_sum(double v, double* red)
{
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
        red[16] = s;
    }
    __syncthreads();
    return red[16];
}

__device__ double block_reduce_max(double v, double* red)
{
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = fmax(s, red[w]);
        red[16] = s;
    }
    __syncthreads();
    return red[16];
}

// z, rho, sorted order of the poles and deflation for each merge.
__global__ __launch_bounds__(256) void dc_prep_kernel(const MergeDesc* __restrict__ md, int n,
                                                      const double* __restrict__ e, const double* __restrict__ Z,
                                                      int ldz, const double* __restrict__ w, MergeArrays ma)
{
    __shared__ double red[17];
    const int mi = blockIdx.x;
    const MergeDesc D = md[mi];
    const int o = D.o, n1 = D.n1, ns = D.n1 + D.n2;
    const int tid = threadIdx.x;
    const double rho0 = e[o + n1 - 1];
    const double sg = (rho0 >= 0.0) ? 1.0 : -1.0;
    double* zf = ma.zfull + o;
    double* df = ma.dfull + o;
    int* perm = ma.perm + o;
    // z and the (locally sorted) poles; merge-path ranks give the ascending order
    double part = 0.0, dmax = 0.0;
    for (int q = tid; q < ns; q += blockDim.x) {
        double zq = (q < n1) ? Z[cm(o + n1 - 1, o + q, ldz)] : sg * Z[cm(o + n1, o + q, ldz)];
        zf[q] = zq;
        df[q] = w[o + q];
        part += zq * zq;
        dmax = fmax(dmax, fabs(w[o + q]));
        int rank;
        double v = w[o + q];
        if (q < n1) {
            int lo = 0, hi = ns - n1;   // count of second-half values < v
            while (lo < hi) { int mid = (lo + hi) >> 1; if (w[o + n1 + mid] < v) lo = mid + 1; else hi = mid; }
            rank = q + lo;
        } else {
            int j = q - n1;
            int lo = 0, hi = n1;        // count of first-half values <= v
            while (lo < hi) { int mid = (lo + hi) >> 1; if (w[o + mid] <= v) lo = mid + 1; else hi = mid; }
            rank = j + lo;
        }
        perm[rank] = q;
    }
    const double zz = block_reduce_sum(part, red);
    dmax = block_reduce_max(dmax, red);
    const double znorm = sqrt(zz);
    const double rho = fabs(rho0) * zz;
    for (int q = tid; q < ns; q += blockDim.x) zf[q] = (znorm > 0.0) ? zf[q] / znorm : 0.0;
    __syncthreads();
    // weights and poles gathered into ascending pole order (the sort-key area
    // of this merge is free until the final ordering), so that the sequential
    // scan below reads memory in order
    double* zsort = ma.skey + 2 * o;
    double* dsort = zsort + ns;
    for (int t = tid; t < ns; t += blockDim.x) {
        const int q = perm[t];
        zsort[t] = zf[q];
        dsort[t] = df[q];
    }
    __syncthreads();
    // sequential deflation scan over the ascending poles by thread 0, the
    // pending candidate's weight and pole carried in registers.  The scan
    // reads (row, weight, pole) from LDS in chunks: waves 1.. stage chunk c+1
    // while thread 0 scans chunk c, so that it never waits on memory.
    constexpr int CH = 1024;
    __shared__ double zc[2][CH], dc[2][CH];
    __shared__ int pc[2][CH];
    for (int t = tid; t < CH && t < ns; t += blockDim.x) {
        zc[0][t] = zsort[t];
        dc[0][t] = dsort[t];
        pc[0][t] = perm[t];
    }
    __syncthreads();
    const double tol = 8.0 * kEps * fmax(dmax, rho);
    int K = 0, ndf = 0, nrot = 0;
    int pcand = -1;   // local row of the pending non-deflated candidate
    double zp = 0.0, dp = 0.0;
    double zs2 = 0.0;
    const int nch = (ns + CH - 1) / CH;
    for (int ch = 0; ch < nch; ++ch) {
        const int cb = ch & 1, c0 = ch * CH;
        if (tid == 0) {
            const int cn = min(CH, ns - c0);
            for (int u = 0; u < cn; ++u) {
                const int q = pc[cb][u];
                const double zq = zc[cb][u];
                const double dq = dc[cb][u];
                if (rho * fabs(zq) <= tol) {
                    ma.dfv[o + ndf] = dq;
                    ma.dfrow[o + ndf] = q;
                    ma.rowpos[o + q] = -1 - ndf;
                    ++ndf;
                    continue;
                }
                if (pcand >= 0) {
                    // |c s (dp - dq)| <= tol for the rotation (c, s) = (zq, zp) / r,
                    // tested as |zq zp (dp - dq)| <= tol r^2 (no root or division
                    // unless the rotation is taken)
                    const double r2 = zp * zp + zq * zq;
                    if (fabs(zq * zp * (dp - dq)) <= tol * r2) {
                        // rotate the weight of pcand onto q and deflate pcand
                        const double r = sqrt(r2);
                        const double c = zq / r, s = zp / r;
                        ma.rot_p[o + nrot] = pcand;
                        ma.rot_q[o + nrot] = q;
                        ma.rot_c[o + nrot] = c;
                        ma.rot_s[o + nrot] = s;
                        ++nrot;
                        const double dpn = c * c * dp + s * s * dq;
                        const double dqn = s * s * dp + c * c * dq;
                        zf[q] = r;
                        zf[pcand] = 0.0;
                        df[pcand] = dpn;
                        df[q] = dqn;
                        ma.dfv[o + ndf] = dpn;
                        ma.dfrow[o + ndf] = pcand;
                        ma.rowpos[o + pcand] = -1 - ndf;
                        ++ndf;
                        pcand = q;
                        zp = r;
                        dp = dqn;
                        continue;
                    }
                    // pcand is final
                    ma.ds[o + K] = dp;
                    ma.zs[o + K] = zp;
                    ma.ndrow[o + K] = pcand;
                    ma.rowpos[o + pcand] = K;
                    zs2 += zp * zp;
                    ++K;
                }
                pcand = q;
                zp = zq;
                dp = dq;
            }
        } else if (tid >= 64 && ch + 1 < nch) {
            const int nb = cb ^ 1, c1 = c0 + CH;
            for (int t = tid - 64; t < CH && c1 + t < ns; t += (int)blockDim.x - 64) {
                zc[nb][t] = zsort[c1 + t];
                dc[nb][t] = dsort[c1 + t];
                pc[nb][t] = perm[c1 + t];
            }
        }
        __syncthreads();
    }
    if (tid != 0) return;
    if (pcand >= 0) {
        ma.ds[o + K] = dp;
        ma.zs[o + K] = zp;
        ma.ndrow[o + K] = pcand;
        ma.rowpos[o + pcand] = K;
        zs2 += zp * zp;
        ++K;
    }
    ma.K[mi] = K;
    ma.nrot[mi] = nrot;
    ma.rho[mi] = rho;
    ma.zs2[mi] = zs2;
}

// Sum over the wave; every lane ends with the same bits (read from one lane).
__device__ __forceinline__ double wave_allsum(double v) { return wave_sum_dpp(v); }

// One root of 1 + rho sum_i z_i^2 / (d_i - lam) = 0 per wave: the lanes split
// the sums over i, and the iteration (identical in every lane) follows the
// two-pole rational model with a bisection safeguard.
constexpr int kRootsPerBlock = 4;
__global__ __launch_bounds__(256) void dc_secular_kernel(const MergeDesc* __restrict__ md, MergeArrays ma,
                                                         int* err)
{
    const int mi = blockIdx.y;
    const int o = md[mi].o;
    const int K = ma.K[mi];
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * kRootsPerBlock + (threadIdx.x >> 6);
    if (j >= K) return;
    const double* ds = ma.ds + o;
    const double* zs = ma.zs + o;
    const double rho = ma.rho[mi];
    if (K == 1) {
        if (lane == 0) {
            ma.org[o] = 0;
            ma.tau[o] = rho * zs[0] * zs[0];
        }
        return;
    }
    int org;
    double lo, hi, tau;
    if (j < K - 1) {
        const double gap = ds[j + 1] - ds[j];
        const double mid = 0.5 * gap;
        double f = 0.0;
        for (int i = lane; i < K; i += 64) f += rho * zs[i] * zs[i] / ((ds[i] - ds[j]) - mid);
        f = 1.0 + wave_allsum(f);
        if (f >= 0.0) { org = j; lo = 0.0; hi = mid; tau = 0.5 * mid; }
        else { org = j + 1; lo = -mid; hi = 0.0; tau = -0.5 * mid; }
    } else {
        org = K - 1;
        lo = 0.0;
        hi = rho * ma.zs2[mi];
        tau = 0.5 * hi;
    }
    const double dorg = ds[org];
    const double dL = ds[j] - dorg;
    const double dR = (j < K - 1) ? ds[j + 1] - dorg : 0.0;
    bool done = false;
    for (int it = 0; it < 120; ++it) {
        double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0, abs_sum = 0.0;
        for (int i = lane; i < K; i += 64) {
            double t = zs[i] / ((ds[i] - dorg) - tau);
            double term = zs[i] * t;
            if (i <= j) { psi += term; dpsi += t * t; }
            else { phi += term; dphi += t * t; }
            abs_sum += fabs(term);
        }
        psi = wave_allsum(psi);
        dpsi = wave_allsum(dpsi);
        phi = wave_allsum(phi);
        dphi = wave_allsum(dphi);
        abs_sum = wave_allsum(abs_sum);
        const double fr = 1.0 / rho + psi + phi;   // f / rho
        const double errb = kEps * (8.0 * (1.0 / rho + abs_sum) + fabs(tau) * (dpsi + dphi));
        if (fabs(fr) <= errb) { done = true; break; }
        if (fr < 0.0) lo = tau; else hi = tau;
        // two-pole rational model matching value and slope of psi and phi
        const double yl = dL - tau;
        const double B1 = dpsi * yl * yl;
        const double a1 = psi - dpsi * yl;
        double tn;
        if (j < K - 1) {
            const double yr = dR - tau;
            const double B2 = dphi * yr * yr;
            const double a2 = phi - dphi * yr;
            const double C = 1.0 / rho + a1 + a2;
            const double g = dR - dL;
            if (org == j) {
                const double aa = C * g + B1 + B2;
                const double disc = aa * aa - 4.0 * C * B1 * g;
                tn = dL + 2.0 * B1 * g / (aa + sqrt(fmax(disc, 0.0)));
            } else {
                const double aa = C * g - B1 - B2;
                const double disc = aa * aa + 4.0 * C * B2 * g;
                tn = dR - 2.0 * B2 * g / (-aa + sqrt(fmax(disc, 0.0)));
            }
        } else {
            const double C = 1.0 / rho + a1 + phi;
            tn = (C > 0.0) ? dL + B1 / C : 0.5 * (lo + hi);
        }
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (tn == tau) { done = true; break; }
        tau = tn;
        if (hi - lo <= 2.0 * kEps * fmax(fabs(lo), fabs(hi))) { done = true; break; }
    }
    if (lane == 0) {
        if (!done) atomicOr(err, 2);
        ma.org[o + j] = org;
        ma.tau[o + j] = tau;
    }
}

// Loewner weights: zhat_q^2 = prod_j (lam_j - d_q) / (rho prod_{j != q} (d_j - d_q)).
__global__ __launch_bounds__(256) void dc_zhat_kernel(const MergeDesc* __restrict__ md, MergeArrays ma)
{
    const int mi = blockIdx.y;
    const int o = md[mi].o;
    const int K = ma.K[mi];
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= K) return;
    const double* ds = ma.ds + o;
    const double dq = ds[q];
    const double rho = ma.rho[mi];
    auto lam_minus = [&](int j) { return ma.tau[o + j] - (dq - ds[ma.org[o + j]]); };
    double prod = lam_minus(K - 1) / rho;
    for (int j = 0; j < q; ++j) prod *= lam_minus(j) / (ds[j] - dq);
    for (int j = q; j < K - 1; ++j) prod *= lam_minus(j) / (ds[j + 1] - dq);
    double zh = sqrt(fabs(prod));
    ma.zh[o + q] = (ma.zs[o + q] >= 0.0) ? zh : -zh;
}

// Final ascending order of the merged eigenvalues: bitonic sort of
// (value, tag) with tag = root index (j) or K + deflated slot.
__global__ __launch_bounds__(1024) void dc_order_kernel(const MergeDesc* __restrict__ md, MergeArrays ma,
                                                        double* w)
{
    const int mi = blockIdx.x;
    const MergeDesc D = md[mi];
    const int o = D.o, ns = D.n1 + D.n2;
    const int K = ma.K[mi];
    int P = 1;
    while (P < ns) P <<= 1;
    double* key = ma.skey + 2 * o;   // 2*ns >= P
    int* tag = ma.stag + 2 * o;
    for (int t = threadIdx.x; t < P; t += blockDim.x) {
        double v;
        int g;
        if (t < K) { v = ma.ds[o + ma.org[o + t]] + ma.tau[o + t]; g = t; }
        else if (t < ns) { v = ma.dfv[o + t - K]; g = t; }
        else { v = INFINITY; g = 0x7fffffff; }
        key[t] = v;
        tag[t] = g;
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < P; t += blockDim.x) {
                int u = t ^ stride;
                if (u > t) {
                    bool up = ((t & size) == 0);
                    double kt = key[t], ku = key[u];
                    int gt = tag[t], gu = tag[u];
                    bool greater = (kt > ku) || (kt == ku && gt > gu);
                    if (greater == up) {
                        key[t] = ku; key[u] = kt;
                        tag[t] = gu; tag[u] = gt;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < ns; t += blockDim.x) {
        int g = tag[t];
        w[o + t] = key[t];
        if (g < K) ma.colroot[o + g] = t;
        else ma.coldef[o + g - K] = t;
    }
}

// One column of U (ns x ns at (o, o), ld ldu) per workgroup: the K root
// columns first, then the deflated ones (the merged eigenvectors are written
// to their ascending places by the products below).
__global__ __launch_bounds__(256) void dc_vectors_kernel(const MergeDesc* __restrict__ md, MergeArrays ma,
                                                         double* U, int ldu)
{
    __shared__ double red[17];
    const int mi = blockIdx.y;
    const MergeDesc D = md[mi];
    const int o = D.o, ns = D.n1 + D.n2;
    const int K = ma.K[mi];
    const int t = blockIdx.x;   // root index j (< K) or deflated slot (t - K)
    if (t >= ns) return;
    const int tid = threadIdx.x;
    if (t >= K) {
        const int slot = t - K;
        const int col = K + slot;   // deflated columns after the K root columns
        const int row = ma.dfrow[o + slot];
        for (int r = tid; r < ns; r += blockDim.x) U[cm(o + r, o + col, ldu)] = (r == row) ? 1.0 : 0.0;
        return;
    }
    const int j = t;
    const int col = j;   // root columns first; their final (sorted) places are colroot
    const double* ds = ma.ds + o;
    const double dorg = ds[ma.org[o + j]];
    const double tj = ma.tau[o + j];
    double part = 0.0;
    for (int q = tid; q < K; q += blockDim.x) {
        double v = ma.zh[o + q] / ((ds[q] - dorg) - tj);
        part += v * v;
    }
    const double nrm = sqrt(block_reduce_sum(part, red));
    const double inv = 1.0 / nrm;
    for (int r = tid; r < ns; r += blockDim.x) {
        int pos = ma.rowpos[o + r];
        double v = 0.0;
        if (pos >= 0) v = ma.zh[o + pos] / ((ds[pos] - dorg) - tj) * inv;
        U[cm(o + r, o + col, ldu)] = v;
    }
}

// U <- G U with G = R_1 R_2 ... R_t (deflation rotations), one column per thread.
__global__ __launch_bounds__(256) void dc_rot_kernel(const MergeDesc* __restrict__ md, MergeArrays ma, double* U,
                                                     int ldu)
{
    const int mi = blockIdx.y;
    const MergeDesc D = md[mi];
    const int o = D.o, ns = D.n1 + D.n2;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ns) return;
    const int nrot = ma.nrot[mi];
    double* col = U + cm(o, o + c, ldu);
    for (int r = nrot - 1; r >= 0; --r) {
        const int p = ma.rot_p[o + r], q = ma.rot_q[o + r];
        const double cc = ma.rot_c[o + r], ss = ma.rot_s[o + r];
        const double up = col[p], uq = col[q];
        col[p] = cc * up + ss * uq;
        col[q] = -ss * up + cc * uq;
    }
}

// Deflated columns of the merged eigenvector block: column K + slot of U is
// G e_row (a few nonzeros along its rotation chain), so its eigenvector is a
// short combination of columns of the block-diagonal input, written to its
// ascending place coldef[slot] when that is below ncol.  One workgroup per
// deflated column; the nonzeros are gathered and put in row order, so the
// sums run in a fixed order.
__global__ __launch_bounds__(256) void dc_deflated_kernel(const MergeDesc* __restrict__ md, MergeArrays ma,
                                                          const double* __restrict__ Zin, double* Zout, int ldz,
                                                          const double* __restrict__ U, int ldu, int ncol)
{
    __shared__ int nzr[256];
    __shared__ double nzv[256];
    __shared__ int cnt;
    const int mi = blockIdx.y;
    const MergeDesc D = md[mi];
    const int o = D.o, n1 = D.n1, ns = D.n1 + D.n2;
    const int K = ma.K[mi];
    const int slot = blockIdx.x;
    if (slot >= ns - K) return;
    const int col = ma.coldef[o + slot];
    if (col >= ncol) return;
    const int tid = threadIdx.x;
    const double* u = U + cm(o, o + K + slot, ldu);
    if (tid == 0) cnt = 0;
    __syncthreads();
    for (int r = tid; r < ns; r += blockDim.x) {
        const double v = u[r];
        if (v != 0.0) {
            const int p = atomicAdd(&cnt, 1);
            if (p < 256) { nzr[p] = r; nzv[p] = v; }
        }
    }
    __syncthreads();
    const int c = cnt;
    if (c <= 256) {
        if (tid == 0) {   // insertion sort by row: a fixed summation order
            for (int a = 1; a < c; ++a) {
                const int r = nzr[a];
                const double v = nzv[a];
                int b = a - 1;
                while (b >= 0 && nzr[b] > r) { nzr[b + 1] = nzr[b]; nzv[b + 1] = nzv[b]; --b; }
                nzr[b + 1] = r;
                nzv[b + 1] = v;
            }
        }
        __syncthreads();
        for (int i = tid; i < ns; i += blockDim.x) {
            const bool top = i < n1;
            double acc = 0.0;
            for (int q = 0; q < c; ++q) {
                const int r = nzr[q];
                if ((r < n1) == top) acc += Zin[cm(o + i, o + r, ldz)] * nzv[q];
            }
            Zout[cm(o + i, o + col, ldz)] = acc;
        }
    } else {
        for (int i = tid; i < ns; i += blockDim.x) {
            const int r0 = (i < n1) ? 0 : n1, r1 = (i < n1) ? n1 : ns;
            double acc = 0.0;
            for (int r = r0; r < r1; ++r) {
                const double v = u[r];
                if (v != 0.0) acc += Zin[cm(o + i, o + r, ldz)] * v;
            }
            Zout[cm(o + i, o + col, ldz)] = acc;
        }
    }
}

}  // namespace

size_t stedc_workspace_bytes(int n)
{
    // MergeArrays: 11 int arrays and 12 double arrays of n (+2n for the sort), plus per-merge scalars
    size_t b = 0;
    b += (size_t)n * sizeof(int) * 12 + (size_t)2 * n * sizeof(int);
    b += (size_t)n * sizeof(double) * 12 + (size_t)2 * n * sizeof(double);
    b += (size_t)(n / LEAF + 2) * (2 * sizeof(int) + 2 * sizeof(double) + sizeof(MergeDesc));
    return b + 4096;
}

// Phase 1 of the tridiagonal solve: every eigenvalue (w, ascending) and every
// merge level except the products of the last one, whose coefficient block U
// is left ready.  Phase 2 (stedc_vectors) forms the eigenvectors of the
// lowest ncol eigenvalues only -- the top merge dominates the cost, and the
// density matrix needs only the states with non-negligible occupation.
// The merge bookkeeping laid out in the solver's scratch (the same layout for
// both phases).
static MergeArrays merge_arrays(void* work, int n, MergeDesc** mdev_out)
{
    char* p = (char*)work;
    auto take = [&](size_t bytes) { void* r = p; p += align_up(bytes, 256); return r; };
    MergeArrays ma;
    ma.K = (int*)take(sizeof(int) * (n / LEAF + 2));
    ma.nrot = (int*)take(sizeof(int) * (n / LEAF + 2));
    ma.rho = (double*)take(sizeof(double) * (n / LEAF + 2));
    ma.zs2 = (double*)take(sizeof(double) * (n / LEAF + 2));
    ma.ndrow = (int*)take(sizeof(int) * n);
    ma.rowpos = (int*)take(sizeof(int) * n);
    ma.dfrow = (int*)take(sizeof(int) * n);
    ma.rot_p = (int*)take(sizeof(int) * n);
    ma.rot_q = (int*)take(sizeof(int) * n);
    ma.org = (int*)take(sizeof(int) * n);
    ma.colroot = (int*)take(sizeof(int) * n);
    ma.coldef = (int*)take(sizeof(int) * n);
    ma.perm = (int*)take(sizeof(int) * n);
    ma.stag = (int*)take(sizeof(int) * 2 * n);
    ma.ds = (double*)take(sizeof(double) * n);
    ma.zs = (double*)take(sizeof(double) * n);
    ma.dfv = (double*)take(sizeof(double) * n);
    ma.rot_c = (double*)take(sizeof(double) * n);
    ma.rot_s = (double*)take(sizeof(double) * n);
    ma.tau = (double*)take(sizeof(double) * n);
    ma.zh = (double*)take(sizeof(double) * n);
    ma.zfull = (double*)take(sizeof(double) * n);
    ma.dfull = (double*)take(sizeof(double) * n);
    ma.skey = (double*)take(sizeof(double) * 2 * n);
    MergeDesc* mdev = (MergeDesc*)take(sizeof(MergeDesc) * (n / LEAF + 2));
    *mdev_out = mdev;
    return ma;
}

int stedc_values(hipStream_t st, int n, const double* d, const double* e, double* w, double* Z, double* Z2,
                 double* U, int ldz, void* work, int* err, DcState* state)
{
    MergeDesc* mdev = nullptr;
    MergeArrays ma = merge_arrays(work, n, &mdev);

    state->n = n;
    state->ldz = ldz;
    state->Z = Z;
    state->Zin = Z;
    state->Zout = Z2;
    state->U = U;
    state->have_last = false;
    fill_i(st, err, 1, 0);
    const int nleaf = ceil_div(n, LEAF);
    hipLaunchKernelGGL(dc_leaf_kernel, dim3(nleaf), dim3(64), 0, st, n, d, e, Z, ldz, w, err);
    if (nleaf == 1) return 0;

    // subproblem sizes per level: blocks of LEAF * 2^lev, merged in pairs; the
    // descriptors of all levels are uploaded once
    std::vector<MergeDesc> all;
    std::vector<int> lev_start;
    for (int size = LEAF; size < n; size *= 2) {
        lev_start.push_back((int)all.size());
        for (int o = 0; o < n; o += 2 * size) {
            int n1 = std::min(size, n - o);
            int n2 = std::min(size, n - o - n1);
            if (n2 <= 0) continue;   // odd block passes through unchanged
            all.push_back(MergeDesc{o, n1, n2});
        }
    }
    lev_start.push_back((int)all.size());
    if (hipMemcpyAsync(mdev, all.data(), sizeof(MergeDesc) * all.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return kStatusHip;
    double* Zin = Z;
    double* Zout = Z2;
    int lev = 0;
    for (int size = LEAF; size < n; size *= 2, ++lev) {
        const int nm = lev_start[lev + 1] - lev_start[lev];
        const MergeDesc* mdl = mdev + lev_start[lev];
        std::vector<MergeDesc> md(all.begin() + lev_start[lev], all.begin() + lev_start[lev + 1]);
        const int maxns = 2 * size;
        const bool last = (2 * size >= n);
        hipLaunchKernelGGL(dc_prep_kernel, dim3(nm), dim3(256), 0, st, mdl, n, e, Zin, ldz, w, ma);
        hipLaunchKernelGGL(dc_secular_kernel, dim3(ceil_div(maxns, kRootsPerBlock), nm), dim3(256), 0, st, mdl, ma,
                           err);
        hipLaunchKernelGGL(dc_zhat_kernel, dim3(ceil_div(maxns, 256), nm), dim3(256), 0, st, mdl, ma);
        hipLaunchKernelGGL(dc_order_kernel, dim3(nm), dim3(1024), 0, st, mdl, ma, w);
        hipLaunchKernelGGL(dc_vectors_kernel, dim3(maxns, nm), dim3(256), 0, st, mdl, ma, U, ldz);
        hipLaunchKernelGGL(dc_rot_kernel, dim3(ceil_div(maxns, 256), nm), dim3(256), 0, st, mdl, ma, U, ldz);
        if (last) {
            state->Zin = Zin;
            state->Zout = Zout;
            state->last = md;
            state->last_dev = mdl;
            state->work = work;
            state->have_last = true;
            return 0;
        }
        // blocks that pass through unchanged keep their columns: copy them across
        for (int o = 0; o < n; o += 2 * size) {
            int n1 = std::min(size, n - o);
            if (n - o - n1 <= 0) copy_matrix(st, n1, n1, Zin + cm(o, o, ldz), ldz, Zout + cm(o, o, ldz), ldz);
        }
        // merged eigenvectors: the root columns by two products each (written
        // to their ascending places), the deflated ones from their few nonzeros
        std::vector<int> Ks(nm);
        if (hipMemcpyAsync(Ks.data(), ma.K + 0, sizeof(int) * nm, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return kStatusHip;
        for (int q = 0; q < nm; ++q) {
            const MergeDesc& m = md[q];
            const int K = Ks[q];
            if (K <= 0) continue;
            dgemm_colmap(st, m.n1, K, m.n1, 1.0, Zin + cm(m.o, m.o, ldz), ldz, U + cm(m.o, m.o, ldz), ldz, 0.0,
                         Zout + cm(m.o, m.o, ldz), ldz, ma.colroot + m.o);
            dgemm_colmap(st, m.n2, K, m.n2, 1.0, Zin + cm(m.o + m.n1, m.o + m.n1, ldz), ldz,
                         U + cm(m.o + m.n1, m.o, ldz), ldz, 0.0, Zout + cm(m.o + m.n1, m.o, ldz), ldz,
                         ma.colroot + m.o);
        }
        hipLaunchKernelGGL(dc_deflated_kernel, dim3(maxns, nm), dim3(256), 0, st, mdl, ma, Zin, Zout, ldz, U, ldz,
                           maxns);
        std::swap(Zin, Zout);
    }
    return 0;
}

// Phase 2: eigenvectors of the lowest ncol eigenvalues into state->Z (n x ncol).
void stedc_vectors(hipStream_t st, DcState& state, int ncol)
{
    if (!state.have_last || ncol <= 0) return;
    const int ldz = state.ldz;
    double* Zin = state.Zin;
    double* Zout = state.Zout;
    double* U = state.U;
    MergeDesc* mdev_all = nullptr;
    MergeArrays ma = merge_arrays(state.work, state.n, &mdev_all);
    const int nm = (int)state.last.size();
    // the last level is one merge (its two halves span all n rows)
    std::vector<int> Ks(nm);
    if (hipMemcpyAsync(Ks.data(), ma.K, sizeof(int) * nm, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return;
    int maxns = 0;
    for (int q = 0; q < nm; ++q) {
        const MergeDesc& m = state.last[q];
        const int ns = m.n1 + m.n2;
        maxns = std::max(maxns, ns);
        // roots ascend with their index, so the wanted ones (ascending place
        // below ncol) are a leading run of the K root columns; the run is taken
        // up to the last wanted root, so an equal-valued neighbour cannot be lost
        const int K = Ks[q];
        std::vector<int> cr(std::max(K, 1));
        if (K > 0 && (hipMemcpyAsync(cr.data(), ma.colroot + m.o, sizeof(int) * K, hipMemcpyDeviceToHost, st) !=
                          hipSuccess ||
                      hipStreamSynchronize(st) != hipSuccess))
            return;
        int J = 0;
        for (int j = 0; j < K; ++j)
            if (cr[j] < ncol) J = j + 1;
        if (J == 0) continue;
        dgemm_colmap(st, m.n1, J, m.n1, 1.0, Zin + cm(m.o, m.o, ldz), ldz, U + cm(m.o, m.o, ldz), ldz, 0.0,
                     Zout + cm(m.o, m.o, ldz), ldz, ma.colroot + m.o);
        dgemm_colmap(st, m.n2, J, m.n2, 1.0, Zin + cm(m.o + m.n1, m.o + m.n1, ldz), ldz,
                     U + cm(m.o + m.n1, m.o, ldz), ldz, 0.0, Zout + cm(m.o + m.n1, m.o, ldz), ldz,
                     ma.colroot + m.o);
    }
    hipLaunchKernelGGL(dc_deflated_kernel, dim3(maxns, nm), dim3(256), 0, st, state.last_dev, ma, Zin, Zout, ldz,
                       U, ldz, ncol);
    if (Zout != state.Z) copy_matrix(st, state.n, std::min(state.n, ncol), Zout, ldz, state.Z, ldz);
    state.have_last = false;
}

// Both phases: all n eigenvalues, eigenvectors of the lowest ncol_final.
int stedc(hipStream_t st, int n, const double* d, const double* e, double* w, double* Z, double* Z2,
          double* U, int ldz, int ncol_final, void* work, int* err, int* err_host_copy)
{
    (void)err_host_copy;
    DcState state;
    int rc = stedc_values(st, n, d, e, w, Z, Z2, U, ldz, work, err, &state);
    if (rc) return rc;
    stedc_vectors(st, state, ncol_final);
    return 0;
}

}  // namespace eg
