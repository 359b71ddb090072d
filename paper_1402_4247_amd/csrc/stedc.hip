// Real symmetric tridiagonal eigensolver on the GPU: the tridiagonal step of
// Eigen_HH (Section III of arXiv:1402.4247 calls a LAPACK routine there; the
// paper does not fix which).  Divide and conquer, batched over k-points:
//
//  * Cuppen's rank-one tearing down to leaves of at most LEAF rows: at a split
//    between rows mid-1 and mid, T = diag(T1', T2') + |beta| u u^T with
//    u = e_{mid-1} + sign(beta) e_mid and the two corner diagonal entries
//    lowered by |beta|;
//  * each leaf solved by the parallel cyclic Jacobi method (Golub & Van Loan
//    §8.5), one wave per leaf;
//  * per merge: z = Q^T u / sqrt(2), rho = 2 |beta|, deflation of negligible
//    z components and of close pole pairs by Givens rotations (Dongarra &
//    Sorensen 1987);
//  * the secular equation 1 + rho sum z_i^2 / (d_i - lambda) = 0 solved for
//    each root in coordinates shifted to its nearer pole, with a two-pole
//    rational model step (Li 1993, "middle way") safeguarded by bisection;
//  * eigenvectors from the Loewner-recomputed z (Gu & Eisenstat 1994), so
//    they are numerically orthogonal whatever the root spacing;
//  * Q_new = Q V as a real product on FP64 MFMA, one launch per tree level.
// The tree over [0, n) splits segment [floor(j n / 2^t), floor((j+1) n / 2^t))
// at depth t; every segment of size >= 2 has two non-empty children.
#include <algorithm>

#include "common.hpp"
#include "lanes.hpp"
#include "kernels.hpp"

namespace kgev {

namespace {

constexpr double EPS = 2.220446049250313e-16;

__device__ __host__ inline int64_t seg_bound(int64_t j, int64_t n, int t) { return (j * n) >> t; }

struct Seg {
    int64_t s, e, mid;
};

__device__ inline Seg seg_of(int64_t j, int64_t n, int t)
{
    Seg g;
    g.s = seg_bound(j, n, t);
    g.e = seg_bound(j + 1, n, t);
    g.mid = seg_bound(2 * j + 1, n, t + 1);
    return g;
}

constexpr int LEAF = 16;   // largest leaf of the tree

// depth of the leaves: the smallest depth whose segments have at most LEAF rows
__host__ __device__ inline int dc_leaf_depth(int64_t n)
{
    int t = 0;
    while (((int64_t)LEAF << t) < n) ++t;
    return t;
}

// row i starts a segment at depth t (i > 0: the boundary before it is torn)
__device__ inline bool starts_segment(int64_t i, int64_t n, int t)
{
    const int64_t j = ((i << t) + n - 1) / n;      // smallest j with j n / 2^t >= i
    return seg_bound(j, n, t) == i;
}

// ---------------------------------------------------------------------------
// Scale T to max |entry| = 1 and lower the diagonal by the rank-one tears of
// the leaf boundaries (depth tl); D = the torn diagonal.
__global__ __launch_bounds__(256) void dc_init(DcWs ws, int tl)
{
    __shared__ double sh[4];
    const int64_t b = blockIdx.x;
    const int n = ws.n;
    const double* d = ws.din + b * ws.s_din;
    const double* e = ws.ein + b * ws.s_din;
    double mx = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        mx = fmax(mx, fabs(d[i]));
        if (i + 1 < n) mx = fmax(mx, fabs(e[i]));
    }
    mx = dpp_wave_max(mx);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    double org = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    if (!(org > 0.0) || !isfinite(org)) org = (org == 0.0) ? 1.0 : org;
    if (threadIdx.x == 0) ws.onrm[b] = org;
    const double inv = 1.0 / org;
    double* D = ws.D[0] + b * ws.n;
    double* es = ws.es + b * ws.n;
    for (int i = threadIdx.x; i < n; i += 256) {
        double v = d[i] * inv;
        if (i > 0 && starts_segment(i, n, tl)) v -= fabs(e[i - 1] * inv);
        if (i + 1 < n && starts_segment(i + 1, n, tl)) v -= fabs(e[i] * inv);
        D[i] = v;
        es[i] = (i + 1 < n) ? e[i] * inv : 0.0;
    }
}

// d (double) of lane i: a wave-uniform read of a lane-distributed array
__device__ inline double rdl(double v, int i) { return lane_read(v, i); }

// LDS written by a wave and then read by other lanes of the same wave: a
// wave-scope fence and a scheduling barrier, no workgroup barrier
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Leaf eigensolver: one wave per leaf segment (at most LEAF rows) of the torn
// tridiagonal, by the parallel cyclic Jacobi method (Golub & Van Loan §8.5):
// the leaf is held as a dense symmetric LEAF x LEAF matrix in LDS (rows past
// the leaf are zero and never rotated), and each sweep takes LEAF - 1 rounds of
// LEAF / 2 disjoint rotations (round-robin pairing with the last index fixed).
// A rotation of the (p, q) plane with c = 1 / sqrt(1 + t^2), s = t c,
// t = sign(tau) / (|tau| + sqrt(1 + tau^2)), tau = (a_qq - a_pp) / (2 a_pq),
// zeroes a_pq; each lane forms the rotation of pair lane mod 8 and applies it
// to two rows (then two columns): the columns of A and of the accumulated V
// together, then the rows of A.  An off-diagonal entry
// at most eps * max_i(|d_i| + |e_i|) is left alone (the normwise deflation
// threshold of implicit QL); a sweep that rotates nothing ends the iteration.
// Eigenvalues go to D[0] ascending, the eigenvectors (columns of V) to the
// leaf's diagonal block of Q[0] (the rest of Q[0] is the identity's zeros).
// The rounds are short dependent chains of LDS traffic, where a QL sweep is a
// chain of rotations, each with a square root and a reciprocal.
constexpr int LEAF_SWEEPS = 30;

__device__ inline void leaf_pair(int r, int k, int& p, int& q)
{
    // round r of the circle method on LEAF indices: index LEAF - 1 is fixed,
    // the others rotate; pair k of the round
    constexpr int M = LEAF - 1;
    if (k == 0) {
        p = r;
        q = M;
    } else {
        p = (r + k) % M;
        q = (r + M - k) % M;
    }
    if (p > q) {
        const int t = p;
        p = q;
        q = t;
    }
}

__global__ __launch_bounds__(64) void dc_leaf(DcWs ws, int tl)
{
    __shared__ double As[LEAF][LEAF + 1];
    __shared__ double Vs[LEAF][LEAF + 1];
    const int64_t b = blockIdx.y;
    const int64_t n = ws.n;
    const Seg g = seg_of(blockIdx.x, n, tl);
    const int s = (int)g.s, ns = (int)(g.e - g.s);
    if (ns < 1) return;
    const int lane = threadIdx.x;
    double* D = ws.D[0] + b * n;
    const double* es = ws.es + b * n;
    const double dr = lane < ns ? D[s + lane] : 0.0;
    const double er = lane + 1 < ns ? es[s + lane] : 0.0;
    // the deflation threshold from the leaf's norm (max over rows of |d| + |e|)
    const double tol = 2.220446049250313e-16 * dpp_wave_max(fabs(dr) + fabs(er));
    for (int e = lane; e < LEAF * LEAF; e += 64) {
        const int i = e / LEAF, j = e % LEAF;
        double a = 0.0;
        if (i < ns && j < ns) {
            if (i == j) a = D[s + i];
            else if (j == i + 1) a = es[s + i];
            else if (i == j + 1) a = es[s + j];
        }
        As[i][j] = a;
        Vs[i][j] = (i == j) ? 1.0 : 0.0;
    }
    wave_sync();
    bool conv = false;
    for (int sweep = 0; sweep < LEAF_SWEEPS; ++sweep) {
        bool rotated = false;
        for (int r = 0; r < LEAF - 1; ++r) {
            // every lane forms the rotation of pair k = lane mod 8, the pair
            // of both its items below, so no LDS round trip shares it
            int p, q;
            leaf_pair(r, lane % (LEAF / 2), p, q);
            const double apq = As[p][q];
            double c = 1.0, sn = 0.0;
            if (fabs(apq) > tol) {
                const double tau = (As[q][q] - As[p][p]) / (2.0 * apq);
                const double t = copysign(1.0, tau) / (fabs(tau) + sqrt(fma(tau, tau, 1.0)));
                c = 1.0 / sqrt(fma(t, t, 1.0));
                sn = t * c;
                rotated = true;
            }
            // a round in which no pair rotates (all of the final sweep) leaves
            // A and V as they are: skip its two phases
            if (!__builtin_amdgcn_ballot_w64(sn != 0.0)) continue;
            wave_sync();
            // columns p, q of A and of V: rows i = lane / 8 and lane / 8 + 8
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i = lane / (LEAF / 2) + 8 * h;
                const double aip = As[i][p], aiq = As[i][q];
                const double vip = Vs[i][p], viq = Vs[i][q];
                As[i][p] = c * aip - sn * aiq;
                As[i][q] = sn * aip + c * aiq;
                Vs[i][p] = c * vip - sn * viq;
                Vs[i][q] = sn * vip + c * viq;
            }
            wave_sync();
            // rows p, q of A: columns j = lane / 8 and lane / 8 + 8; the
            // rotated entry is set to its exact value 0
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int j = lane / (LEAF / 2) + 8 * h;
                const double apj = As[p][j], aqj = As[q][j];
                const bool rot = sn != 0.0;
                As[p][j] = (rot && j == q) ? 0.0 : c * apj - sn * aqj;
                As[q][j] = (rot && j == p) ? 0.0 : sn * apj + c * aqj;
            }
            wave_sync();
        }
        if (!__builtin_amdgcn_ballot_w64(rotated)) {
            conv = true;
            break;
        }
    }
    if (!conv && lane == 0 && ws.status) atomicOr(ws.status + b, ST_NOCONV);
    // ascending order: the rank of lane j's value (ties by index)
    const double lam = lane < ns ? As[lane][lane] : 0.0;
    int rank = 0;
    for (int k = 0; k < ns; ++k) {
        const double dk = rdl(lam, k);
        rank += (dk < lam || (dk == lam && k < lane)) ? 1 : 0;
    }
    if (lane < ns) D[s + rank] = lam;
    double* Q = ws.Q[0] + b * ws.sQ;
    for (int j = 0; j < ns; ++j) {
        const int rj = __builtin_amdgcn_readlane(rank, j);
        if (lane < ns) Q[(int64_t)(s + lane) + (int64_t)(s + rj) * n] = Vs[lane][j];
    }
}

// Q = I for the leaves (buffer 0); grid (ceil(n*n/256), nk)
__global__ __launch_bounds__(256) void dc_eye(DcWs ws)
{
    const int64_t b = blockIdx.y;
    const int64_t nn = (int64_t)ws.n * ws.n;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nn) return;
    const int64_t i = q % ws.n, j = q / ws.n;
    ws.Q[0][b * ws.sQ + q] = (i == j) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
// Deflation for one merge (one workgroup per segment and problem).
__global__ __launch_bounds__(256) void dc_deflate(DcWs ws, int t, int rb, int lds_cap)
{
    __shared__ double sh[8];
    extern __shared__ double dyn[];   // lds_cap doubles sd, lds_cap doubles sz, lds_cap ints perm
    const int64_t b = blockIdx.y;
    const int64_t n = ws.n;
    const Seg g = seg_of(blockIdx.x, n, t);
    const int ns = (int)(g.e - g.s);
    if (ns <= 0) return;
    const int64_t s = g.s;
    const double* Dr = ws.D[rb] + b * n;
    double* Qr = ws.Q[rb] + b * ws.sQ;
    int* kc = ws.kcnt + b * n;
    int* ndc = ws.ndcnt + b * n;
    // the serial deflation scan reads these at every step: keep them in LDS
    // when the segment fits
    const bool in_lds = (int)(g.e - g.s) <= lds_cap;
    int* perm = in_lds ? reinterpret_cast<int*>(dyn + 2 * lds_cap) : ws.perm + b * n + s;
    double* sd = in_lds ? dyn : ws.sd + b * n + s;
    double* sz = in_lds ? dyn + lds_cap : ws.sz + b * n + s;
    int* ndx = ws.ndx + b * n + s;
    double* ndd = ws.ndd + b * n + s;
    double* ndz = ws.ndz + b * n + s;
    int* dfx = ws.dfx + b * n + s;
    double* dfd = ws.dfd + b * n + s;
    int* rota = ws.rota + b * n + s;
    int* rotb = ws.rotb + b * n + s;
    double* rotc = ws.rotc + b * n + s;
    double* rots = ws.rots + b * n + s;
    const int tid = threadIdx.x;

    if (ns == 1) {
        if (tid == 0) {
            kc[s] = 0;
            ndc[s] = 1;
            dfx[0] = 0;
            dfd[0] = Dr[s];
            ws.nrot[b * n + s] = 0;
            ws.rho[b * n + s] = 0.0;
        }
        return;
    }
    const int n1 = (int)(g.mid - g.s);
    const double beta = ws.es[b * n + g.mid - 1];
    const double rho = 2.0 * fabs(beta);
    const double sgn = (beta >= 0.0) ? 1.0 : -1.0;
    const double rs2 = 0.70710678118654752440;

    // stable merge of the two sorted halves: perm[pos] = local column.  perm
    // starts as the identity so it stays a valid index list even if the
    // inputs hold NaNs (then positions may collide).
    for (int c = tid; c < ns; c += 256) perm[c] = c;
    __syncthreads();
    double dmx = 0.0, zmx = 0.0;
    for (int c = tid; c < ns; c += 256) {
        const double dc = Dr[s + c];
        const double zc = (c < n1) ? Qr[(g.mid - 1) + (s + c) * n] * rs2 : sgn * Qr[g.mid + (s + c) * n] * rs2;
        int pos;
        if (c < n1) {
            int lo = n1, hi = ns;      // count right-half entries strictly below dc
            while (lo < hi) { int md = (lo + hi) >> 1; if (Dr[s + md] < dc) lo = md + 1; else hi = md; }
            pos = c + (lo - n1);
        } else {
            int lo = 0, hi = n1;       // count left-half entries <= dc
            while (lo < hi) { int md = (lo + hi) >> 1; if (Dr[s + md] <= dc) lo = md + 1; else hi = md; }
            pos = (c - n1) + lo;
        }
        pos = min(max(pos, 0), ns - 1);
        perm[pos] = c;
        sd[pos] = dc;
        sz[pos] = zc;
        dmx = fmax(dmx, fabs(dc));
        zmx = fmax(zmx, fabs(zc));
    }
    dmx = dpp_wave_max(dmx);
    zmx = dpp_wave_max(zmx);
    if ((tid & 63) == 0) { sh[tid >> 6] = dmx; sh[4 + (tid >> 6)] = zmx; }
    __syncthreads();
    dmx = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    zmx = fmax(fmax(sh[4], sh[5]), fmax(sh[6], sh[7]));
    const double tol = 8.0 * EPS * fmax(dmx, zmx);

    __shared__ int s_nrot;
    if (tid == 0) {
        int K = 0, nd = 0, nr = 0;
        if (rho * zmx <= tol) {
            for (int q = 0; q < ns; ++q) { dfx[nd] = perm[q]; dfd[nd] = sd[q]; ++nd; }
        } else {
            // the pending kept candidate (pole d_p, component z_p, column c_p)
            // is carried in registers; a rotation folds it into the next one
            bool have = false;
            double zp = 0.0, dpv = 0.0;
            int cp = 0;
            // the candidates are read from LDS four at a time, ahead of the
            // serial decisions that use them
            constexpr int DQ = 4;
            for (int q0 = 0; q0 < ns; q0 += DQ) {
                double zq4[DQ], dq4[DQ];
                int cq4[DQ];
#pragma unroll
                for (int u = 0; u < DQ; ++u) {
                    const int q = q0 + u < ns ? q0 + u : q0;
                    zq4[u] = sz[q];
                    dq4[u] = sd[q];
                    cq4[u] = perm[q];
                }
#pragma unroll
                for (int u = 0; u < DQ; ++u) {
                    if (q0 + u >= ns) break;
                    const double zq = zq4[u], dq = dq4[u];
                    const int cq = cq4[u];
                    if (rho * fabs(zq) <= tol) {
                        dfx[nd] = cq; dfd[nd] = dq; ++nd;
                    } else if (!have) {
                        have = true; zp = zq; dpv = dq; cp = cq;
                    } else {
                        // |gap c s| <= tol with c = z_q / tau, s = -z_p / tau,
                        // tau^2 = z_q^2 + z_p^2, tested without the square
                        // root and the divisions
                        const double gap = dq - dpv;
                        if (fabs(gap * zq * zp) <= tol * (zq * zq + zp * zp)) {
                            const double tau = hypot(zq, zp);
                            const double c = zq / tau, sn = -zp / tau;
                            rota[nr] = cp; rotb[nr] = cq; rotc[nr] = c; rots[nr] = sn; ++nr;
                            dfx[nd] = cp; dfd[nd] = dpv * c * c + dq * sn * sn; ++nd;
                            zp = tau;
                            dpv = dpv * sn * sn + dq * c * c;
                            cp = cq;
                        } else {
                            ndx[K] = cp; ndd[K] = dpv; ndz[K] = zp; ++K;
                            zp = zq; dpv = dq; cp = cq;
                        }
                    }
                }
            }
            if (have) { ndx[K] = cp; ndd[K] = dpv; ndz[K] = zp; ++K; }
        }
        kc[s] = K;
        ndc[s] = nd;
        ws.nrot[b * n + s] = nr;
        ws.rho[b * n + s] = rho;
        s_nrot = nr;
    }
    __syncthreads();
    const int nr = s_nrot;
    // apply the deflation rotations, in order, to the columns of Q (rows s..e).
    // Consecutive rotations chain through their second column (the pending
    // candidate), so that column is carried in a register: no rotation waits
    // for the store of the one before it to come back from memory.
    for (int r = tid; r < ns; r += 256) {
        const int64_t row = s + r;
        int cur = -1;            // column held in cv (not yet stored), or -1
        double cv = 0.0;
        for (int q = 0; q < nr; ++q) {
            const int ca = rota[q], cb = rotb[q];
            const double x = ca == cur ? cv : Qr[row + (s + ca) * n];
            const double y = cb == cur ? cv : Qr[row + (s + cb) * n];
            if (cur >= 0 && cur != ca && cur != cb) Qr[row + (s + cur) * n] = cv;
            Qr[row + (s + ca) * n] = rotc[q] * x + rots[q] * y;
            cur = cb;
            cv = rotc[q] * y - rots[q] * x;
        }
        if (cur >= 0) Qr[row + (s + cur) * n] = cv;
    }
}

// ---------------------------------------------------------------------------
// Secular equation: SEC_LANES lanes cooperate on one root: lane `sub` sums
// the terms q = sub mod SEC_LANES and a butterfly of xor steps adds the
// partial sums.  Floating-point addition is commutative, so every lane of the
// root ends with bitwise equal sums and takes the same branches.  Sixteen
// lanes (four roots per wave) gave the top merges enough waves to hide the
// divide latency: 1.1% off the n = 2000 x 16 step against four lanes, with 32
// lanes equal and 64 slower.
constexpr int SEC_LANES = 16;

__device__ inline double root_sum(double v)
{
    return dpp_sum<SEC_LANES>(v);
}

__device__ inline void secular_eval(int K, const double* dl, const double* zl, double rho, int j, double dorg,
                                    double tau, int sub, double& f, double& psi, double& dpsi, double& phi,
                                    double& dphi)
{
    psi = 0.0; dpsi = 0.0; phi = 0.0; dphi = 0.0;
    for (int q = sub; q < K; q += SEC_LANES) {
        const double del = (dl[q] - dorg) - tau;
        const double r = 1.0 / del;
        const double tq = zl[q] * zl[q] * r;
        if (q <= j) { psi += tq; dpsi = fma(tq, r, dpsi); }
        else { phi += tq; dphi = fma(tq, r, dphi); }
    }
    psi = rho * root_sum(psi);
    dpsi = rho * root_sum(dpsi);
    phi = rho * root_sum(phi);
    dphi = rho * root_sum(dphi);
    f = 1.0 + psi + phi;
}

__global__ __launch_bounds__(64) void dc_secular(DcWs ws, int t)
{
    const int64_t b = blockIdx.z;
    const int64_t n = ws.n;
    const Seg g = seg_of(blockIdx.y, n, t);
    if (g.e - g.s < 2) return;
    const int64_t s = g.s;
    const int K = ws.kcnt[b * n + s];
    const int gt = blockIdx.x * 64 + threadIdx.x;
    const int j = gt / SEC_LANES, sub = gt % SEC_LANES;
    if (j >= K) return;          // the lanes of a root leave together
    const double* dl = ws.ndd + b * n + s;
    const double* zl = ws.ndz + b * n + s;
    const double rho = ws.rho[b * n + s];

    int org;
    double lo, hi;
    double f, psi, dpsi, phi, dphi;
    if (K == 1) {
        // one pole: lambda = d + rho z^2 exactly
        const double tau1 = rho * zl[0] * zl[0];
        if (sub == 0) {
            ws.orgi[b * n + s] = 0;
            ws.tauv[b * n + s] = tau1;
            ws.lam[b * n + s] = dl[0] + tau1;
        }
        return;
    }
    if (j < K - 1) {
        const double half = 0.5 * (dl[j + 1] - dl[j]);
        secular_eval(K, dl, zl, rho, j, dl[j], half, sub, f, psi, dpsi, phi, dphi);
        if (f >= 0.0) { org = j; lo = 0.0; hi = half; }
        else { org = j + 1; lo = -half; hi = 0.0; }
    } else {
        double zz = 0.0;
        for (int q = sub; q < K; q += SEC_LANES) zz = fma(zl[q], zl[q], zz);
        zz = root_sum(zz);
        org = j; lo = 0.0; hi = rho * zz;
        for (int g2 = 0; g2 < 8; ++g2) {
            secular_eval(K, dl, zl, rho, j, dl[org], hi, sub, f, psi, dpsi, phi, dphi);
            if (f >= 0.0) break;
            lo = hi; hi *= 2.0;
        }
    }
    const double dorg = dl[org];
    const double P1 = dl[j] - dorg;
    const double P2 = (j < K - 1) ? dl[j + 1] - dorg : 0.0;
    double tau = 0.5 * (lo + hi);
    bool conv = false;
    for (int it = 0; it < 400; ++it) {
        secular_eval(K, dl, zl, rho, j, dorg, tau, sub, f, psi, dpsi, phi, dphi);
        if (f == 0.0) { conv = true; break; }
        if (f < 0.0) lo = tau; else hi = tau;
        if (fabs(f) <= 8.0 * EPS * (1.0 + fabs(psi) + fabs(phi)) * (double)(K > 8 ? 8 : K)) { conv = true; break; }
        if (hi - lo <= 4.0 * EPS * fmax(fabs(lo), fabs(hi))) { conv = true; break; }
        // two-pole rational model through (tau, f, f')
        double cand = 0.5 * (lo + hi);
        const double d1 = P1 - tau;
        if ((it & 7) != 7) {
            if (j < K - 1) {
                const double d2 = P2 - tau;
                const double s1 = dpsi * d1 * d1, s2 = dphi * d2 * d2;
                const double c = 1.0 + (psi - dpsi * d1) + (phi - dphi * d2);
                const double Bq = c * (d1 + d2) + s1 + s2;
                const double Cq = d1 * d2 * f;
                double eta;
                bool okq = true;
                if (c == 0.0) {
                    eta = Cq / Bq;
                } else {
                    const double disc = Bq * Bq - 4.0 * c * Cq;
                    if (disc < 0.0) okq = false;
                    const double sq = sqrt(fmax(disc, 0.0));
                    const double den = (Bq >= 0.0) ? (Bq + sq) : (Bq - sq);
                    eta = (den != 0.0) ? 2.0 * Cq / den : 0.0;
                    const double x2 = tau + eta;
                    if (!(x2 > lo && x2 < hi)) eta = den / (2.0 * c);
                }
                const double x = tau + eta;
                if (okq && x > lo && x < hi && isfinite(x)) cand = x;
            } else {
                const double s1 = dpsi * d1 * d1;
                const double c = 1.0 + (psi - dpsi * d1) + phi;
                if (c != 0.0) {
                    const double x = tau + d1 + s1 / c;
                    if (x > lo && x < hi && isfinite(x)) cand = x;
                }
            }
        }
        if (cand == tau) cand = 0.5 * (lo + hi);
        tau = cand;
    }
    if (sub != 0) return;
    ws.orgi[b * n + s + j] = org;
    ws.tauv[b * n + s + j] = tau;
    ws.lam[b * n + s + j] = dorg + tau;
    if (!conv && ws.status) atomicOr(ws.status + b, ST_NOCONV);
}

// z recomputed from the roots (Loewner), one thread per pole.
__global__ __launch_bounds__(64) void dc_zhat(DcWs ws, int t)
{
    const int64_t b = blockIdx.z;
    const int64_t n = ws.n;
    const Seg g = seg_of(blockIdx.y, n, t);
    if (g.e - g.s < 2) return;
    const int64_t s = g.s;
    const int K = ws.kcnt[b * n + s];
    // SEC_LANES lanes per index i: lane `sub` multiplies the factors
    // q = sub mod SEC_LANES, a butterfly of products combines them (bitwise
    // equal in every lane of the group)
    const int gt = blockIdx.x * 64 + threadIdx.x;
    const int i = gt / SEC_LANES, sub = gt % SEC_LANES;
    if (i >= K) return;          // the lanes of an index leave together
    const double* dl = ws.ndd + b * n + s;
    const double* zl = ws.ndz + b * n + s;
    const int* org = ws.orgi + b * n + s;
    const double* tv = ws.tauv + b * n + s;
    const double rho = ws.rho[b * n + s];
    const double di = dl[i];
    double p = sub == 0 ? ((dl[org[i]] - di) + tv[i]) / rho : 1.0;
    for (int q = sub; q < K; q += SEC_LANES) {
        if (q == i) continue;
        p *= ((dl[org[q]] - di) + tv[q]) / (dl[q] - di);
    }
    p = dpp_prod<SEC_LANES>(p);
    if (sub == 0) ws.zhat[b * n + s + i] = copysign(sqrt(fmax(p, 0.0)), zl[i]);
}

// Eigenvectors of D + rho z z^T: column j = zhat / (d - lambda_j), normalised.
// One wave per column, the lanes over its rows (coalesced stores).
__global__ __launch_bounds__(64) void dc_vectors(DcWs ws, int t)
{
    const int64_t b = blockIdx.z;
    const int64_t n = ws.n;
    const Seg g = seg_of(blockIdx.y, n, t);
    if (g.e - g.s < 2) return;
    const int64_t s = g.s;
    const int K = ws.kcnt[b * n + s];
    const int j = blockIdx.x;
    if (j >= K) return;
    const int lane = threadIdx.x;
    const double* dl = ws.ndd + b * n + s;
    const double* zh = ws.zhat + b * n + s;
    const int oj = ws.orgi[b * n + s + j];
    const double tj = ws.tauv[b * n + s + j];
    const double dorg = dl[oj];
    double ss = 0.0;
    for (int i = lane; i < K; i += 64) {
        const double v = zh[i] / ((dl[i] - dorg) - tj);
        ss += v * v;
    }
    ss = dpp_wave_sum(ss);
    const double inv = 1.0 / sqrt(ss);
    double* Vc = ws.Vsec + b * ws.sQ + (s + j) * n + s;
    for (int i = lane; i < K; i += 64) Vc[i] = zh[i] / ((dl[i] - dorg) - tj) * inv;
}

// Final ascending order of the merged eigenvalues (secular roots and deflated
// poles): one thread per value counts the values that precede it.
__global__ __launch_bounds__(64) void dc_order(DcWs ws, int t, int wb)
{
    const int64_t b = blockIdx.z;
    const int64_t n = ws.n;
    const Seg g = seg_of(blockIdx.y, n, t);
    const int ns = (int)(g.e - g.s);
    if (ns < 1) return;
    const int64_t s = g.s;
    const int K = ws.kcnt[b * n + s];
    const int nd = ws.ndcnt[b * n + s];
    // SEC_LANES lanes per value, each counting a strided share of the others
    const int gt = blockIdx.x * 64 + threadIdx.x;
    const int q = gt / SEC_LANES, sub = gt % SEC_LANES;
    if (q >= K + nd) return;          // the lanes of a value leave together
    const double* lam = ws.lam + b * n + s;
    const double* dfd = ws.dfd + b * n + s;
    const double v = (q < K) ? lam[q] : dfd[q - K];
    int rank = 0;
    for (int r = sub; r < K + nd; r += SEC_LANES) {
        const double u = (r < K) ? lam[r] : dfd[r - K];
        if (u < v || (u == v && r < q)) ++rank;
    }
    rank = dpp_sum<SEC_LANES>(rank);
    if (sub != 0) return;
    rank = min(rank, ns - 1);
    ws.D[wb][b * n + s + rank] = v;
    ws.cmap[b * n + s + q] = rank;      // entries [0,K): product columns, [K,K+nd): deflated
}

// Deflated columns move unchanged (after rotation) to their place, and every
// column of the segment gets zeros in the rows of its parent segment that lie
// outside it (the parent merge reads its whole diagonal block).
__global__ __launch_bounds__(256) void dc_place(DcWs ws, int t, int rb, int wb)
{
    const int64_t b = blockIdx.z;
    const int64_t n = ws.n;
    const Seg g = seg_of(blockIdx.y, n, t);
    const int ns = (int)(g.e - g.s);
    const int q = blockIdx.x;
    if (q >= ns) return;
    const int64_t s = g.s;
    double* Qw = ws.Q[wb] + b * ws.sQ;
    if (t > 0) {
        const Seg pg = seg_of(blockIdx.y >> 1, n, t - 1);
        double* col = Qw + (s + q) * n;
        for (int64_t r = pg.s + threadIdx.x; r < pg.e; r += 256)
            if (r < g.s || r >= g.e) col[r] = 0.0;
    }
    const int K = ws.kcnt[b * n + s];
    const int nd = ws.ndcnt[b * n + s];
    if (q >= nd) return;
    const int src = ws.dfx[b * n + s + q];
    const int dst = ws.cmap[b * n + s + K + q];
    const double* Qr = ws.Q[rb] + b * ws.sQ + (s + src) * n + s;
    double* Qd = Qw + (s + dst) * n + s;
    for (int r = threadIdx.x; r < ns; r += 256) Qd[r] = Qr[r];
}

// Q_new(s:e, s + cmap[j]) = sum_q Q(s:e, s + ndx[q]) V(q, j): real product on
// FP64 MFMA with a column gather on A and a column scatter on C.
constexpr int DB = 64, DK = 16;
__global__ __launch_bounds__(256) void dc_gemm(DcWs ws, int t, int rb, int wb, int tiles)
{
    __shared__ double sA[2][DK][DB + 1];
    __shared__ double sB[2][DK][DB + 1];
    const int64_t b = blockIdx.z;
    const int64_t n = ws.n;
    const Seg g = seg_of(blockIdx.y, n, t);
    const int ns = (int)(g.e - g.s);
    if (ns < 2) return;
    const int64_t s = g.s;
    const int K = ws.kcnt[b * n + s];
    const int tm = blockIdx.x % tiles, tn = blockIdx.x / tiles;
    const int i0 = tm * DB, j0 = tn * DB;
    if (i0 >= ns || j0 >= K) return;
    const double* Qr = ws.Q[rb] + b * ws.sQ;
    const double* Vs = ws.Vsec + b * ws.sQ;
    const int* ndx = ws.ndx + b * n + s;
    const int* cmap = ws.cmap + b * n + s;
    double* Qw = ws.Q[wb] + b * ws.sQ;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int li = lane & 15, lk = lane >> 4;
    d4_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[a][c][r] = 0.0;

    const int nkt = (K + DK - 1) / DK;
    // tile loads from clamped (in-bounds) indices with no branch, so the next
    // K step stays in flight during the MFMA work; the bounds mask is applied
    // when the registers are stored to LDS
    double ra[4], rbv[4];
    unsigned oka = 0, okb = 0;
    auto gload = [&](int k0) {
        // A tile: rows i0..i0+63 (lanes), k = k0 + kq + 4q, columns gathered through ndx
        const int r = tid & 63, kq = tid >> 6;
        const int ic = i0 + r < ns ? i0 + r : 0;
        oka = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + kq + 4 * q;
            const int kc = k < K ? k : 0;
            ra[q] = Qr[(s + ic) + (s + ndx[kc]) * n];
            oka |= (unsigned)(i0 + r < ns && k < K) << q;
        }
        // B tile: k = k0 + (tid & 15), cols j0 + (tid >> 4) + 16 q
        const int kk = tid & 15, jq = tid >> 4;
        const int k = k0 + kk;
        const int kc = k < K ? k : 0;
        okb = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int jj = j0 + jq + 16 * q;
            const int jc = jj < K ? jj : 0;
            rbv[q] = Vs[(s + kc) + (s + jc) * n];
            okb |= (unsigned)(jj < K && k < K) << q;
        }
    };
    auto sstore = [&](int buf) {
        const int r = tid & 63, kq = tid >> 6;
#pragma unroll
        for (int q = 0; q < 4; ++q) sA[buf][kq + 4 * q][r] = ((oka >> q) & 1u) ? ra[q] : 0.0;
        const int kk = tid & 15, jq = tid >> 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) sB[buf][kk][jq + 16 * q] = ((okb >> q) & 1u) ? rbv[q] : 0.0;
    };
    int cur = 0;
    if (nkt > 0) { gload(0); sstore(0); }
    __syncthreads();
    for (int kt = 0; kt < nkt; ++kt) {
        if (kt + 1 < nkt) gload((kt + 1) * DK);
#pragma unroll
        for (int ks = 0; ks < DK; ks += 4) {
            double a0 = sA[cur][ks + lk][wm * 32 + li];
            double a1 = sA[cur][ks + lk][wm * 32 + 16 + li];
            double b0 = sB[cur][ks + lk][wn * 32 + li];
            double b1 = sB[cur][ks + lk][wn * 32 + 16 + li];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (kt + 1 < nkt) sstore(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wm * 32 + a * 16 + Mfma<double>::row(lk, r);
                const int jj = j0 + wn * 32 + c * 16 + li;
                if (i < ns && jj < K) Qw[(s + i) + (s + cmap[jj]) * n] = acc[a][c][r];
            }
}

__global__ __launch_bounds__(256) void dc_finish(DcWs ws, int fb, double* w)
{
    const int64_t b = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= ws.n) return;
    w[b * ws.s_w + i] = ws.D[fb][b * ws.n + i] * ws.onrm[b];
}

}  // namespace

hipError_t stedc(hipStream_t st, const DcWs& ws0, double* w, double* Z, double* Qscratch, int64_t nk)
{
    DcWs ws = ws0;
    const int64_t n = ws.n;
    if (n < 1 || nk < 1) return hipSuccess;
    const int L = dc_leaf_depth(n);
    // the leaves write buffer 0 and the last merge level buffer L & 1: make
    // that the caller's Z
    ws.Q[L & 1] = Z;
    ws.Q[(L & 1) ^ 1] = Qscratch;
    hipLaunchKernelGGL(dc_init, dim3((unsigned)nk), dim3(256), 0, st, ws, L);
    hipLaunchKernelGGL(dc_eye, dim3((unsigned)((n * n + 255) / 256), (unsigned)nk), dim3(256), 0, st, ws);
    hipLaunchKernelGGL(dc_leaf, dim3(1u << L, (unsigned)nk), dim3(64), 0, st, ws, L);
    for (int t = L - 1; t >= 0; --t) {
        const int rb = (L - t - 1) & 1, wb = (L - t) & 1;
        const unsigned segs = 1u << t;
        const int64_t nsmax = ((n + segs - 1) / segs) + 1;
        const int cap = (int)std::min<int64_t>(nsmax, 3200);
        const size_t dyn_bytes = (size_t)cap * (2 * sizeof(double) + sizeof(int));
        hipLaunchKernelGGL(dc_deflate, dim3(segs, (unsigned)nk), dim3(256), dyn_bytes, st, ws, t, rb, cap);
        const unsigned gxs = (unsigned)((nsmax * SEC_LANES + 63) / 64);
        hipLaunchKernelGGL(dc_secular, dim3(gxs, segs, (unsigned)nk), dim3(64), 0, st, ws, t);
        hipLaunchKernelGGL(dc_zhat, dim3(gxs, segs, (unsigned)nk), dim3(64), 0, st, ws, t);
        hipLaunchKernelGGL(dc_vectors, dim3((unsigned)nsmax, segs, (unsigned)nk), dim3(64), 0, st, ws, t);
        hipLaunchKernelGGL(dc_order, dim3(gxs, segs, (unsigned)nk), dim3(64), 0, st, ws, t, wb);
        hipLaunchKernelGGL(dc_place, dim3((unsigned)nsmax, segs, (unsigned)nk), dim3(256), 0, st, ws, t, rb, wb);
        const int tiles = (int)((nsmax + DB - 1) / DB);
        hipLaunchKernelGGL(dc_gemm, dim3((unsigned)(tiles * tiles), segs, (unsigned)nk), dim3(256), 0, st, ws, t, rb, wb,
                           tiles);
    }
    hipLaunchKernelGGL(dc_finish, dim3((unsigned)((n + 255) / 256), (unsigned)nk), dim3(256), 0, st, ws, L & 1, w);
    return hipGetLastError();
}

}  // namespace kgev
