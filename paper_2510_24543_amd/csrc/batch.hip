// Batched multi-instance PCG for gfx950: the pointwise kernels of one PCG
// round over a group of instances with the same grid shape, and the scalar
// decisions of the CG loop (arXiv:2510.24543, Sec. III Algorithm 1, Sec. IV,
// Sec. V) on the device, one thread per instance.  A round is
//   direction reduce -> decide_dir -> direction write + line-search FFTs ->
//   decide_step -> trial + Hamiltonian FFTs -> decide_accept,
// and every kernel skips the instances whose flags say the step does not
// apply to them (converged, backtracking, restarting), so the same kernel
// sequence serves all instances and can be replayed from a graph.
#include "bec_internal.h"
#include "pcg_rules.h"
#include "pw_math.h"

namespace bec {
namespace {

struct LdsNodes {
    const double (*nd)[kNodeVals];
    __device__ double operator()(int q, int k) const { return nd[q][k]; }
};

__device__ __forceinline__ void load_nodes(const BInstParams& P, double (*nd)[kNodeVals])
{
    for (int t = threadIdx.x; t < (P.n_a + P.n_b) * kNodeVals; t += blockDim.x)
        nd[t / kNodeVals][t % kNodeVals] = P.node5[t / kNodeVals][t % kNodeVals];
    __syncthreads();
}

__device__ __forceinline__ double btrap(const BGroup& g, int l, long long i)
{
    const uint32_t ii = (uint32_t)i;   // points per instance < 2^31 (checked at creation)
    const uint32_t ix = (uint32_t)(((uint64_t)ii * g.m_nyz) >> g.s_nyz);
    const uint32_t rem = ii - ix * (uint32_t)(g.ny * g.nz);
    const uint32_t iy = (uint32_t)(((uint64_t)rem * g.m_nz) >> g.s_nz);
    const uint32_t iz = rem - iy * (uint32_t)g.nz;
    return g.vx[(long long)l * g.nx + ix] + g.vy[(long long)l * g.ny + iy] + g.vz[(long long)l * g.nz + iz];
}

template <int M>
__device__ __forceinline__ void bblock_store(const double (&acc)[M], double* partials_l, int nblk)
{
    __shared__ double sh[M][kPwThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = acc[m];
    wave_sum_down(v);
    if (lane == 0)
#pragma unroll
        for (int m = 0; m < M; ++m) sh[m][w] = v[m];
    __syncthreads();
    if (threadIdx.x < M) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kPwThreads / 64; ++k) s += sh[threadIdx.x][k];
        partials_l[(long long)threadIdx.x * nblk + blockIdx.x] = s;
    }
}

#define BSTRIDE(i, N)                                                                          \
    for (long long i = (long long)blockIdx.x * kPwThreads + threadIdx.x; i < (N);             \
         i += (long long)gridDim.x * kPwThreads)

__global__ __launch_bounds__(kPwThreads) void b_norm2_kernel(BGroup g)
{
    const int l = g.ids[blockIdx.y], inst = g.first + l;
    const long long N = g.N;
    const double2* f = reinterpret_cast<const double2*>(g.psi_user[inst]);
    double acc[2] = {0.0, 0.0};
    BSTRIDE(i, N)
    {
        acc[0] += sq2(f[i]);
        acc[1] += sq2(f[N + i]);
    }
    bblock_store<2>(acc, g.partials + (long long)l * kMaxSums * g.nblk, g.nblk);
}

__global__ __launch_bounds__(kPwThreads) void b_heval_epi_kernel(BGroup g)
{
    const int l = g.ids[blockIdx.y], inst = g.first + l;
    if (!g.act_trial[inst]) return;
    __shared__ double nd[kMaxNodes][kNodeVals];
    const BInstParams& P = g.ip[inst];
    load_nodes(P, nd);
    const LdsNodes nodes{nd};
    const long long N = g.N;
    const int tb = 1 - g.st[inst].cur;
    const double2* psi = g.psi + ((long long)l * 2 + tb) * 2 * N;
    const double2* Tpsi = g.W + (long long)l * 3 * N;
    const double2* phi = Tpsi + 2 * N;
    double2* hpsi = g.hpsi + ((long long)l * 2 + tb) * 2 * N;
    double2* aux = g.aux + ((long long)l * 2 + tb) * 2 * N;
    const int n_a = P.n_a, n_b = P.n_b, lhy = P.lhy_on;
    const double K5 = P.K5, K3 = P.K3;
    double acc[kHevalSums];
#pragma unroll
    for (int m = 0; m < kHevalSums; ++m) acc[m] = 0.0;
    BSTRIDE(i, N)
    {
        const double2 s1 = psi[i], s2 = psi[N + i];
        const double2 t1 = Tpsi[i], t2 = Tpsi[N + i];
        const double2 ph = phi[i];
        const double n1 = sq2(s1), n2 = sq2(s2);
        const double V = btrap(g, l, i);
        double e = 0.0, d1 = 0.0, d2 = 0.0;
        if (lhy) lhy_point(nodes, LhyTab{P.lhytab, P.lhy_K}, n_a, n_b, K5, K3, n1, n2, e, d1, d2);
        const double m1 = d1 / P.Nat[0], m2 = d2 / P.Nat[1];
        const double U1 = V + P.G[0][0] * n1 + P.G[0][1] * n2 + P.Gdd[0][0] * ph.x + P.Gdd[0][1] * ph.y + m1;
        const double U2 = V + P.G[1][0] * n1 + P.G[1][1] * n2 + P.Gdd[1][0] * ph.x + P.Gdd[1][1] * ph.y + m2;
        const double2 h1 = make_double2(t1.x + U1 * s1.x, t1.y + U1 * s1.y);
        const double2 h2 = make_double2(t2.x + U2 * s2.x, t2.y + U2 * s2.y);
        hpsi[i] = h1;
        hpsi[N + i] = h2;
        aux[i] = ph;
        aux[N + i] = make_double2(m1, m2);
        acc[0] += redot(s1, t1);
        acc[1] += redot(s2, t2);
        acc[2] += V * n1;
        acc[3] += V * n2;
        acc[4] += n1 * n1;
        acc[5] += n1 * n2;
        acc[6] += n2 * n2;
        acc[7] += n1 * ph.x;
        acc[8] += n1 * ph.y;
        acc[9] += n2 * ph.x;
        acc[10] += n2 * ph.y;
        acc[11] += e;
        acc[12] += redot(s1, h1);
        acc[13] += redot(s2, h2);
        acc[14] += n1;
        acc[15] += n2;
        acc[16] += m1 * n1;
        acc[17] += m2 * n2;
    }
    bblock_store<kHevalSums>(acc, g.partials + (long long)l * kMaxSums * g.nblk, g.nblk);
}

struct BRZ {
    double2 r[2], z[2];
};

// 1 / ([shift_c + V + sum_j G_cj n_j + muLHY_c]_+ + sigma): the inverse P_V diagonal
__device__ __forceinline__ double b_pv_inv(const BInstParams& P, int c, double shift, double sigma, double V, double n1,
                                           double n2, double ml)
{
    const double q = shift + V + P.G[c][0] * n1 + P.G[c][1] * n2 + ml;
    return 1.0 / ((q > 0.0 ? q : 0.0) + sigma);
}

// residual r = H psi - mu psi and z at point i; z by the group's zmode, or by
// the instance's fallback (S.zlevel 2: P_V^-1 r, 3: r)
__device__ __forceinline__ BRZ b_resid(const BGroup& g, const BInstParams& P, const BInstState& S, int l,
                                       long long i, const double2* hpsi, const double2* aux, double2 s1, double2 s2)
{
    const long long N = g.N;
    BRZ o;
    const double2 h1 = hpsi[i], h2 = hpsi[N + i];
    o.r[0] = make_double2(h1.x - S.mu[0] * s1.x, h1.y - S.mu[0] * s1.y);
    o.r[1] = make_double2(h2.x - S.mu[1] * s2.x, h2.y - S.mu[1] * s2.y);
    const int zm = S.zlevel == 2 ? 1 : S.zlevel == 3 ? 0 : g.zmode;
    if (zm == 0) {
        o.z[0] = o.r[0];
        o.z[1] = o.r[1];
        return o;
    }
    const double2* zb = g.zbuf + (long long)l * 2 * N;
    if (zm == 2) {
        o.z[0] = zb[i];
        o.z[1] = zb[N + i];
        return o;
    }
    const double n1 = sq2(s1), n2 = sq2(s2);
    const double V = btrap(g, l, i);
    const double2 ml = aux[N + i];
    const double q[2] = {b_pv_inv(P, 0, S.shift[0], g.sigma, V, n1, n2, ml.x),
                         b_pv_inv(P, 1, S.shift[1], g.sigma, V, n1, n2, ml.y)};
    double w[2] = {1.0, 1.0};
    if (zm == 4) rule_blend(S.hsum, S.shift, g.blend, w);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        if (zm == 1) {
            o.z[c] = make_double2(q[c] * o.r[c].x, q[c] * o.r[c].y);
        } else if (zm == 3) {
            const double sq = sqrt(q[c]);
            const double2 v = zb[c * N + i];
            o.z[c] = make_double2(sq * v.x, sq * v.y);
        } else {
            const double a = w[c] * q[c], b = 1.0 - w[c];
            const double2 v = zb[c * N + i];
            o.z[c] = make_double2(a * o.r[c].x + b * v.x, a * o.r[c].y + b * v.y);
        }
    }
    return o;
}

// zbuf = r, P_V^-1 r or D^-1/2 r (g.papply) for the instances that compute a
// new z this round; the k-space passes then apply P_Delta^-1 in place.
__global__ __launch_bounds__(kPwThreads) void b_make_r_kernel(BGroup g)
{
    const int l = g.ids[blockIdx.y], inst = g.first + l;
    if (!g.act_pre[inst]) return;
    const BInstState& S = g.st[inst];
    const BInstParams& P = g.ip[inst];
    const long long N = g.N;
    const double2* psi = g.psi + ((long long)l * 2 + S.cur) * 2 * N;
    const double2* hpsi = g.hpsi + ((long long)l * 2 + S.cur) * 2 * N;
    const double2* aux = g.aux + ((long long)l * 2 + S.cur) * 2 * N;
    double2* out = g.zbuf + (long long)l * 2 * N;
    BSTRIDE(i, N)
    {
        const double2 s[2] = {psi[i], psi[N + i]};
        double2 r[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const double2 h = hpsi[c * N + i];
            r[c] = make_double2(h.x - S.mu[c] * s[c].x, h.y - S.mu[c] * s[c].y);
        }
        if (g.papply != 0) {
            const double n1 = sq2(s[0]), n2 = sq2(s[1]);
            const double V = btrap(g, l, i);
            const double2 ml = aux[N + i];
            const double mlc[2] = {ml.x, ml.y};
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double q = b_pv_inv(P, c, S.shift[c], g.sigma, V, n1, n2, mlc[c]);
                if (g.papply == 2) q = sqrt(q);
                r[c] = make_double2(q * r[c].x, q * r[c].y);
            }
        }
        out[i] = r[0];
        out[N + i] = r[1];
    }
}

__global__ void b_mark_pre_kernel(int n, const BInstState* st, int* act_pre)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const BInstState& S = st[i];
    act_pre[i] = (S.status == kBRunning && S.phase == kBNewDir && S.zlevel == 0) ? 1 : 0;
}

__global__ __launch_bounds__(kPwThreads) void b_dir_reduce_kernel(BGroup g)
{
    const int l = g.ids[blockIdx.y], inst = g.first + l;
    const BInstState& S = g.st[inst];
    if (S.status != kBRunning || S.phase != kBNewDir) return;
    const BInstParams& P = g.ip[inst];
    const long long N = g.N;
    const int cur = S.cur, have_prev = S.have_prev;
    const double2* psi = g.psi + ((long long)l * 2 + cur) * 2 * N;
    const double2* hpsi = g.hpsi + ((long long)l * 2 + cur) * 2 * N;
    const double2* aux = g.aux + ((long long)l * 2 + cur) * 2 * N;
    const double2* r_old = g.r_old + (long long)l * 2 * N;
    const double2* p = g.p + (long long)l * 2 * N;
    double acc[kDirReduceSums];
#pragma unroll
    for (int m = 0; m < kDirReduceSums; ++m) acc[m] = 0.0;
    BSTRIDE(i, N)
    {
        const double2 s[2] = {psi[i], psi[N + i]};
        const BRZ q = b_resid(g, P, S, l, i, hpsi, aux, s[0], s[1]);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            acc[6 * c + 0] += sq2(q.r[c]);
            acc[6 * c + 3] += redot(q.z[c], s[c]);
            acc[6 * c + 5] += redot(q.r[c], q.z[c]);
            if (have_prev) {
                const double2 ro = r_old[c * N + i], po = p[c * N + i];
                const double2 y = make_double2(q.r[c].x - ro.x, q.r[c].y - ro.y);
                acc[6 * c + 1] += redot(y, q.z[c]);
                acc[6 * c + 2] += redot(y, po);
                acc[6 * c + 4] += redot(po, s[c]);
            }
        }
    }
    bblock_store<kDirReduceSums>(acc, g.partials + (long long)l * kMaxSums * g.nblk, g.nblk);
}

__global__ __launch_bounds__(kPwThreads) void b_dir_write_kernel(BGroup g)
{
    const int l = g.ids[blockIdx.y], inst = g.first + l;
    if (!g.act_dir[inst]) return;
    __shared__ double nd[kMaxNodes][kNodeVals];
    const BInstParams& P = g.ip[inst];
    load_nodes(P, nd);
    const LdsNodes nodes{nd};
    const BInstState& S = g.st[inst];
    const long long N = g.N;
    const int cur = S.cur;
    const double beta = S.beta, c0 = S.c[0], c1 = S.c[1];
    const double2* psi = g.psi + ((long long)l * 2 + cur) * 2 * N;
    const double2* hpsi = g.hpsi + ((long long)l * 2 + cur) * 2 * N;
    const double2* aux = g.aux + ((long long)l * 2 + cur) * 2 * N;
    double2* p = g.p + (long long)l * 2 * N;
    double2* r_out = g.r_old + (long long)l * 2 * N;
    double2* rho_o = g.rho + (long long)l * N;
    const int n_a = P.n_a, n_b = P.n_b, lhy = P.lhy_on;
    double acc[kDirWriteSums];
#pragma unroll
    for (int m = 0; m < kDirWriteSums; ++m) acc[m] = 0.0;
    BSTRIDE(i, N)
    {
        const double2 s[2] = {psi[i], psi[N + i]};
        const BRZ q = b_resid(g, P, S, l, i, hpsi, aux, s[0], s[1]);
        const double2 h[2] = {hpsi[i], hpsi[N + i]};
        const double2 ph = aux[i], ml = aux[N + i];
        const double mlc[2] = {ml.x, ml.y};
        const double n[2] = {sq2(s[0]), sq2(s[1])};
        const double V = btrap(g, l, i);
        const double cc[2] = {c0, c1};
        double2 pv[2];
        double rho[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            double2 d = make_double2(-q.z[c].x, -q.z[c].y);
            if (beta != 0.0) {
                const double2 po = p[c * N + i];
                d.x += beta * po.x;
                d.y += beta * po.y;
            }
            pv[c] = make_double2(d.x - cc[c] * s[c].x, d.y - cc[c] * s[c].y);
            p[c * N + i] = pv[c];
            r_out[c * N + i] = q.r[c];
            rho[c] = redot(s[c], pv[c]);
            const double2 hmf = make_double2(h[c].x - mlc[c] * s[c].x, h[c].y - mlc[c] * s[c].y);
            const double U = V + P.G[c][0] * n[0] + P.G[c][1] * n[1] + P.Gdd[c][0] * ph.x + P.Gdd[c][1] * ph.y;
            const double pp = sq2(pv[c]);
            acc[0 + c] += pp;
            acc[2 + c] += redot(pv[c], q.r[c]);
            acc[4 + c] += redot(pv[c], hmf);
            acc[6 + c] += redot(s[c], hmf);
            acc[8 + c] += U * pp;
            acc[10 + c] += mlc[c] * pp;
            acc[12 + c] += mlc[c] * n[c];
            acc[16 + c] += rho[c];
        }
        rho_o[i] = make_double2(rho[0], rho[1]);
        if (lhy) {
            double L1, L2;
            lhy_model(nodes, LhyTab{P.lhytab, P.lhy_K}, n_a, n_b, n[0], n[1], 2.0 * rho[0], 2.0 * rho[1], L1, L2);
            acc[14] += L1;
            acc[15] += L2;
        }
    }
    bblock_store<kDirWriteSums>(acc, g.partials + (long long)l * kMaxSums * g.nblk, g.nblk);
}

__global__ __launch_bounds__(kPwThreads) void b_copy_out_kernel(BGroup g)
{
    const int l = g.ids[blockIdx.y], inst = g.first + l;
    const long long N = g.N;
    const double2* src = g.psi + ((long long)l * 2 + g.st[inst].cur) * 2 * N;
    double2* dst = reinterpret_cast<double2*>(g.psi_user[inst]);
    BSTRIDE(i, 2 * N) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void b_reduce_kernel(const double* partials, long long inst_stride,
                                                       long long row_stride, int nblk, const int* ids,
                                                       double* sums_first, int off)
{
    __shared__ double sh[4];
    const int m = blockIdx.x, l = ids[blockIdx.y];
    const double* row = partials + (long long)l * inst_stride + (long long)m * row_stride;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += row[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) sums_first[(long long)l * kBSumStride + off + m] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// ---------------------------------------------------------------- decisions
__device__ void state_from_hsum(const BInstParams& P, const double* S, double& E, double mu[2], double shift[2],
                                double norm2[2])
{
    const double dV = P.dV;
    const double snn[2][2] = {{S[4], S[5]}, {S[5], S[6]}};
    E = dV * S[11];
    for (int i = 0; i < 2; ++i) {
        norm2[i] = dV * S[14 + i];
        const double ek = P.Nat[i] * dV * S[i], et = P.Nat[i] * dV * S[2 + i];
        E += ek + et;
        double gdd_phi = 0.0;
        for (int j = 0; j < 2; ++j) {
            E += 0.5 * P.Nat[i] * P.G[i][j] * dV * snn[i][j] + 0.5 * P.Nat[i] * P.Gdd[i][j] * dV * S[7 + 2 * i + j];
            gdd_phi += P.Gdd[i][j] * S[7 + 2 * i + j];
        }
        mu[i] = S[12 + i] / S[14 + i];
        shift[i] = (S[12 + i] - gdd_phi) / S[14 + i];
    }
}

__device__ void geodesic_ab(BInstState& st, double alpha)
{
    for (int i = 0; i < 2; ++i) {
        if (st.pnorm[i] > 0.0) {
            const double th = alpha * st.pnorm[i];
            const double ca = cos(th), sb = sin(th) / st.pnorm[i];
            const double nrm2 = ca * ca * st.norm2[i] + sb * sb * st.pnorm[i] * st.pnorm[i] + 2.0 * ca * sb * st.psip[i];
            const double s = 1.0 / sqrt(nrm2);
            st.a[i] = ca * s;
            st.b[i] = sb * s;
        } else {
            st.a[i] = 1.0 / sqrt(st.norm2[i]);
            st.b[i] = 0.0;
        }
    }
}

__global__ void b_decide_init_kernel(int n, const BInstParams* ip, BInstState* st, const double* sums, int* act_dir,
                                     int* act_trial, int* tsel)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    BInstState& S = st[i];
    const double* R = sums + (long long)i * kBSumStride;
    S.status = kBRunning;
    S.phase = kBInit;
    S.cur = 0;
    S.iter = S.have_prev = S.level = S.path = S.nbt = S.n_restarts = S.n_backtracks = S.rounds = 0;
    S.stall_it = 0;
    S.zlevel = 0;
    S.stall_ref = __builtin_inf();
    S.E_prev = __builtin_nan("");
    S.alpha_prev = S.rz_old = 0.0;
    const double n0 = ip[i].dV * R[kSR + 0], n1 = ip[i].dV * R[kSR + 1];
    act_dir[i] = 0;
    if (!(n0 > 0.0) || !(n1 > 0.0) || !isfinite(n0) || !isfinite(n1)) {
        S.status = kBNonFinite;
        act_trial[i] = 0;
        return;
    }
    S.a[0] = 1.0 / sqrt(n0);
    S.a[1] = 1.0 / sqrt(n1);
    S.b[0] = S.b[1] = 0.0;
    act_trial[i] = 1;
    tsel[i] = 1;
}

__global__ void b_decide_dir_kernel(int n, BOpts o, const BInstParams* ip, BInstState* st, const double* sums,
                                    int* act_dir)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    BInstState& S = st[i];
    act_dir[i] = 0;
    if (S.status != kBRunning) return;
    const BInstParams& P = ip[i];
    const double dV = P.dV;
    ++S.rounds;
    if (S.phase == kBNewDir) {
        const double* R = sums + (long long)i * kBSumStride + kSR;
        S.res[0] = sqrt(dV * R[0]);
        S.res[1] = sqrt(dV * R[6]);
        const double res_max = fmax(S.res[0], S.res[1]);
        if (!isfinite(res_max) || !isfinite(S.E)) { S.status = kBNonFinite; return; }
        if (res_max < o.tol_grad) { S.status = kBConverged; return; }
        if (o.tol_dE > 0.0 && S.iter > 0 && fabs(S.E - S.E_prev) < o.tol_dE) { S.status = kBConverged; return; }
        if (res_max < 0.5 * S.stall_ref) {     // the stall rule of bec_opts.stall_window
            S.stall_ref = res_max;
            S.stall_it = S.iter;
        } else if (o.stall_window > 0 && S.iter - S.stall_it >= o.stall_window) {
            S.status = kBStalled;
            return;
        }
        if (S.iter >= o.max_iter) { S.status = kBNotConv; return; }
        // a fallback z (S.zlevel > 0) is a restart: beta = 0
        const bool fallback = S.zlevel > 0;
        const bool restart = fallback || !S.have_prev || o.beta_mode == 2 ||
                             (o.restart_period > 0 && S.iter % o.restart_period == 0);
        double beta = 0.0;
        if (!restart) {
            double num = 0.0, den = 0.0;
            for (int c = 0; c < 2; ++c) {
                num += P.Ntot_w[c] * dV * R[6 * c + 1];
                den += P.Ntot_w[c] * dV * R[6 * c + 2];
            }
            if (o.beta_mode == 1) den = S.rz_old;
            beta = (den > 0.0 && isfinite(den) && isfinite(num)) ? num / den : 0.0;
            if (beta < 0.0) beta = 0.0;
        }
        S.level = fallback ? S.zlevel : (beta > 0.0 ? 0 : 1);
        if (!fallback) S.path = 0;
        S.nbt = 0;
        for (int c = 0; c < 2; ++c) {
            S.zpsi[c] = R[6 * c + 3];
            S.ppsi[c] = R[6 * c + 4];
            S.rz[c] = R[6 * c + 5];
        }
        S.beta = S.level == 0 ? beta : 0.0;
        for (int c = 0; c < 2; ++c) S.c[c] = -dV * S.zpsi[c] + S.beta * dV * S.ppsi[c];
        act_dir[i] = 1;
    } else if (S.phase == kBRedo) {
        S.beta = 0.0;
        for (int c = 0; c < 2; ++c) S.c[c] = -dV * S.zpsi[c];
        act_dir[i] = 1;
    }
}

__global__ void b_decide_step_kernel(int n, BOpts o, const BInstParams* ip, BInstState* st, const double* sums,
                                     const int* act_dir, int* act_trial, int* tsel)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    BInstState& S = st[i];
    act_trial[i] = 0;
    if (S.status != kBRunning) return;
    const BInstParams& P = ip[i];
    const double dV = P.dV;
    const double* Sm = sums + (long long)i * kBSumStride;
    if (act_dir[i]) {
        const double* D = Sm + kSW;
        const double* LS = Sm + kSL;
        double rp = 0.0, E1 = 0.0, E2 = 0.0;
        for (int c = 0; c < 2; ++c) {
            S.pnorm[c] = sqrt(dV * D[c]);
            S.psip[c] = dV * D[16 + c];
            rp += 2.0 * P.Nat[c] * dV * D[2 + c];
            E1 += 2.0 * P.Nat[c] * dV * D[4 + c];                     // E'_i
        }
        for (int c = 0; c < 2; ++c) {
            const double pTp = dV * Sm[kSP + c] * P.inv_npts;          // <p_i, T p_i> by Parseval
            const double pn2 = S.pnorm[c] * S.pnorm[c];
            E2 += 2.0 * P.Nat[c] * (pTp + dV * D[8 + c] - pn2 * dV * D[6 + c]);
            for (int j = 0; j < 2; ++j) {
                const double rr = (c == 0 && j == 0) ? LS[0] : (c == 1 && j == 1) ? LS[2] : LS[1];
                E2 += 4.0 * P.Nat[c] * dV * (P.G[c][j] * rr + P.Gdd[c][j] * LS[3 + 2 * c + j]);
            }
            if (P.lhy_on) E2 += 2.0 * P.Nat[c] * dV * (D[10 + c] - pn2 * D[12 + c]);
        }
        if (P.lhy_on) {
            E1 += P.K3 * dV * D[14];
            E2 += 2.0 * P.K3 * dV * D[15];
        }
        S.rp = rp;
        S.E1 = E1;
        S.E2 = E2;
        if (!(rp < 0.0 && isfinite(rp))) {
            // not a descent direction: beta = 0; then, for the composite family
            // (pc >= 3), z = P_V^-1 r and z = r, each with a new direction reduce
            if (S.level == 0) {
                S.level = 1;
                S.n_restarts++;
                S.phase = kBRedo;
            } else if (S.level == 1 && o.pc >= 3) {
                S.zlevel = 2;
                S.path |= 4;
                S.phase = kBNewDir;
            } else if (S.level == 2) {
                S.zlevel = 3;
                S.phase = kBNewDir;
            } else {
                S.status = kBStagnated;
            }
            return;
        }
        S.rz_now = P.Ntot_w[0] * dV * S.rz[0] + P.Ntot_w[1] * dV * S.rz[1];
        const double pmax = fmax(S.pnorm[0], S.pnorm[1]);
        double alpha;
        if (E2 > 0.0 && isfinite(E2) && isfinite(E1) && -E1 / E2 > 0.0) alpha = -E1 / E2;
        else alpha = S.alpha_prev > 0.0 ? S.alpha_prev : 0.1 / pmax;
        if (alpha * pmax > o.theta_max) alpha = o.theta_max / pmax;
        S.alpha = alpha;
        S.nbt = 0;
        geodesic_ab(S, alpha);
        act_trial[i] = 1;
        tsel[i] = 1 - S.cur;
    } else if (S.phase == kBBacktrack) {
        S.alpha *= 0.5;
        S.nbt++;
        S.n_backtracks++;
        geodesic_ab(S, S.alpha);
        act_trial[i] = 1;
        tsel[i] = 1 - S.cur;
    }
}

__global__ void b_decide_accept_kernel(int n, BOpts o, const BInstParams* ip, BInstState* st, const double* sums,
                                       int* act_trial)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!act_trial[i]) return;
    act_trial[i] = 0;
    BInstState& S = st[i];
    const BInstParams& P = ip[i];
    const double* H = sums + (long long)i * kBSumStride + kSH;
    double Et, mu[2], shift[2], norm2[2];
    state_from_hsum(P, H, Et, mu, shift, norm2);
    const bool fin = isfinite(Et) && isfinite(mu[0]) && isfinite(mu[1]);
    bool ok;
    if (S.phase == kBInit) {
        if (!fin) { S.status = kBNonFinite; return; }
        ok = true;
    } else {
        const double tau = o.tau_rel * fabs(S.E);
        ok = fin && (S.nbt == 0 ? Et <= S.E + tau : Et <= S.E + o.armijo_c1 * S.alpha * S.E1 + tau);
    }
    if (ok) {
        if (S.phase != kBInit) {
            if (S.nbt > 0) S.path |= 1;
            S.E_prev = S.E;
            S.rz_old = S.rz_now;
            S.alpha_prev = S.alpha;
            S.have_prev = 1;
            S.iter++;
        }
        S.E = Et;
        for (int c = 0; c < 2; ++c) {
            S.mu[c] = mu[c];
            S.shift[c] = shift[c];
            S.norm2[c] = norm2[c];
        }
        for (int m = 0; m < kHevalSums; ++m) S.hsum[m] = H[m];
        S.cur = 1 - S.cur;
        S.phase = kBNewDir;
        S.nbt = 0;
        S.zlevel = 0;
    } else if (S.nbt < o.max_backtrack) {
        S.phase = kBBacktrack;
    } else if (S.level == 0) {
        S.level = 1;
        S.n_restarts++;
        S.path |= 2;
        S.phase = kBRedo;
    } else {
        S.status = kBStagnated;
    }
}

dim3 bgrid(const BGroup& g) { return dim3((unsigned)g.nblk, (unsigned)g.n_ids); }
dim3 dgrid(int n) { return dim3((unsigned)((n + 63) / 64)); }

}  // namespace

hipError_t launch_b_norm2(const BGroup& g, hipStream_t s)
{
    hipLaunchKernelGGL(b_norm2_kernel, bgrid(g), dim3(kPwThreads), 0, s, g);
    return hipGetLastError();
}
hipError_t launch_b_heval_epi(const BGroup& g, hipStream_t s)
{
    hipLaunchKernelGGL(b_heval_epi_kernel, bgrid(g), dim3(kPwThreads), 0, s, g);
    return hipGetLastError();
}
hipError_t launch_b_dir_reduce(const BGroup& g, hipStream_t s)
{
    hipLaunchKernelGGL(b_dir_reduce_kernel, bgrid(g), dim3(kPwThreads), 0, s, g);
    return hipGetLastError();
}
hipError_t launch_b_mark_pre(int n_inst, const BInstState* st, int* act_pre, hipStream_t s)
{
    hipLaunchKernelGGL(b_mark_pre_kernel, dgrid(n_inst), dim3(64), 0, s, n_inst, st, act_pre);
    return hipGetLastError();
}

hipError_t launch_b_make_r(const BGroup& g, hipStream_t s)
{
    hipLaunchKernelGGL(b_make_r_kernel, bgrid(g), dim3(kPwThreads), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_b_dir_write(const BGroup& g, hipStream_t s)
{
    hipLaunchKernelGGL(b_dir_write_kernel, bgrid(g), dim3(kPwThreads), 0, s, g);
    return hipGetLastError();
}
hipError_t launch_b_copy_out(const BGroup& g, hipStream_t s)
{
    hipLaunchKernelGGL(b_copy_out_kernel, bgrid(g), dim3(kPwThreads), 0, s, g);
    return hipGetLastError();
}
hipError_t launch_b_reduce(const double* partials, long long inst_stride, long long row_stride, int nblk, int M,
                           const int* ids, int n_ids, double* sums_first, int off, hipStream_t s)
{
    hipLaunchKernelGGL(b_reduce_kernel, dim3((unsigned)M, (unsigned)n_ids), dim3(256), 0, s, partials, inst_stride,
                       row_stride, nblk, ids, sums_first, off);
    return hipGetLastError();
}
hipError_t launch_b_decide_init(int n, const BInstParams* ip, BInstState* st, const double* sums, int* act_dir,
                                int* act_trial, int* tsel, hipStream_t s)
{
    hipLaunchKernelGGL(b_decide_init_kernel, dgrid(n), dim3(64), 0, s, n, ip, st, sums, act_dir, act_trial, tsel);
    return hipGetLastError();
}
hipError_t launch_b_decide_dir(int n, BOpts o, const BInstParams* ip, BInstState* st, const double* sums,
                               int* act_dir, hipStream_t s)
{
    hipLaunchKernelGGL(b_decide_dir_kernel, dgrid(n), dim3(64), 0, s, n, o, ip, st, sums, act_dir);
    return hipGetLastError();
}
hipError_t launch_b_decide_step(int n, BOpts o, const BInstParams* ip, BInstState* st, const double* sums,
                                const int* act_dir, int* act_trial, int* tsel, hipStream_t s)
{
    hipLaunchKernelGGL(b_decide_step_kernel, dgrid(n), dim3(64), 0, s, n, o, ip, st, sums, act_dir, act_trial, tsel);
    return hipGetLastError();
}
hipError_t launch_b_decide_accept(int n, BOpts o, const BInstParams* ip, BInstState* st, const double* sums,
                                  int* act_trial, hipStream_t s)
{
    hipLaunchKernelGGL(b_decide_accept_kernel, dgrid(n), dim3(64), 0, s, n, o, ip, st, sums, act_trial);
    return hipGetLastError();
}

}  // namespace bec
