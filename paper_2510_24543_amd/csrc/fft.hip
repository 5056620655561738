// Batched 3D complex128 FFT passes for gfx950.
//
// A 3D transform is three axis passes (z, y, x forward; x, y, z inverse).  One
// pass transforms every pencil along one axis, in place or out of place.  A
// workgroup owns whole pencils: it loads them once from HBM into registers,
// runs a self-sorting Stockham factorisation (radix 2/3/4/6/8/12/16 butterflies
// in registers, one LDS exchange between stages), and stores them once.
// Thread-to-element maps are chosen for coalescing: along the contiguous z
// axis consecutive lanes read consecutive elements of a pencil; along the
// strided y and x axes consecutive lanes take consecutive pencils, so each
// load instruction reads whole 16-byte columns side by side.
//
// The x pass (last forward axis, first inverse axis) can fuse a diagonal
// k-space operator: forward x, multiply, inverse x in registers -- the
// kinetic term |k|^2/2, the dipolar kernel Ud(k), the kinetic preconditioner
// 1/(a + |k|^2/2) -- or reduce the Parseval sum of |k|^2/2 |v|^2 without a
// store.  The paper evaluates the kinetic term, the dipolar convolution and
// the kinetic preconditioner with FFTs (Sec. IV.B, Sec. VI.B).
#include "fft_core.h"

#include <algorithm>

namespace bec {
namespace {

using namespace fftcore;

// Launch kinds.  The kernel body is the same for all of them; the kind only
// names the instantiation, so that a kernel trace times the passes of the
// energy evaluation (kinetic axis terms), of the line search (Parseval axis
// sums) and the other passes separately.
struct GenericPass {};
struct EnergyPass {};     // the x pass of the energy evaluation (kinetic axis terms, dipolar multiply)
struct EnergyPassY {};    // the y pass of the energy evaluation (kinetic axis terms)
struct LineSearchPass {};

// KMODE: 0 forward plain pass (fields Plain or ParsevalAxis), 1 inverse plain pass, 2 fused pass with
// per-field ops: forward, operator, inverse (the x pass; the y pass with kinetic axis terms); its
// Plain fields are forward only.
// WLOC (strided axes only): each wavefront holds 64/T whole pencils, lanes with
// the same t on consecutive pencils (a load instruction covers 64/T adjacent
// columns per element row), so the LDS exchanges need no workgroup barrier.
// Otherwise consecutive lanes take consecutive pencils of the whole block and
// a pencil's threads span wavefronts.
template <int L, int T, int R0, int R1, int R2, int NTHR, bool CONTIG, int KMODE, typename KIND, bool WLOC>
__global__ __launch_bounds__(NTHR) void fft_pass_kernel(FftPassArgs A)
{
    static_assert(!WLOC || (T <= 64 && 64 % T == 0 && NTHR % 64 == 0), "wave-local pencils");
    using PL = Plan<L, T, R0, R1, R2, CONTIG || WLOC>;
    constexpr int E = L / T, PB = NTHR / T, PW = WLOC ? 64 / T : 1;
    constexpr int RS = WLOC ? lds_row_wave<L, PW>() : lds_row<L>();
    __shared__ double2 lds[PB * RS];
    const int f = KMODE == 2 ? A.forder[blockIdx.y] : (int)blockIdx.y;
    const int inst = A.inst_ids ? A.inst_ids[blockIdx.z] : (int)blockIdx.z;
    if (A.active && A.active[inst] == 0) return;   // uniform per block
    const long long soff = (long long)inst * A.src_stride[f] +
                           (A.src_sel ? (long long)A.src_sel[inst] * A.src_sel_stride[f] : 0);
    const long long doff = (long long)inst * A.dst_stride[f];
    const int tid = threadIdx.x;
    const int pl = CONTIG ? tid / T : (WLOC ? (tid >> 6) * PW + (tid & 63) % PW : tid % PB);
    const int t = CONTIG ? tid % T : (WLOC ? (tid & 63) / PW : tid / PB);
    const long long pg = (long long)blockIdx.x * PB + pl;
    const bool geo2 = A.S2 > 0 && f == 2;           // field 2 with its own geometry (uniform per block)
    const long long S = geo2 ? A.S2 : A.S;
    const bool valid = pg < (geo2 ? A.npencil2 : A.npencil);
    long long base = 0, s = 0;
    if (valid) {
        const long long o = pg / S;
        s = pg - o * S;
        base = o * (long long)L * S + s;
    }
    const double2* __restrict__ src = A.src[f] + soff;
    double2* __restrict__ dst = A.dst[f] + doff;
    const double2* __restrict__ tw = A.tw;
    const int op = KMODE == 2 ? A.op[f] : kOpPlain;
    double2* row = lds + pl * RS;

    double2 v[E];
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int j = t + b * T + r * (L / R0);
            v[b * R0 + r] = valid ? src[base + (long long)j * S] : make_double2(0.0, 0.0);
        }

    constexpr int RL = PL::RL;
    if (KMODE < 2) {
        PL::template fwd_like<KMODE == 0 ? -1 : +1>(v, row, t, tw);
        if (CONTIG && KMODE == 0 && A.op[f] == kOpHalfSpectra) {   // uniform per block
            // rho^_1(k) = (F(k) + conj F(-k)) / 2, rho^_2(k) = (F(k) - conj F(-k)) / (2i), k = 0..L/2,
            // F(-k) through the pencil's LDS row
#pragma unroll
            for (int b = 0; b < E / RL; ++b)
#pragma unroll
                for (int r = 0; r < RL; ++r) row[lds_pad(t + b * T + r * (L / RL))] = v[b * RL + r];
            pencil_sync<true>();
            if (valid) {
                double2* d = dst + pg * (long long)(L + 2);
                for (int k = t; k <= L / 2; k += T) {
                    const double2 fk = row[lds_pad(k)], fm = row[lds_pad(k == 0 ? 0 : L - k)];
                    d[2 * k] = make_double2(0.5 * (fk.x + fm.x), 0.5 * (fk.y - fm.y));
                    d[2 * k + 1] = make_double2(0.5 * (fk.y + fm.y), -0.5 * (fk.x - fm.x));
                }
            }
            return;
        }
        if (KMODE == 0 && A.op[f] == kOpParsevalAxis) {      // uniform per block (f = blockIdx.y)
            const double dka = A.kaxis[(A.per_inst_tab ? (long long)inst * L : 0) + 1];
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b < E / RL; ++b)
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    const int j = t + b * T + r * (L / RL);
                    const double k = kwave<L>(dka, j);
                    const double2 w = v[b * RL + r];
                    acc += 0.5 * (k * k) * (w.x * w.x + w.y * w.y);
                }
            if (!valid) acc = 0.0;
            __syncthreads();
            const double tot = block_sum<NTHR>(acc, reinterpret_cast<double*>(lds));
            if (threadIdx.x == 0)
                A.partials[((long long)inst * A.nfield + f) * A.nblk_x + blockIdx.x] = tot * A.pscale;
            return;
        }
        if (valid) {
            const double sc = A.scale;
#pragma unroll
            for (int b = 0; b < E / RL; ++b)
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    const int j = t + b * T + r * (L / RL);
                    dst[base + (long long)j * S] = sc == 1.0 ? v[b * RL + r] : cscale(v[b * RL + r], sc);
                }
        }
        return;
    }

    // fused pass: forward, then the per-field operator
    PL::template fwd_like<-1>(v, row, t, tw);
    if (op == kOpPlain) {                              // a forward-only field of a mixed pass
        if (valid) {
            const double sc = A.scale;
#pragma unroll
            for (int b = 0; b < E / RL; ++b)
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    const int j = t + b * T + r * (L / RL);
                    dst[base + (long long)j * S] = sc == 1.0 ? v[b * RL + r] : cscale(v[b * RL + r], sc);
                }
        }
        return;
    }
    if (op == kOpDipSums) {
        // the line search's model sums in k-space: this pencil holds rho^_1 (even slot) or
        // rho^_2 (odd slot) at k_z = slot / 2; the other density at the same k is on the
        // lane one up or down (pencils 2m, 2m + 1 share a wavefront, same element index)
        static_assert(!WLOC || PW >= 2, "a density pair shares a wavefront");
        constexpr int M = kLsEpiSums;
        const long long nzh = A.nz + 2;
        const int iy = (int)(s / nzh), slot = (int)(s - (long long)iy * nzh), kz = slot >> 1;
        const bool first = (slot & 1) == 0;
        const int ay = iy <= A.ny / 2 ? iy : A.ny - iy;
        const double* __restrict__ udk = A.udtab + (A.per_inst_tab ? (long long)inst * A.udsize : 0);
        double acc[M];
#pragma unroll
        for (int m = 0; m < M; ++m) acc[m] = 0.0;
#pragma unroll
        for (int b = 0; b < E / RL; ++b)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int j = t + b * T + r * (L / RL);
                const double2 a = v[b * RL + r];
                const double2 o = make_double2(__shfl_xor(a.x, 1, 64), __shfl_xor(a.y, 1, 64));
                if (valid && first) {
                    const int ax = j <= L / 2 ? j : L - j;
                    const double u = udk[((long long)ax * (A.ny / 2 + 1) + ay) * (A.nz / 2 + 1) + kz];
                    const double p11 = a.x * a.x + a.y * a.y, p12 = a.x * o.x + a.y * o.y;
                    const double p22 = o.x * o.x + o.y * o.y;
                    acc[0] += p11;
                    acc[1] += p12;
                    acc[2] += p22;
                    acc[3] += u * p11;
                    acc[4] += u * p12;
                    acc[6] += u * p22;
                }
            }
        const double wt = ((kz == 0 || 2 * kz == A.nz) ? 1.0 : 2.0) * A.inv_n;
#pragma unroll
        for (int m = 0; m < M; ++m) acc[m] *= wt;
        acc[5] = acc[4];                               // sum rho_2 (U * rho_1) = sum rho_1 (U * rho_2)
        // fixed-order block reduction of the M sums into ls_partials [m][block]
        double* sh = reinterpret_cast<double*>(lds);
        const int lane = tid & 63, w = tid >> 6;
        __syncthreads();
        wave_sum_down(acc);
        if (lane == 0)
#pragma unroll
            for (int m = 0; m < M; ++m) sh[m * (NTHR / 64) + w] = acc[m];
        __syncthreads();
        if (tid < M) {
            double sum = 0.0;
            for (int k = 0; k < NTHR / 64; ++k) sum += sh[tid * (NTHR / 64) + k];
            A.ls_partials[((long long)inst * M + tid) * gridDim.x + blockIdx.x] = sum;
        }
        return;
    }
    const double dkx = A.kx[(A.per_inst_tab ? (long long)inst * A.nx : 0) + 1];
    const double dka = A.kaxis ? A.kaxis[(A.per_inst_tab ? (long long)inst * L : 0) + 1] : 0.0;
    const double* __restrict__ udt = A.udtab + (A.per_inst_tab ? (long long)inst * A.udsize : 0);
    double ky2 = 0.0, kz2 = 0.0;
    int ay = 0, az = 0;
    {
        const int iy = (int)(s / A.nz), iz = (int)(s - (long long)iy * A.nz);
        const double ky = A.ky[iy + (A.per_inst_tab ? (long long)inst * A.ny : 0)];
        const double kz = A.kz[iz + (A.per_inst_tab ? (long long)inst * A.nz : 0)];
        ky2 = ky * ky;
        kz2 = kz * kz;
        ay = iy <= A.ny / 2 ? iy : A.ny - iy;
        az = iz <= A.nz / 2 ? iz : A.nz - iz;
    }
    if (op == kOpParseval || op == kOpExpKin || op == kOpParsevalAxis) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < E / RL; ++b)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int j = t + b * T + r * (L / RL);
                const double kx = kwave<L>(op == kOpParsevalAxis ? dka : dkx, j);
                const double2 w = v[b * RL + r];
                const double kk = op == kOpParsevalAxis ? kx * kx : kx * kx + ky2 + kz2;
                acc += 0.5 * kk * (w.x * w.x + w.y * w.y);
            }
        if (!valid) acc = 0.0;
        __syncthreads();
        const double tot = block_sum<NTHR>(acc, reinterpret_cast<double*>(lds));
        if (threadIdx.x == 0)
            A.partials[((long long)inst * A.nfield + f) * A.nblk_x + blockIdx.x] =
                op == kOpParsevalAxis ? tot * A.pscale : tot;
        if (op == kOpParseval || op == kOpParsevalAxis) return;
        __syncthreads();                               // lds is reused by the inverse transform
    }
    const double inv_n = A.inv_n;
    double pa = A.prec_a[f];
    if (A.prec_state && op == kOpMulPrec && f < 2) {   // shift decided from device sums
        double mu[2], sh[2];
        rule_mu_shift(A.prec_state, A.prec_Gdd, mu, sh);
        pa = (sh[f] < 0.0 ? 0.0 : sh[f]) + A.prec_sigma;
    }
    if (A.prec_bst && op == kOpMulPrec && f < 2) {     // batched: the instance's shift
        const double sh = A.prec_bst[inst].shift[f];
        pa = (sh < 0.0 ? 0.0 : sh) + A.prec_sigma;
    }
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int j = t + b * T + r * (L / RL);
            double m;
            if (op == kOpMulKin) {
                const double kx = kwave<L>(dkx, j);
                m = 0.5 * (kx * kx + ky2 + kz2);
            } else if (op == kOpExpKin) {
                const double kx = kwave<L>(dkx, j);
                m = exp(-pa * 0.5 * (kx * kx + ky2 + kz2));
            } else if (op == kOpMulDip) {
                const int ax = j <= L / 2 ? j : L - j;
                m = udt[((long long)ax * (A.ny / 2 + 1) + ay) * (A.nz / 2 + 1) + az];
            } else if (op == kOpKinAxis) {
                const double k = kwave<L>(dka, j);
                m = 0.5 * (k * k);
            } else {
                const double kx = kwave<L>(dkx, j);
                m = 1.0 / (pa + 0.5 * (kx * kx + ky2 + kz2));
            }
            v[b * RL + r] = cscale(v[b * RL + r], m * (op == kOpKinAxis ? A.inv_na : inv_n));
        }
    PL::inv_rev(v, row, t, tw);
    if (valid) {
        if (op == kOpKinAxis && A.acc[f]) {
            // acc may be the destination: every value is read before it is stored, through
            // pointers without the restrict qualifier
            const double2* acc = A.acc[f] + doff;
            double2* out = A.dst[f] + doff;
            double2 q[E];
#pragma unroll
            for (int b = 0; b < E / R0; ++b)
#pragma unroll
                for (int r = 0; r < R0; ++r) q[b * R0 + r] = acc[base + (long long)(t + b * T + r * (L / R0)) * S];
#pragma unroll
            for (int b = 0; b < E / R0; ++b)
#pragma unroll
                for (int r = 0; r < R0; ++r) {
                    const int j = t + b * T + r * (L / R0);
                    const double2 o = v[b * R0 + r], a = q[b * R0 + r];
                    out[base + (long long)j * S] = make_double2(o.x + a.x, o.y + a.y);
                }
            return;
        }
#pragma unroll
        for (int b = 0; b < E / R0; ++b)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int j = t + b * T + r * (L / R0);
                dst[base + (long long)j * S] = v[b * R0 + r];
            }
    }
}

// T_z of one component held in registers after its forward z transform: times
// k_z^2/2 / n_z, inverse z transform, stored in natural order.
template <int L, int T, int R0, int R1, int R2>
__device__ __forceinline__ void kin_z_store(double2* w, double2* row, int t, const FftPassArgs& A, double2* d,
                                            long long base, bool valid)
{
    using PL = Plan<L, T, R0, R1, R2, true>;
    constexpr int E = L / T, RL = PL::RL;
    const double dk = A.kaxis[1];
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const double k = kwave<L>(dk, t + b * T + r * (L / RL));
            w[b * RL + r] = cscale(w[b * RL + r], 0.5 * (k * k) * A.inv_na);
        }
    PL::inv_rev(w, row, t, A.tw);
    if (valid) {
#pragma unroll
        for (int b = 0; b < E / R0; ++b)
#pragma unroll
            for (int r = 0; r < R0; ++r) d[base + t + b * T + r * (L / R0)] = w[b * R0 + r];
    }
}

// Forward z pass with the trial update fused into its loads (see TrialZArgs):
// all loads of both components are issued first, then the two components are
// transformed one after the other, then the packed density kept from them.
template <int L, int T, int R0, int R1, int R2, int NTHR>
__device__ __forceinline__ void trial_z_body(const FftPassArgs& A, const TrialZArgs& Z, double2* d0, double2* d1,
                                             double2* d2, double2* lds)
{
    using PL = Plan<L, T, R0, R1, R2, true>;
    constexpr int E = L / T, RS = lds_row<L>(), RL = PL::RL;
    constexpr int PB = NTHR / T;
    const int tid = threadIdx.x;
    const int pl = tid / T, t = tid % T;
    const long long pg = (long long)blockIdx.x * PB + pl;
    const bool valid = pg < A.npencil;
    const long long base = valid ? pg * (long long)L : 0;
    const long long N = Z.N;
    double2* row = lds + pl * RS;
    double2 w0[E], w1[E];
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = b * R0 + r;
            const long long j = base + t + b * T + r * (L / R0);
            w0[k] = make_double2(0.0, 0.0);
            w1[k] = make_double2(0.0, 0.0);
            if (valid) {
                const double2 x0 = Z.psi_src[j], x1 = Z.psi_src[N + j];
                w0[k] = make_double2(Z.a[0] * x0.x, Z.a[0] * x0.y);
                w1[k] = make_double2(Z.a[1] * x1.x, Z.a[1] * x1.y);
                if (Z.p) {
                    const double2 q0 = Z.p[j], q1 = Z.p[N + j];
                    w0[k].x += Z.b[0] * q0.x;
                    w0[k].y += Z.b[0] * q0.y;
                    w1[k].x += Z.b[1] * q1.x;
                    w1[k].y += Z.b[1] * q1.y;
                }
            }
        }
    double dn0[E];
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = b * R0 + r;
            const long long j = base + t + b * T + r * (L / R0);
            if (valid) {
                Z.psi_dst[j] = w0[k];
                Z.psi_dst[N + j] = w1[k];
            }
            dn0[k] = w0[k].x * w0[k].x + w0[k].y * w0[k].y;
        }
    PL::template fwd_like<-1>(w0, row, t, A.tw);
    if (Z.kin_z) {
        kin_z_store<L, T, R0, R1, R2>(w0, row, t, A, d0, base, valid);
    } else if (valid) {
#pragma unroll
        for (int b = 0; b < E / RL; ++b)
#pragma unroll
            for (int r = 0; r < RL; ++r) d0[base + t + b * T + r * (L / RL)] = w0[b * RL + r];
    }
    // w0 is free now: it takes the packed density of the loaded points
#pragma unroll
    for (int k = 0; k < E; ++k) w0[k] = make_double2(dn0[k], w1[k].x * w1[k].x + w1[k].y * w1[k].y);
    PL::template fwd_like<-1>(w1, row, t, A.tw);
    if (Z.kin_z) {
        kin_z_store<L, T, R0, R1, R2>(w1, row, t, A, d1, base, valid);
    } else if (valid) {
#pragma unroll
        for (int b = 0; b < E / RL; ++b)
#pragma unroll
            for (int r = 0; r < RL; ++r) d1[base + t + b * T + r * (L / RL)] = w1[b * RL + r];
    }
    PL::template fwd_like<-1>(w0, row, t, A.tw);
    if (valid) {
#pragma unroll
        for (int b = 0; b < E / RL; ++b)
#pragma unroll
            for (int r = 0; r < RL; ++r) d2[base + t + b * T + r * (L / RL)] = w0[b * RL + r];
    }
}

// Inverse z pass of the packed density rho_1 + i rho_2 of the line search with
// the model epilogue: K*rho stays in registers; per block the sums
// rho_i rho_j (11, 12, 22) and rho_i (K*rho)_j (11, 12, 21, 22).

template <int L, int T, int R0, int R1, int R2, int NTHR>
__global__ __launch_bounds__(NTHR) void fft_trial_z_kernel(FftPassArgs A, TrialZArgs Z)
{
    __shared__ double2 lds[(NTHR / T) * lds_row<L>()];
    if (Z.coef) {   // coefficients decided on the device by the step kernel
        Z.a[0] = Z.coef[0];
        Z.a[1] = Z.coef[1];
        Z.b[0] = Z.coef[2];
        Z.b[1] = Z.coef[3];
    }
    if (Z.norm_sums) {   // normalisation from the previous step's device sums (the host's formula)
        Z.a[0] = 1.0 / sqrt(Z.norm_dV * Z.norm_sums[0]);
        Z.a[1] = 1.0 / sqrt(Z.norm_dV * Z.norm_sums[1]);
        Z.b[0] = Z.b[1] = 0.0;
    }
    trial_z_body<L, T, R0, R1, R2, NTHR>(A, Z, A.dst[0], A.dst[1], A.dst[2], lds);
}

// The same for every running instance of a batch group (grid.z = instance):
// the trial point of instance l from its current state and search direction
// (or the caller's field on its first evaluation), transformed into its slice
// of the group's work fields.
template <int L, int T, int R0, int R1, int R2, int NTHR>
__global__ __launch_bounds__(NTHR) void fft_btrial_z_kernel(FftPassArgs A, BGroup g)
{
    __shared__ double2 lds[(NTHR / T) * lds_row<L>()];
    const int l = g.ids[blockIdx.z], inst = g.first + l;
    if (!g.act_trial[inst]) return;                 // uniform per block
    const BInstState& S = g.st[inst];
    const long long N = g.N;
    const bool init = S.phase == kBInit;
    TrialZArgs Z;
    Z.psi_src = init ? reinterpret_cast<const double2*>(g.psi_user[inst]) : g.psi + ((long long)l * 2 + S.cur) * 2 * N;
    Z.p = init ? nullptr : g.p + (long long)l * 2 * N;
    Z.a[0] = S.a[0];
    Z.a[1] = S.a[1];
    Z.b[0] = S.b[0];
    Z.b[1] = S.b[1];
    Z.coef = nullptr;
    Z.norm_sums = nullptr;
    Z.psi_dst = g.psi + ((long long)l * 2 + (1 - S.cur)) * 2 * N;
    Z.N = N;
    Z.kin_z = 0;
    double2* w = g.W + (long long)l * 3 * N;
    trial_z_body<L, T, R0, R1, R2, NTHR>(A, Z, w, w + N, w + 2 * N, lds);
}

template <int L, int T, int R0, int R1, int R2, int NTHR, bool WLOC>
hipError_t launch_cfg(bool contiguous, const FftPassArgs& A0, hipStream_t st)
{
    FftPassArgs A = A0;
    {   // fused passes: the fields with an inverse transform dispatched first
        int k = 0;
        for (int pass = 0; pass < 2; ++pass)
            for (int f = 0; f < A.nfield; ++f) {
                const bool light = A.op[f] == kOpPlain || A.op[f] == kOpParseval || A.op[f] == kOpParsevalAxis;
                if (light == (pass == 1)) A.forder[k++] = f;
            }
    }
    constexpr int PB = NTHR / T;
    const long long np = A.S2 > 0 && A.nfield > 2 ? std::max(A.npencil, A.npencil2) : A.npencil;
    dim3 grid((unsigned)((np + PB - 1) / PB), (unsigned)A.nfield, (unsigned)(A.n_inst > 0 ? A.n_inst : 1));
    // plain: every field Plain or ParsevalAxis (a one-axis pass; ParsevalAxis
    // fields only in a forward pass); otherwise the fused pass (mode 2)
    bool plain = true, axis_sums = false, kin = false, halfs = false;
    for (int f = 0; f < A.nfield; ++f) {
        plain = plain && (A.op[f] == kOpPlain || A.op[f] == kOpParsevalAxis || A.op[f] == kOpHalfSpectra);
        axis_sums = axis_sums || A.op[f] == kOpParsevalAxis;
        kin = kin || A.op[f] == kOpKinAxis;
        halfs = halfs || A.op[f] == kOpHalfSpectra;
    }
    if (plain && axis_sums && A.sign >= 0) return hipErrorInvalidValue;
    if (halfs && (!contiguous || A.sign >= 0)) return hipErrorInvalidValue;   // a forward z pass only
#define BEC_LAUNCH_PASS(C, K, KIND) \
    hipLaunchKernelGGL((fft_pass_kernel<L, T, R0, R1, R2, NTHR, C, K, KIND, (C) ? false : WLOC>), grid, dim3(NTHR), 0, st, A)
    if (contiguous) {
        // the contiguous (z) axis never runs the fused mode
        if (!plain) return hipErrorInvalidValue;
        if (A.sign >= 0) BEC_LAUNCH_PASS(true, 1, GenericPass);
        else if (axis_sums) BEC_LAUNCH_PASS(true, 0, LineSearchPass);
        else BEC_LAUNCH_PASS(true, 0, GenericPass);
    } else if (plain) {
        if (A.sign >= 0) BEC_LAUNCH_PASS(false, 1, GenericPass);
        else if (axis_sums) BEC_LAUNCH_PASS(false, 0, LineSearchPass);
        else BEC_LAUNCH_PASS(false, 0, GenericPass);
    } else if (kin) {
        if (A.npencil == A.S) BEC_LAUNCH_PASS(false, 2, EnergyPass);     // x: the pencils are the (y, z) columns
        else BEC_LAUNCH_PASS(false, 2, EnergyPassY);
    } else if (axis_sums) {
        BEC_LAUNCH_PASS(false, 2, LineSearchPass);
    } else {
        BEC_LAUNCH_PASS(false, 2, GenericPass);
    }
#undef BEC_LAUNCH_PASS
    return hipGetLastError();
}

}  // namespace

static bool find_variant(int L, int v, Variant* out)
{
#define BEC_FIND(LL, VV, T, R0, R1, R2, NT, W)      \
    if (L == LL && v == VV) {                       \
        *out = Variant{T, R0, R1, R2, NT, W};       \
        return true;                                \
    }
    BEC_FFT_VARIANTS(BEC_FIND)
#undef BEC_FIND
    return false;
}

bool fft_supported(int L)
{
    Variant v;
    return find_variant(L, 0, &v);
}

int fft_num_variants(int L)
{
    int n = 0;
    Variant v;
    while (find_variant(L, n, &v)) ++n;
    return n;
}

int fft_blocks(int L, int variant, long long npencil)
{
    Variant v;
    if (!find_variant(L, variant, &v)) return 0;
    const int pb = v.nthr / v.T;
    return (int)((npencil + pb - 1) / pb);
}

int fft_fused_default_variant(int L)
{
    // the most threads per pencil that still keep a pencil inside one wavefront
    // (fewest elements per thread: the fused kernels hold three fields), in
    // 256-thread blocks where there is a choice
    int best = 0, bestT = 0, bestN = 0;
    Variant v;
    for (int k = 0; find_variant(L, k, &v); ++k) {
        if (v.T > 64 || 64 % v.T != 0) continue;
        const bool better = v.T > bestT || (v.T == bestT && v.nthr == 256 && bestN != 256);
        if (better) {
            best = k;
            bestT = v.T;
            bestN = v.nthr;
        }
    }
    return best;
}

int fft_max_blocks(int L, long long npencil)
{
    int m = 0;
    for (int k = 0; k < fft_num_variants(L); ++k) m = std::max(m, fft_blocks(L, k, npencil));
    return m;
}

hipError_t fft_trial_z_pass(int L, int variant, const FftPassArgs& A, const TrialZArgs& Z, hipStream_t st)
{
    if (A.S != 1) return hipErrorInvalidValue;
#define BEC_TCASE(LL, VV, T, R0, R1, R2, NT, W)                                                          \
    if (L == LL && variant == VV) {                                                                      \
        const dim3 grid((unsigned)((A.npencil + NT / T - 1) / (NT / T)));                                \
        hipLaunchKernelGGL((fft_trial_z_kernel<LL, T, R0, R1, R2, NT>), grid, dim3(NT), 0, st, A, Z);    \
        return hipGetLastError();                                                                        \
    }
    BEC_FFT_VARIANTS(BEC_TCASE)
#undef BEC_TCASE
    return hipErrorInvalidValue;
}

hipError_t fft_btrial_z_pass(int L, int variant, const FftPassArgs& A, const BGroup& g, hipStream_t st)
{
    if (A.S != 1) return hipErrorInvalidValue;
#define BEC_BCASE(LL, VV, T, R0, R1, R2, NT, W)                                                           \
    if (L == LL && variant == VV) {                                                                       \
        const dim3 grid((unsigned)((A.npencil + NT / T - 1) / (NT / T)), 1u, (unsigned)g.n_ids);          \
        hipLaunchKernelGGL((fft_btrial_z_kernel<LL, T, R0, R1, R2, NT>), grid, dim3(NT), 0, st, A, g);    \
        return hipGetLastError();                                                                         \
    }
    BEC_FFT_VARIANTS(BEC_BCASE)
#undef BEC_BCASE
    return hipErrorInvalidValue;
}

hipError_t fft_pass(int L, int variant, bool contiguous, const FftPassArgs& A, hipStream_t st)
{
#define BEC_CASE(LL, VV, T, R0, R1, R2, NT, W) \
    if (L == LL && variant == VV) return launch_cfg<LL, T, R0, R1, R2, NT, (W) != 0>(contiguous, A, st);
    BEC_FFT_VARIANTS(BEC_CASE)
#undef BEC_CASE
    return hipErrorInvalidValue;
}

}  // namespace bec
