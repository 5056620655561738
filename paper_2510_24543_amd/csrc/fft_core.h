// Building blocks of the FFT passes for gfx950, shared by the pass kernels
// (fft.hip) and the passes fused with pointwise work (fft_fused.hip): complex
// helpers, radix 2/3/4/6/8/12/16 butterflies in registers, Stockham stages with
// their LDS exchanges, the plans of one length, and the table of plan variants.
#pragma once

#include "bec_internal.h"
#include "dft_consts.h"

namespace bec {
namespace fftcore {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// v * W_R^m with W_R = exp(D 2 pi i / R); R divides 48; folds at compile time.
template <int D>
__device__ __forceinline__ double2 twmul(double2 v, int R, int m)
{
    const int idx = ((m * (48 / R)) % 48 + 48) % 48;
    if (idx == 0) return v;
    if (idx == 24) return make_double2(-v.x, -v.y);
    if (idx == 12) return D < 0 ? make_double2(v.y, -v.x) : make_double2(-v.y, v.x);
    if (idx == 36) return D < 0 ? make_double2(-v.y, v.x) : make_double2(v.y, -v.x);
    const double2 w = make_double2(kCos48[idx], D < 0 ? -kSin48[idx] : kSin48[idx]);
    return cmul(v, w);
}

template <int R, int D> struct Dft;

template <int D> struct Dft<1, D> {
    __device__ static void run(double2*) {}
};

template <int D> struct Dft<2, D> {
    __device__ static void run(double2* v)
    {
        const double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <int D> struct Dft<3, D> {
    __device__ static void run(double2* v)
    {
        const double s3 = kSin48[16];                       // sin(2 pi / 3)
        const double2 a = v[0], t = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        const double2 m = make_double2(a.x - 0.5 * t.x, a.y - 0.5 * t.y);
        const double2 isd = make_double2(-s3 * d.y, s3 * d.x);   // i sin(2pi/3) d
        v[0] = cadd(a, t);
        if (D < 0) { v[1] = csub(m, isd); v[2] = cadd(m, isd); }
        else       { v[1] = cadd(m, isd); v[2] = csub(m, isd); }
    }
};

template <int D> struct Dft<4, D> {
    __device__ static void run(double2* v)
    {
        const double2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        const double2 t2 = cadd(v[1], v[3]), d = csub(v[1], v[3]);
        const double2 t3 = D < 0 ? make_double2(d.y, -d.x) : make_double2(-d.y, d.x);
        v[0] = cadd(t0, t2);
        v[1] = cadd(t1, t3);
        v[2] = csub(t0, t2);
        v[3] = csub(t1, t3);
    }
};

// Cooley-Tukey split R = R1 R2 inside registers:
// X[k1 + R1 k2] = sum_n2 W_R2^(n2 k2) W_R^(n2 k1) sum_n1 x[n2 + R2 n1] W_R1^(n1 k1)
template <int R1, int R2, int D>
__device__ __forceinline__ void dft_split(double2* v)
{
    constexpr int R = R1 * R2;
    double2 a[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        double2 t[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[n2 + R2 * n1];
        Dft<R1, D>::run(t);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) a[n2 * R1 + k1] = twmul<D>(t[k1], R, n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        double2 t[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) t[n2] = a[n2 * R1 + k1];
        Dft<R2, D>::run(t);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    }
}

template <int D> struct Dft<6, D> {
    __device__ static void run(double2* v) { dft_split<2, 3, D>(v); }
};
template <int D> struct Dft<8, D> {
    __device__ static void run(double2* v) { dft_split<2, 4, D>(v); }
};
template <int D> struct Dft<12, D> {
    __device__ static void run(double2* v) { dft_split<4, 3, D>(v); }
};
template <int D> struct Dft<16, D> {
    __device__ static void run(double2* v) { dft_split<4, 4, D>(v); }
};

// Powers w[r] = w1^r, r = 1..R-1, of a twiddle by repeated squaring (at most
// five products deep for R = 16, a few units in the last place), so that a
// butterfly loads one twiddle instead of R - 1: the loads, not the arithmetic,
// are the scarce issue slots of these passes.  D > 0 conjugates w1.
template <int R, int D>
__device__ __forceinline__ void twiddle_powers(double2 w1, double2* w)
{
    if (D > 0) w1.y = -w1.y;
    w[1] = w1;
#pragma unroll
    for (int r = 2; r < R; ++r) w[r] = (r % 2 == 0) ? cmul(w[r / 2], w[r / 2]) : cmul(w[r - 1], w1);
}

// Stockham stage of radix R after a span NS of earlier radices.  Thread t owns
// butterflies j = t + b T; butterfly j reads X[j + r L/R] (registers
// v[b R + r]), applies W_L^(r k L/(NS R)), k = j mod NS, and a length-R DFT.
// Where NS divides T every butterfly of the thread has the same k.
template <int L, int T, int R, int NS, int D>
__device__ __forceinline__ void stage(double2* v, int t, const double2* __restrict__ tw)
{
    constexpr int E = L / T, NB = E / R;
    static_assert(E % R == 0, "radix must divide the elements per thread");
    if constexpr (NS > 1) {
        constexpr bool same_k = T % NS == 0;
        double2 w[R];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (b == 0 || !same_k) {
                const int k = (int)((unsigned)(t + b * T) % (unsigned)NS);
                twiddle_powers<R, D>(tw[k * (L / (NS * R))], w);
            }
#pragma unroll
            for (int r = 1; r < R; ++r) v[b * R + r] = cmul(v[b * R + r], w[r]);
            Dft<R, D>::run(v + b * R);
        }
    } else {
#pragma unroll
        for (int b = 0; b < NB; ++b) Dft<R, D>::run(v + b * R);
    }
}

// Wavenumber of index j on a length-L axis, k_j = dk (j < L/2 ? j : j - L), with
// dk the table's entry for j = 1 (the tables hold the same formula, rounded once
// instead of twice): computed, so the passes do not load a table entry per element.
template <int L>
__device__ __forceinline__ double kwave(double dk, int j)
{
    return dk * (double)(j < L / 2 ? j : j - L);
}

// LDS rows are padded by one element after every 8: the stride-R writes of
// the first stages (R = 4..16, with the lanes of one pencil adjacent in the
// contiguous z pass) then fall on different banks.
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 3); }
template <int L>
constexpr int lds_row() { return L + L / 8 + 1; }

// Row stride for PW pencils per wavefront side by side on the strided axes
// (lane = t PW + pencil): a 16-byte LDS access serves 8 lanes per cycle, i.e.
// 8 / PW element indices t of each of PW pencils when PW < 8.  A stride of
// 8 / PW modulo 8 (in 16-byte units) puts those lanes on distinct banks for the
// stride-R writes and unit-stride reads of the exchanges (an odd stride when
// PW >= 8, where the 8 lanes are 8 pencils at the same index).
template <int L, int PW>
constexpr int lds_row_wave()
{
    if constexpr (PW >= 8) {
        return lds_row<L>() % 2 ? lds_row<L>() : lds_row<L>() + 1;
    } else {
        constexpr int base = L + L / 8;              // > lds_pad(L - 1)
        return base + ((8 / PW - base % 8) % 8 + 8) % 8;
    }
}

// Ordering of an LDS exchange among the threads of one pencil.  WAVE: the
// pencil's threads lie in one wavefront (the contiguous z passes: consecutive
// lanes take consecutive elements of a pencil and T divides 64), whose LDS
// instructions execute in program order, so only the compiler must keep the
// writes before the reads (and the reads before the next writes); otherwise the
// pencil spans wavefronts and needs a workgroup barrier.
template <bool WAVE>
__device__ __forceinline__ void pencil_sync()
{
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
}

// Output of stage (R, NS): v[b R + r] goes to Y[(j/NS) NS R + (j mod NS) + r NS].
// The next stage (radix RN) reads X[t + b T + r L/RN].
template <int L, int T, int R, int NS, int RN, bool WAVE>
__device__ __forceinline__ void exchange(double2* v, double2* row, int t)
{
    constexpr int E = L / T;
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
        const int j = t + b * T;
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) row[lds_pad(base + r * NS)] = v[b * R + r];
    }
    pencil_sync<WAVE>();
#pragma unroll
    for (int b = 0; b < E / RN; ++b)
#pragma unroll
        for (int r = 0; r < RN; ++r) v[b * RN + r] = row[lds_pad(t + b * T + r * (L / RN))];
    pencil_sync<WAVE>();
}

// Full length-L transform of the registers, radices R0 R1 R2 (1 = absent).
// Input in stage-0 layout of R0, output in natural layout of the last radix.
template <int L, int T, int R0, int R1, int R2, int D, bool WAVE>
__device__ __forceinline__ void run_fft(double2* v, double2* row, int t, const double2* __restrict__ tw)
{
    stage<L, T, R0, 1, D>(v, t, tw);
    if constexpr (R1 > 1) {
        exchange<L, T, R0, 1, R1, WAVE>(v, row, t);
        stage<L, T, R1, R0, D>(v, t, tw);
        if constexpr (R2 > 1) {
            exchange<L, T, R1, R0, R2, WAVE>(v, row, t);
            stage<L, T, R2, R0 * R1, D>(v, t, tw);
        }
    }
}

// WAVE: see pencil_sync (true for the contiguous-axis kernels)
template <int L, int T, int R0, int R1, int R2, bool WAVE = false>
struct Plan {
    static_assert(!WAVE || (T <= 64 && 64 % T == 0), "a pencil must not straddle wavefronts");
    static constexpr int RL = R2 > 1 ? R2 : (R1 > 1 ? R1 : R0);   // last forward radix
    static constexpr int E = L / T;
    template <int D>
    __device__ static void fwd_like(double2* v, double2* row, int t, const double2* tw)
    {
        run_fft<L, T, R0, R1, R2, D, WAVE>(v, row, t, tw);
    }
    // inverse run with reversed radices: starts in the layout the forward ends in
    __device__ static void inv_rev(double2* v, double2* row, int t, const double2* tw)
    {
        if constexpr (R2 > 1) run_fft<L, T, R2, R1, R0, +1, WAVE>(v, row, t, tw);
        else if constexpr (R1 > 1) run_fft<L, T, R1, R0, 1, +1, WAVE>(v, row, t, tw);
        else run_fft<L, T, R0, 1, 1, +1, WAVE>(v, row, t, tw);
    }
};

template <int NTHR>
__device__ double block_sum(double v, double* sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NTHR / 64; ++i) r += sh[i];
    return r;
}

}  // namespace fftcore

// Plan variants per length: threads per pencil T, radices (R0, R1, R2), threads
// per workgroup, wave-local pencils on the strided axes (W, see fft_pass_kernel).
// Variant 0 is the default; the autotuner picks among them.
struct Variant {
    int T, R0, R1, R2, nthr, wloc;
};

#define BEC_FFT_VARIANTS(X)                                                                          \
    X(8, 0, 1, 8, 1, 1, 128, 0) X(8, 1, 1, 8, 1, 1, 64, 0) X(8, 2, 1, 8, 1, 1, 256, 0)               \
    X(16, 0, 4, 4, 4, 1, 256, 0) X(16, 1, 2, 8, 2, 1, 256, 0) X(16, 2, 4, 4, 4, 1, 128, 0)           \
    X(16, 3, 4, 4, 4, 1, 256, 1)                                                                     \
    X(32, 0, 4, 8, 4, 1, 256, 0) X(32, 1, 4, 4, 8, 1, 256, 0) X(32, 2, 4, 8, 4, 1, 128, 0)           \
    X(32, 3, 8, 4, 4, 2, 256, 0) X(32, 4, 4, 8, 4, 1, 256, 1)                                        \
    X(48, 0, 4, 12, 4, 1, 256, 0) X(48, 1, 4, 4, 12, 1, 256, 0) X(48, 2, 4, 12, 4, 1, 128, 0)        \
    X(48, 3, 4, 12, 4, 1, 256, 1)                                                                    \
    X(64, 0, 8, 8, 8, 1, 256, 0) X(64, 1, 4, 16, 4, 1, 256, 0) X(64, 2, 8, 8, 8, 1, 128, 0)          \
    X(64, 3, 8, 8, 8, 1, 512, 0) X(64, 4, 16, 4, 4, 4, 256, 0) X(64, 5, 16, 4, 4, 4, 128, 0)         \
    X(64, 6, 16, 4, 4, 4, 256, 1) X(64, 7, 8, 8, 8, 1, 256, 1)                                       \
    X(96, 0, 4, 12, 8, 1, 128, 0) X(96, 1, 4, 12, 8, 1, 256, 0) X(96, 2, 8, 6, 4, 4, 256, 0)         \
    X(96, 3, 8, 12, 4, 2, 256, 0) X(96, 4, 8, 6, 4, 4, 256, 1) X(96, 5, 8, 12, 4, 2, 256, 1)         \
    X(128, 0, 8, 16, 8, 1, 256, 0) X(128, 1, 8, 8, 16, 1, 256, 0) X(128, 2, 8, 16, 8, 1, 128, 0)     \
    X(128, 3, 8, 16, 8, 1, 512, 0) X(128, 4, 16, 8, 4, 4, 256, 0) X(128, 5, 16, 8, 4, 4, 512, 0)     \
    X(128, 6, 16, 8, 4, 4, 128, 0) X(128, 7, 16, 4, 4, 8, 256, 0) X(128, 8, 16, 8, 4, 4, 256, 1)     \
    X(128, 9, 16, 8, 4, 4, 128, 1) X(128, 10, 8, 16, 8, 1, 256, 1)                                   \
    X(256, 0, 16, 16, 16, 1, 256, 0) X(256, 1, 16, 16, 16, 1, 128, 0) X(256, 2, 16, 16, 16, 1, 512, 0) \
    X(256, 3, 32, 8, 8, 4, 256, 0) X(256, 4, 16, 16, 4, 4, 256, 0) X(256, 5, 32, 8, 8, 4, 512, 0)    \
    X(256, 6, 16, 16, 16, 1, 256, 1) X(256, 7, 32, 8, 8, 4, 256, 1)

}  // namespace bec
