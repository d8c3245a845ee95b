// HIP kernels of the srm3 generator for gfx950 (CDNA4, wave64).
//
//  phases      : Philox phase of every line -> unit phase factors, in two layouts
//  pair sum    : T_k = sum_{p={i,j} in P(k)} W(i_w, j_w) z_i z_j   (Section 4.3 pair term)
//  tfft        : C_k = A_pure z_k + A_pair (T_k + diagonal fix), placed at bin
//                (k_kappa, k_omega mod n_t), inverse DFT along t (Stockham, LDS)
//  xfft        : inverse DFT along x over the n_kappa live rows, real part out
#include <algorithm>
#include <cstring>
#include <string>

#include "srm3_internal.hpp"

namespace srm3 {

namespace {

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ void two_sum(T &s, T &c, T x)
{
    // Knuth's error-free transformation: s + x == snew + err exactly.
    const T snew = s + x;
    const T bp = snew - s;
    const T err = (s - (snew - bp)) + (x - bp);
    s = snew;
    c += err;
}

// Complex products of the pair sum use a 3-multiply form whose per-lane
// operand needs one add per step: with a = z_i (uniform) and b = z_j (per lane)
//     k1 = a.re (b.re + b.im),  k2 = (a.re + a.im) b.im,  k3 = (a.im - a.re) b.re
//     a b = (k1 - k2) + i (k1 + k3).
// The a operand is stored as the three values (a.re, a.re + a.im, a.im - a.re),
// formed in FP64 by the phase kernel.
template <typename T2, typename T>
__device__ __forceinline__ void b_ops(const T2 &v, T &bsum, T &bim, T &bre)
{
    bsum = v.x + v.y;
    bim = v.y;
    bre = v.x;
}

// Read-only data that does not change while a kernel runs, in the constant
// address space: uniform loads through such a pointer become scalar loads even
// where the kernel stores elsewhere earlier (the persistent loop).
// (The host pass of the compiler only parses kernel bodies; it sees plain
// pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
#else
template <typename T>
using cptr = const T *;
#endif

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p)
{
    return (cptr<T>)p;
}

// A pointer that every lane of the wave holds, taken from the first lane so
// that address arithmetic on it stays scalar.
template <typename T>
__device__ __forceinline__ T *uniform_ptr(T *p)
{
    const unsigned long long v = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(v));
    const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(v >> 32));
    return reinterpret_cast<T *>((static_cast<unsigned long long>(hi) << 32) | lo);
}

// Device memory in the global address space: loads through such a pointer are
// global (not flat) loads also where the pointer itself was read from memory.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;
#else
template <typename T>
using gptr = const T *;
#endif

template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T *p)
{
    return (gptr<T>)p;
}

// The b operand is read with buffer loads: the realization's phase rows form
// one buffer resource (uniform), the lane's column is a fixed per-lane byte
// offset and the row a uniform byte offset, so stepping along kappa costs no
// vector address arithmetic (and reads past the buffer return zero).
#if defined(__HIP_DEVICE_COMPILE__)
using brsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ brsrc make_brsrc(const void *p, unsigned bytes)
{
    // the resource lives in scalar registers (the base is wave-uniform);
    // word 3 of a gfx9 raw buffer resource: 32-bit data format, no swizzle
    return __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(const_cast<void *>(p)), static_cast<short>(0),
                                             static_cast<int>(__builtin_amdgcn_readfirstlane(bytes)), 0x00020000);
}
// (The loaded vector is copied out whole: extracting its lanes one by one has
// been folded by the compiler into a single-dword load.)
__device__ __forceinline__ float2 bload(brsrc r, unsigned voff, unsigned soff, float)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(voff), static_cast<int>(soff), 0);
    static_assert(sizeof(v) == sizeof(float2), "b64 load is two floats");
    float2 f;
    __builtin_memcpy(&f, &v, sizeof(f));
    return f;
}
__device__ __forceinline__ double2 bload(brsrc r, unsigned voff, unsigned soff, double)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, static_cast<int>(voff), static_cast<int>(soff), 0);
    static_assert(sizeof(v) == sizeof(double2), "b128 load is two doubles");
    double2 d;
    __builtin_memcpy(&d, &v, sizeof(d));
    return d;
}
__device__ __forceinline__ float bload32(brsrc r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(voff),
                                                                          static_cast<int>(soff), 0));
}
__device__ __forceinline__ double bload64(brsrc r, unsigned voff, unsigned soff)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(voff), static_cast<int>(soff), 0);
    double d;
    __builtin_memcpy(&d, &v, sizeof(d));
    return d;
}
#else
struct brsrc {
    const void *p;
};
__device__ inline brsrc make_brsrc(const void *p, unsigned) { return brsrc{p}; }
__device__ inline float2 bload(brsrc, unsigned, unsigned, float) { return float2{}; }
__device__ inline double2 bload(brsrc, unsigned, unsigned, double) { return double2{}; }
__device__ inline float bload32(brsrc, unsigned, unsigned) { return 0.0f; }
__device__ inline double bload64(brsrc, unsigned, unsigned) { return 0.0; }
#endif

// Layout of the a operand (re, re + im, im - re) of support column ic, row kk:
// FP32 keeps three kappa-contiguous planes (a block's rows load as wide scalar
// loads); FP64 interleaves the three values per row, padded to four, so that
// rows load one at a time and the scalar register window stays small.
template <typename T> struct ALayout;
template <> struct ALayout<float> {
    static constexpr int ES = 1;       // element stride between rows
    static constexpr int NS = 3;       // slots per (column, row)
    __device__ static long plane(const Geometry &g) { return static_cast<long>(g.ncw) * g.nkp; }
};
template <> struct ALayout<double> {
    static constexpr int ES = 4;
    static constexpr int NS = 4;
    __device__ static long plane(const Geometry &) { return 1; }
};

// ---------------------------------------------------------------------------
// Phase factor e^{i phi} of a 32-bit fixed-point phase u (phi = 2 pi u / 2^32)
// in FP64, shared by every kernel that draws phases: the top 8 bits select
// e^{2 pi i (u >> 24) / 256} from a 256-entry table (FP64 sincospi, built in
// LDS by each block), the low 24 bits give theta = 2 pi (u mod 2^24) / 2^32 <
// 2 pi / 256, whose cosine and sine come from their Taylor series through
// theta^6 and theta^7 (the next terms are below 1e-17), and the two factors
// are multiplied: a few ulp of FP64, for a fraction of a sincos.  The
// arithmetic is written out in fma() calls so that no call site can contract
// it differently (phases drawn by different kernels agree bitwise).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void phase_table_fill(double2 *tab)
{
    for (int m = threadIdx.x; m < 256; m += blockDim.x) {
        double sn, cs;
        sincospi(static_cast<double>(m) * (1.0 / 128.0), &sn, &cs);
        tab[m] = make_double2(cs, sn);
    }
}

__device__ __forceinline__ void phase_cs(uint32_t u, const double2 *tab, double &c, double &s)
{
    const double2 t = tab[u >> 24];
    const double th = static_cast<double>(u & 0xFFFFFFu) * 1.4629180792671596e-09;   // 2 pi / 2^32
    const double t2 = th * th;
    const double ct = fma(t2, fma(t2, fma(t2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
    const double st = th * fma(t2, fma(t2, fma(t2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), 1.0);
    // explicit fused products: every kernel that inlines this rounds alike
    c = fma(t.x, ct, -(t.y * st));
    s = fma(t.y, ct, t.x * st);
}

// Phase words.  One Philox4x32-10 call (key = the realization's seed) serves
// the four consecutive frequencies k_omega = 4 q .. 4 q + 3 of row k_kappa:
// counter (k_kappa, q, 0, 0), word k_omega - 4 q.  q = floor(k_omega / 4).
// ---------------------------------------------------------------------------
__host__ __device__ inline int floor_div4(int kw) { return (kw >= 0 ? kw : kw - 3) / 4; }

__device__ __forceinline__ void phase_words(int kk, int q, uint64_t seed, uint32_t (&w)[4])
{
    philox_words4(static_cast<uint32_t>(kk), static_cast<uint32_t>(q), 0u, 0u, seed, w);
}

// Phase factor of a line with its per-line complex factor rho_k (if any).
__device__ __forceinline__ void phase_line(uint32_t u, const double2 *ptab, const double *__restrict__ lr, long l,
                                           double &co, double &s)
{
    phase_cs(u, ptab, co, s);
    if (lr) {
        // per-line complex bicoherence factor rho_k carried by the phase factor
        const double xr = lr[2 * l], xi = lr[2 * l + 1];
        const double cr = fma(co, xr, -(s * xi)), ci = fma(co, xi, s * xr);   // fused as in phase_cs
        co = cr;
        s = ci;
    }
}

// ---------------------------------------------------------------------------
// Phases with the a operand.  A block covers a tile of 64 frequencies (16
// generator calls, aligned to multiples of 4 in k_omega) x TR rows of one
// realization.  The generator words are drawn call by call into LDS; then
// each thread takes one column and TR / 4 of its rows, writes the phase rows
// along the columns, and stages the kappa-contiguous a operand in LDS to
// write it along the rows.  TR = 16 serves plans with few rows.
// ---------------------------------------------------------------------------
template <typename T, int TR>
__global__ __launch_bounds__(256) void phase_kernel(SeedChunk seeds, const uint64_t *__restrict__ seeds_dev,
                                                    int b0, Geometry g,
                                                    typename vec<T>::v2 *__restrict__ zrow,
                                                    T *__restrict__ zcol, const double *__restrict__ lr)
{
    static_assert(TR % 16 == 0, "rows per tile");
    __shared__ T at[3][64][TR + 1];
    __shared__ __align__(16) uint32_t wt[TR][68];
    __shared__ double2 ptab[256];
    phase_table_fill(ptab);
    const int bl = blockIdx.z;
    const int b = b0 + bl;
    const int k0 = blockIdx.y * TR;
    const uint64_t seed = seeds_dev ? seeds_dev[b] : seeds.s[bl];
    // the tile's first frequency: a multiple of 4 at or below -(n_omega - 1)
    const int q0 = floor_div4(-(g.nw - 1)) + 16 * static_cast<int>(blockIdx.x);
    const int kw0 = 4 * q0;
    {
        const int gi = threadIdx.x & 15;
        const int q = q0 + gi;
        const bool live = 4 * q + 3 >= -(g.nw - 1) && 4 * q <= g.nw - 1;
#pragma unroll
        for (int i = 0; i < TR / 16; ++i) {
            const int kt = (threadIdx.x >> 4) + 16 * i;
            const int kk = k0 + kt;
            uint32_t w[4] = {0u, 0u, 0u, 0u};
            if (live && kk < g.nk) phase_words(kk, q, seed, w);
            *reinterpret_cast<uint4 *>(&wt[kt][4 * gi]) = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
    __syncthreads();   // words and phase table
    const int ct = threadIdx.x & 63;
    const int kw = kw0 + ct;
    const int c = kw + g.nw - 1;
    const int c0 = kw0 + g.nw - 1;
    const int ic0 = c0 - (g.nw - g.W);   // support column of the tile's first column
    const bool planes = zcol && ic0 + 63 >= 0 && ic0 < g.ncw;
#pragma unroll 4
    for (int i = 0; i < TR / 4; ++i) {
        const int kt = (threadIdx.x >> 6) + 4 * i;
        const int kk = k0 + kt;
        double s = 0.0, co = 0.0;   // rows past n_kappa (padding) hold zero
        if (c >= 0 && c < g.nc && kk < g.nk) {
            const long l = static_cast<long>(kk) * g.nc + c;
            phase_line(wt[kt][ct], ptab, lr, l, co, s);
            typename vec<T>::v2 v;
            v.x = static_cast<T>(co);
            v.y = static_cast<T>(s);
            zrow[static_cast<long>(b) * g.nk * g.nc + l] = v;
        }
        if (planes) {
            at[0][ct][kt] = static_cast<T>(co);
            at[1][ct][kt] = static_cast<T>(co + s);
            at[2][ct][kt] = static_cast<T>(s - co);
        }
    }
    if (!planes) return;   // zcol null: no direct-form pair sum follows
    __syncthreads();
    using L = ALayout<T>;
    const long plane = L::plane(g);
    T *zb = zcol + static_cast<long>(b) * L::NS * g.ncw * g.nkp;
    const int kt = threadIdx.x % TR;
    const int kk = k0 + kt;
#pragma unroll 4
    for (int i = 0; i < 64 * TR / 256; ++i) {
        const int ct2 = threadIdx.x / TR + (256 / TR) * i;
        const int ic = ic0 + ct2;
        if (ic < 0 || ic >= g.ncw || kk >= g.nkp) continue;
        T *zc = zb + (static_cast<long>(ic) * g.nkp + kk) * L::ES;
        if constexpr (L::NS == 4) {
            // (re, re + im), (im - re, 0): two 16-byte stores per row
            double2 *z2 = reinterpret_cast<double2 *>(zc);
            z2[0] = make_double2(at[0][ct2][kt], at[1][ct2][kt]);
            z2[1] = make_double2(at[2][ct2][kt], 0.0);
        } else {
            zc[0] = at[0][ct2][kt];
            zc[plane] = at[1][ct2][kt];
            zc[2 * plane] = at[2][ct2][kt];
        }
    }
}

// Phase rows only (no a operand: the kappa-DFT, 2-D FFT, per-pair and
// process paths).  A block takes 512 consecutive generator calls (row-major
// over (k_kappa, q)) of one realization, two per thread; their lines form one
// contiguous run of the phase rows, staged in LDS and written out along it.
constexpr int kPhaseRowCalls = 512;

template <typename T>
__global__ __launch_bounds__(256) void phase_rows_kernel(SeedChunk seeds, const uint64_t *__restrict__ seeds_dev,
                                                         int b0, Geometry g, typename vec<T>::v2 *__restrict__ zrow,
                                                         const double *__restrict__ lr)
{
    using T2 = typename vec<T>::v2;
    __shared__ T2 zl[4 * kPhaseRowCalls];
    __shared__ double2 ptab[256];
    phase_table_fill(ptab);
    __syncthreads();
    const int bl = blockIdx.y;
    const int b = b0 + bl;
    const uint64_t seed = seeds_dev ? seeds_dev[b] : seeds.s[bl];
    const int qmin = floor_div4(-(g.nw - 1)), qmax = floor_div4(g.nw - 1);
    const int ng = qmax - qmin + 1;
    const long calls = static_cast<long>(g.nk) * ng;
    const long u0 = static_cast<long>(blockIdx.x) * kPhaseRowCalls;
    const long u1 = std::min(u0 + kPhaseRowCalls, calls) - 1;
    // first and last line of the block's calls (the rows' end calls are partial)
    auto first_line = [&](long u) {
        const int kk = static_cast<int>(u / ng), q = qmin + static_cast<int>(u - static_cast<long>(kk) * ng);
        return static_cast<long>(kk) * g.nc + std::max(4 * q, -(g.nw - 1)) + g.nw - 1;
    };
    const long L0 = first_line(u0);
    const int kk1 = static_cast<int>(u1 / ng), q1 = qmin + static_cast<int>(u1 - static_cast<long>(kk1) * ng);
    const long L1 = static_cast<long>(kk1) * g.nc + std::min(4 * q1 + 3, g.nw - 1) + g.nw - 1;
#pragma unroll
    for (int i = 0; i < kPhaseRowCalls / 256; ++i) {
        const long u = u0 + threadIdx.x + 256 * i;
        if (u > u1) break;
        const int kk = static_cast<int>(u / ng);
        const int q = qmin + static_cast<int>(u - static_cast<long>(kk) * ng);
        uint32_t w[4];
        phase_words(kk, q, seed, w);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int kw = 4 * q + j;
            if (kw < -(g.nw - 1) || kw > g.nw - 1) continue;
            const long l = static_cast<long>(kk) * g.nc + kw + g.nw - 1;
            double co, s;
            phase_line(w[j], ptab, lr, l, co, s);
            T2 v;
            v.x = static_cast<T>(co);
            v.y = static_cast<T>(s);
            zl[l - L0] = v;
        }
    }
    __syncthreads();
    T2 *zb = zrow + static_cast<long>(b) * g.nk * g.nc + L0;
    for (int i = threadIdx.x; i <= L1 - L0; i += 256) zb[i] = zl[i];
}

// ---------------------------------------------------------------------------
// Pair sum.
//
// Output line k = (kk, kw).  Unordered pairs are split by kappa: pairs with
// i_kappa > j_kappa are every ordered split of the frequency with j_kappa <
// kk/2; pairs inside row kk/2 (kk even) are the ordered splits with weight 1/2
// plus, for kw even, half the self pair (added when the coefficient is
// assembled).  So
//     T_k = sum_{jk <= kk/2} f(jk) sum_{iw} W(iw, kw - iw) z[kk - jk][iw] z[jk][kw - iw],
//     f = 1 for 2 jk < kk, 1/2 for 2 jk == kk.
// A wave owns 64 consecutive output columns (one per lane) and R consecutive
// rows K0..K0+R-1.  For a fixed partner column iw the weight W(iw, kw - iw)
// does not depend on kappa, so the inner sum over jk runs on the raw phases,
//     P_r(iw) = sum_jk f(jk) z[K0 + r - jk][iw] z[jk][kw - iw],
// and the weight is applied once per partner column, T_r += W P_r.  The
// a-operand z[kk-jk][iw] is the same for all lanes (scalar registers, a
// sliding window along kappa), the b-operand z[jk][kw-iw] is per lane and
// reused over the R rows.  Complex products use the 3-multiply form above
// (a sums stored with the a planes, b.re + b.im formed per step):
//     P1 += a.re (b.re + b.im),  P2 += (a.re + a.im) b.im,  P3 += (a.im - a.re) b.re
//     re = P1 - P2,  im = P1 + P3.
// In FP32 the weighted sums are flushed every few hundred terms into an
// error-free (two-sum) accumulator.
// ---------------------------------------------------------------------------
struct PairsumArgs {
    const void *zrow;
    const void *zcol;
    const void *wtab;
    void *tout;
    Geometry g;
    int batch;
    int n_rowblocks;
    int n_ctiles;
    int n_cgroups;
    int flush_terms;
    int per_xcd;      // > 0: XCD-blocked order (see pairsum_kernel), 0: interleaved
};

constexpr int kNumXcd = 8;   // MI355X: workgroups are dealt round-robin to 8 XCDs
constexpr int kFlushTerms = 2048;

constexpr int kWavesPerBlock = 4;

// NS steps of the kappa loop starting at b-row J, fully unrolled so that the
// sliding a-window is plain register renaming.  Steps s < NFULL are at full
// weight; step s >= NFULL is triangular with t = s - NFULL (row r > 2t full,
// r == 2t half, r < 2t skipped).  On entry w0/w1/w2[r] = a-values of row
// K0 - J + r (three planes); a full bulk block (NS == R == NFULL) leaves the
// values of rows K0 - J - R + r there for the next block.  bA/bB carry b-rows
// J, J + 1 in and J + NS, J + NS + 1 out (prefetched two steps ahead).  The
// first block of a partner column (FIRST) starts the sums with its first
// step, which touches every row: all rows are full there when NFULL > 0, and
// rows r > 0 full, row 0 half when NFULL == 0.
template <typename T, int R, int NS, int NFULL, bool FIRST>
__device__ __forceinline__ void pair_block(T (&P1)[R], T (&P2)[R], T (&P3)[R], T (&w0)[R], T (&w1)[R],
                                           T (&w2)[R], typename vec<T>::v2 &bA, typename vec<T>::v2 &bB,
                                           brsrc bbuf, unsigned bvoff, unsigned brow_bytes, int J,
                                           int jk_last, cptr<T> a0_, cptr<T> a1_, cptr<T> a2_, int K0)
{
    using TB = typename vec<T>::v2;
    constexpr bool BULK = (NS == R && NFULL == R);
    // v[m] = a-values of row K0 - J - R + m, m in [0, 2R)
    T v0[2 * R], v1[2 * R], v2[2 * R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        v0[R + r] = w0[r];
        v1[R + r] = w1[r];
        v2[R + r] = w2[r];
    }
    TB bq[NS + 2];
    bq[0] = bA;
    bq[1] = bB;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int jk = J + s;
        if (BULK || s + 2 < NS)
            bq[s + 2] = bload(bbuf, bvoff, static_cast<unsigned>(min(jk + 2, jk_last)) * brow_bytes, T(0));
        T bsum, bim, bre;
        b_ops(bq[s], bsum, bim, bre);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int m = r - s + R;
            const int t = s - NFULL;
            if (s < NFULL || r > 2 * t) {
                if (FIRST && s == 0) {
                    P1[r] = v0[m] * bsum;
                    P2[r] = v1[m] * bim;
                    P3[r] = v2[m] * bre;
                } else {
                    P1[r] = fma_(v0[m], bsum, P1[r]);
                    P2[r] = fma_(v1[m], bim, P2[r]);
                    P3[r] = fma_(v2[m], bre, P3[r]);
                }
            } else if (r == 2 * t) {
                const T h = T(0.5);
                if (FIRST && s == 0) {
                    P1[r] = v0[m] * (h * bsum);
                    P2[r] = v1[m] * (h * bim);
                    P3[r] = v2[m] * (h * bre);
                } else {
                    P1[r] = fma_(v0[m], h * bsum, P1[r]);
                    P2[r] = fma_(v1[m], h * bim, P2[r]);
                    P3[r] = fma_(v2[m], h * bre, P3[r]);
                }
            }
        }
        // a-values of row K0 - J - 1 - s (m = R - 1 - s), first used at step s + 1
        if (BULK || s + 1 < NS) {
            const int row = (BULK ? K0 - J - 1 - s : max(K0 - J - 1 - s, 0)) * ALayout<T>::ES;
            v0[R - 1 - s] = a0_[row];
            v1[R - 1 - s] = a1_[row];
            v2[R - 1 - s] = a2_[row];
        }
    }
    bA = bq[NS];
    bB = bq[NS + 1];
    if (BULK) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            w0[r] = v0[r];
            w1[r] = v1[r];
            w2[r] = v2[r];
        }
    }
}

// One tile of the pair sum for one realization: output rows K0 = kb*R ..
// K0+R-1 and the 64 output columns of column tile ct (one per lane).
template <typename T, int R, bool COMP>
__device__ __forceinline__ void pairsum_tile(const Geometry &g, const typename vec<T>::v2 *__restrict__ zrow_b,
                                             const T *__restrict__ zcol_b,
                                             const typename vec<T>::v2 *__restrict__ wtab,
                                             typename vec<T>::v2 *__restrict__ tout_b, int kb, int ct,
                                             int flush_terms)
{
    using T2 = typename vec<T>::v2;
    using TB = typename vec<T>::v2;
    const int lane = threadIdx.x & 63;
    const int K0 = kb * R;
    const int kc = ct * 64 + lane;
    const bool lane_ok = kc < g.nc;
    const int kw = kc - (g.nw - 1);
    const int Wm1 = g.W - 1;
    const int kw_lo = ct * 64 - (g.nw - 1);
    const int kw_hi = min(ct * 64 + 63, g.nc - 1) - (g.nw - 1);
    const int iw_lo = max(-Wm1, kw_lo - Wm1);
    const int iw_hi = min(Wm1, kw_hi + Wm1);
    const long nc = g.nc;

    using L = ALayout<T>;
    const long plane = L::plane(g);
    const unsigned brow_bytes = static_cast<unsigned>(nc * sizeof(TB));
    const brsrc bbuf = make_brsrc(zrow_b, static_cast<unsigned>(static_cast<long>(g.nk) * brow_bytes));
    const T *zcol_u = uniform_ptr(zcol_b);

    T sre[R], sim[R], cre[R], cim[R];
    T Kre[R], Kim[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        sre[r] = sim[r] = cre[r] = cim[r] = T(0);
        Kre[r] = Kim[r] = T(0);
    }

    const int nbulk = K0 / 2;
    const int jk_last = nbulk + R / 2 - 1;   // last b row used (rows < n_kappa)
    const int steps_per_ic = nbulk + R / 2;
    const int flush_every = COMP ? max(1, flush_terms / steps_per_ic) : 0x7fffffff;
    int since_flush = 0;

    for (int iw = iw_lo; iw <= iw_hi; ++iw) {
        const int jw = kw - iw;
        const bool ok = lane_ok && jw > -g.W && jw < g.W;
        T2 w;
        if (ok) {
            w = wtab[static_cast<long>(iw + Wm1) * g.ncw + (jw + Wm1)];
        } else {
            w.x = T(0);
            w.y = T(0);
        }
        const int jc = min(max(jw + g.nw - 1, 0), g.nc - 1);
        const unsigned bvoff = static_cast<unsigned>(jc) * static_cast<unsigned>(sizeof(TB));
        const cptr<T> a0_ = as_const(zcol_u) + static_cast<long>(iw + Wm1) * g.nkp * L::ES;
        const cptr<T> a1_ = a0_ + plane;
        const cptr<T> a2_ = a0_ + 2 * plane;

        // a-window: (w0, w1, w2)[r] = (re, re + im, im - re) of z[K0 + r][iw]
        T w0[R], w1[R], w2[R];
        T P1[R], P2[R], P3[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            w0[r] = a0_[(K0 + r) * L::ES];
            w1[r] = a1_[(K0 + r) * L::ES];
            w2[r] = a2_[(K0 + r) * L::ES];
        }
        TB bA = bload(bbuf, bvoff, 0u, T(0));
        TB bB = bload(bbuf, bvoff, static_cast<unsigned>(min(1, jk_last)) * brow_bytes, T(0));
        // bulk: nbulk = K0/2 steps in blocks of R, then R/2 full steps when
        // nbulk is an odd multiple of R/2, then the R/2 triangular steps
        const int nblk = __builtin_amdgcn_readfirstlane(nbulk / R);
        int J = 0;
#define SRM3_PAIR_BLOCK(NS_, NFULL_, FIRST_)                                                                  \
    pair_block<T, R, NS_, NFULL_, FIRST_>(P1, P2, P3, w0, w1, w2, bA, bB, bbuf, bvoff, brow_bytes, J, jk_last, \
                                          a0_, a1_, a2_, K0)
        if (nblk > 0) {
            SRM3_PAIR_BLOCK(R, R, true);
            J = R;
            if (nblk > 1) {
#pragma clang loop unroll(disable)
                do {
                    SRM3_PAIR_BLOCK(R, R, false);
                    J += R;
                } while (J < nblk * R);
            }
            if (nbulk - J > 0)
                SRM3_PAIR_BLOCK(R, R / 2, false);
            else
                SRM3_PAIR_BLOCK(R / 2, 0, false);
        } else if (nbulk > 0) {
            SRM3_PAIR_BLOCK(R, R / 2, true);
        } else {
            SRM3_PAIR_BLOCK(R / 2, 0, true);
        }
#undef SRM3_PAIR_BLOCK
        // T_r += W P_r
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const T pre = P1[r] - P2[r];
            const T pim = P1[r] + P3[r];
            Kre[r] = fma_(w.x, pre, Kre[r]);
            Kre[r] = fma_(-w.y, pim, Kre[r]);
            Kim[r] = fma_(w.x, pim, Kim[r]);
            Kim[r] = fma_(w.y, pre, Kim[r]);
        }
        if (COMP && ++since_flush >= flush_every) {
            since_flush = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                two_sum(sre[r], cre[r], Kre[r]);
                two_sum(sim[r], cim[r], Kim[r]);
                Kre[r] = Kim[r] = T(0);
            }
        }
    }

#pragma unroll
    for (int r = 0; r < R; ++r) {
        T re, im;
        if (COMP) {
            two_sum(sre[r], cre[r], Kre[r]);
            two_sum(sim[r], cim[r], Kim[r]);
            re = sre[r] + cre[r];
            im = sim[r] + cim[r];
        } else {
            re = Kre[r];
            im = Kim[r];
        }
        const int kk = K0 + r;
        if (lane_ok && kk < g.nk) {
            T2 v;
            v.x = re;
            v.y = im;
            tout_b[static_cast<long>(kk) * nc + kc] = v;
        }
    }
}

template <typename T, int R, bool COMP>
__global__ __launch_bounds__(256) void pairsum_kernel(PairsumArgs a)
{
    using T2 = typename vec<T>::v2;
    const Geometry &g = a.g;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    // Work item -> (realization b, row block kb, column group cg).  In the
    // XCD-blocked order each XCD (block id mod 8) walks its own contiguous
    // range of realizations, heaviest row blocks first within a realization,
    // so the z rows of the realization in flight stay in that XCD's L2.  The
    // interleaved order (small batches) walks row blocks heaviest first across
    // all realizations, spreading every row block over all XCDs.
    const int bid = blockIdx.x;
    int b, kb, cg;
    if (a.per_xcd > 0) {
        const int work = (bid % kNumXcd) * a.per_xcd + bid / kNumXcd;
        const int per_b = a.n_rowblocks * a.n_cgroups;
        if (work >= a.batch * per_b) return;
        b = work / per_b;
        const int rem = work - b * per_b;
        kb = a.n_rowblocks - 1 - rem / a.n_cgroups;
        cg = rem - (rem / a.n_cgroups) * a.n_cgroups;
    } else {
        const int per_kb = a.batch * a.n_cgroups;
        kb = a.n_rowblocks - 1 - bid / per_kb;
        const int rem = bid - (bid / per_kb) * per_kb;
        b = rem / a.n_cgroups;
        cg = rem - b * a.n_cgroups;
    }
    const int ct = cg * kWavesPerBlock + wave;
    if (ct >= a.n_ctiles) return;
    const long plane = static_cast<long>(g.ncw) * g.nkp;
    const long lines = static_cast<long>(g.nk) * g.nc;
    pairsum_tile<T, R, COMP>(g, static_cast<const typename vec<T>::v2 *>(a.zrow) + b * lines,
                             static_cast<const T *>(a.zcol) + b * ALayout<T>::NS * plane,
                             static_cast<const T2 *>(a.wtab), static_cast<T2 *>(a.tout) + b * lines, kb, ct,
                             a.flush_terms);
}

// ---------------------------------------------------------------------------
// Pair sum on the matrix cores (FP32).
//
// Grouped by the kappa split jk instead of the partner column, the sum of the
// vector kernel reads
//     T[kk][kw] = sum_jk f(kk, jk) sum_iw A_jk[kk][iw] B_jk[iw][kw],
//     A_jk[kk][iw] = z[kk - jk][iw],   B_jk[iw][kw] = W(iw, kw - iw) z[jk][kw - iw],
// with f = 1 for 2 jk < kk, 1/2 for 2 jk == kk, 0 above.  For fixed jk the iw
// sum is a dense product of a block of phase rows (A, rows kk) and a block of
// weighted phases (B) that every output row shares, so it runs as 16x16x4
// FP32 MFMAs with iw as the reduction index: one B element is formed per
// (jk, 4 partner columns, 16 output columns) and used by all the rows of the
// wave's tile.  Complex products take three real products, with A stored as
// (re, re + im, im - re) (the a planes of the phase kernel) and B as
// (re + im, im, re):
//     P1 += A_re (B_re + B_im),  P2 += (A_re + A_im) B_im,  P3 += (A_im - A_re) B_re,
//     Re T = P1 - P2,  Im T = P1 + P3.
// FP32 sums are flushed into error-free (two-sum) accumulators every few
// hundred steps; FP64 sums stay whole.  A wave owns RT x CT tiles of 16 x 16
// outputs; partner columns are stepped 4 at a time (outer loop, weights kept
// in registers), kappa splits one at a time (inner loop).  Operand layouts of
// the 16x16x4 MFMAs (lane l, i = l % 16, q = l / 16): A[i][q], B[q][i] in;
// out D[4 q + e][i] for v_mfma_f32_16x16x4_f32, D[q + 4 e][i] for
// v_mfma_f64_16x16x4_f64 (e = 0..3).
// ---------------------------------------------------------------------------

struct MfmaArgs {
    const void *zrow;   // [B][nk][nc] float2
    const void *zcol;   // [B][3][ncw][nkp] float planes (re, re + im, im - re)
    const void *wtab;   // [ncw][ncw] float2
    void *tout;         // [B][nk][nc] float2
    Geometry g;
    int batch;
    int n_rg;           // row groups of 16 RT rows
    int n_cg;           // column groups: kWavesPerBlock waves of 16 CT columns
    int per_xcd;        // > 0: XCD-blocked order, 0: interleaved
    int flush_steps;    // kappa steps between two-sum flushes
};

constexpr int kMfmaFlushSteps = 256;   // 1024 products per accumulator element
constexpr long kMfmaPrioBlocks = 16 * 256;   // launches of at least 16 blocks per CU raise the MFMA priority

// Per-precision pieces of the matrix-core pair sum: the 16x16x4 MFMA and its
// output row layout, the a
// operand layout (FP32: three kappa-contiguous planes; FP64: the three values
// of a (column, row) side by side, rows 32 bytes apart) and whether the sums
// are flushed into two-sum pairs (FP32 only).
template <typename T> struct MfmaT;
template <> struct MfmaT<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static constexpr bool COMP = true;
    static constexpr bool PLANAR = true;
    static constexpr unsigned ROW_BYTES = 4;
    __device__ static v4 mfma(float x, float y, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0); }
    __device__ static int drow(int q, int e) { return 4 * q + e; }   // output row of lane group q, element e
    __device__ static float aload(brsrc r, unsigned voff, unsigned soff) { return bload32(r, voff, soff); }
};
template <> struct MfmaT<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static constexpr bool COMP = false;
    static constexpr bool PLANAR = false;
    static constexpr unsigned ROW_BYTES = 32;
    __device__ static v4 mfma(double x, double y, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0); }
    __device__ static int drow(int q, int e) { return q + 4 * e; }   // rows interleaved (checked on the device)
    __device__ static double aload(brsrc r, unsigned voff, unsigned soff) { return bload64(r, voff, soff); }
};

// One wave's RT x CT tiles of one realization: output rows from K0 = 16 RT rg,
// columns c0 .. c0 + 16 CT - 1.  PRIO: issue each split's MFMAs at raised
// wave priority.
template <typename T, int RT, int CT, bool PRIO>
__device__ __forceinline__ void mfma_tile(const Geometry &g, const typename vec<T>::v2 *__restrict__ zrow_b,
                                          const T *__restrict__ zcol_b, const typename vec<T>::v2 *__restrict__ wtab,
                                          typename vec<T>::v2 *__restrict__ tout_b, int rg, int c0, int flush_steps)
{
    using T2 = typename vec<T>::v2;
    using M = MfmaT<T>;
    using V4 = typename M::v4;
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lq = lane >> 4;
    const int K0 = rg * 16 * RT;
    const int Wm1 = g.W - 1;
    const int kw_lo = c0 - (g.nw - 1);
    const int kw_hi = min(c0 + 16 * CT - 1, g.nc - 1) - (g.nw - 1);
    const int iw_lo = max(-Wm1, kw_lo - Wm1);
    const int iw_hi = min(Wm1, kw_hi + Wm1);
    const int kk_max = min(K0 + 16 * RT - 1, g.nk - 1);
    const int jk_end = kk_max / 2;   // last kappa split any row of the wave uses
    const int jb = K0 / 2;           // splits below jb are at full weight for every row

    const long lines = static_cast<long>(g.nk) * g.nc;
    const long plane = static_cast<long>(g.ncw) * g.nkp;
    // b rows through a buffer resource (uniform row offset, per-lane column).
    // The a planes' resource starts `shift` rows before them: per-lane offsets
    // stay fixed for a partner step and the split moves the uniform offset
    // (shift - jk rows, never negative).  Reads of rows a split does not use
    // stay inside the plan's workspace (the phase rows precede the a planes);
    // their values (not necessarily finite) are replaced by zero, skipped with
    // their tile, or land in an output row that is not stored.
    const unsigned row_bytes = static_cast<unsigned>(g.nc * sizeof(T2));
    const brsrc zb = make_brsrc(zrow_b, static_cast<unsigned>(lines * sizeof(T2)));
    const int shift = jk_end + 2;
    constexpr unsigned RS = M::ROW_BYTES;   // bytes between kappa rows of one a value
    const brsrc za = make_brsrc(reinterpret_cast<const char *>(zcol_b) - static_cast<long>(shift) * RS,
                                static_cast<unsigned>(ALayout<T>::NS * plane * sizeof(T) + (shift + 64) * RS));
    // bytes between the three a values of one (column, row)
    const unsigned plane_bytes = M::PLANAR ? static_cast<unsigned>(plane * sizeof(T)) : static_cast<unsigned>(sizeof(T));

    // FP32 flushes the MFMA sums into two-sum pairs; FP64 keeps them whole
    constexpr int NS = M::COMP ? 4 : 1;
    V4 P1[RT][CT], P2[RT][CT], P3[RT][CT];
    T sre[RT][CT][NS], cre[RT][CT][NS], sim[RT][CT][NS], cim[RT][CT][NS];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            P1[r][c] = P2[r][c] = P3[r][c] = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int e = 0; e < NS; ++e) sre[r][c][e] = cre[r][c][e] = sim[r][c][e] = cim[r][c][e] = T(0);
        }
    auto flush = [&]() {
        if constexpr (M::COMP) {
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int c = 0; c < CT; ++c) {
#pragma unroll
                    for (int e = 0; e < NS; ++e) {
                        two_sum(sre[r][c][e], cre[r][c][e], P1[r][c][e] - P2[r][c][e]);
                        two_sum(sim[r][c][e], cim[r][c][e], P1[r][c][e] + P3[r][c][e]);
                    }
                    P1[r][c] = P2[r][c] = P3[r][c] = V4{T(0), T(0), T(0), T(0)};
                }
        }
    };

    // Partner step iw0 (4 columns): the lane's a-plane byte offset (row
    // K0 + li of column ic, plane 0), its b column offsets and weights.
    auto setup = [&](int s0, unsigned &ao, unsigned (&bo)[CT], T2 (&w)[CT]) {
        const int iw = s0 + lq;
        const int ic = min(iw + Wm1, g.ncw - 1);
        ao = static_cast<unsigned>(ic * g.nkp + K0 + li) * RS;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int col = c0 + 16 * c + li;
            const int jw = col - (g.nw - 1) - iw;
            const bool ok = col < g.nc && iw <= Wm1 && jw > -g.W && jw < g.W;
            w[c].x = T(0);
            w[c].y = T(0);
            if (ok) w[c] = wtab[static_cast<long>(iw + Wm1) * g.ncw + (jw + Wm1)];
            bo[c] = ok ? static_cast<unsigned>(jw + g.nw - 1) * static_cast<unsigned>(sizeof(T2)) : 0u;
        }
    };
    // operands of split jk: b phases per column tile, a planes per row tile
    auto load_split = [&](T2 (&zs)[CT], T (&as)[RT][3], unsigned ao, const unsigned (&bo)[CT], int jk) {
#pragma unroll
        for (int c = 0; c < CT; ++c) zs[c] = bload(zb, bo[c], static_cast<unsigned>(jk) * row_bytes, T(0));
        const unsigned so = static_cast<unsigned>(shift - jk) * RS;
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const unsigned o = ao + 16u * RS * r;
            as[r][0] = M::aload(za, o, so);
            as[r][1] = M::aload(za, o + plane_bytes, so);
            as[r][2] = M::aload(za, o + 2 * plane_bytes, so);
        }
    };
    auto split = [&](int jk, bool tail, const unsigned (&bo)[CT], const T2 (&wc)[CT], const T2 (&zc)[CT],
                     const T (&ac)[RT][3]) {
        T bs[CT], bi[CT], br[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const T Br = fma_(wc[c].x, zc[c].x, -wc[c].y * zc[c].y);
            const T Bi = fma_(wc[c].x, zc[c].y, wc[c].y * zc[c].x);
            bs[c] = Br + Bi;
            bi[c] = Bi;
            br[c] = Br;
        }
        // PRIO: the split's MFMAs at raised wave priority, so that a wave that
        // reaches them issues them back to back while the other waves of the
        // SIMD do their VALU work
        if (PRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            if (tail && 2 * jk > K0 + 16 * r + 15) continue;   // no row of this tile uses the split
            T x0 = ac[r][0], x1 = ac[r][1], x2 = ac[r][2];
            if (tail) {
                // rows above the split keep their values, the split's own row
                // is halved, rows below it are replaced by zero (a select, not
                // a product: the values read there lie outside the a planes
                // and need not be finite)
                const int kk = K0 + 16 * r + li;
                const T h = 2 * jk == kk ? T(0.5) : T(1);
                const bool use = 2 * jk <= kk;
                x0 = use ? x0 * h : T(0);
                x1 = use ? x1 * h : T(0);
                x2 = use ? x2 * h : T(0);
            }
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                P1[r][c] = M::mfma(x0, bs[c], P1[r][c]);
                P2[r][c] = M::mfma(x1, bi[c], P2[r][c]);
                P3[r][c] = M::mfma(x2, br[c], P3[r][c]);
            }
        }
        if (PRIO) __builtin_amdgcn_s_setprio(0);
    };

    int since = 0;
    for (int iw0 = iw_lo; iw0 <= iw_hi; iw0 += 4) {
        unsigned ao;
        unsigned boff[CT];
        T2 wc[CT];
        setup(iw0, ao, boff, wc);
        // two operand sets: even splits in set 0, odd ones in set 1; each
        // split first requests the next split's operands (the scheduling
        // barrier keeps those loads ahead of this split's MFMAs; past the
        // last split they read unused rows)
        T2 z0[CT], z1[CT];
        T a0[RT][3], a1[RT][3];
        load_split(z0, a0, ao, boff, 0);
        auto pair = [&](int jk, bool tail, bool both) {
            load_split(z1, a1, ao, boff, jk + 1);
            __builtin_amdgcn_sched_barrier(0);
            split(jk, tail, boff, wc, z0, a0);
            if (!both) return;
            load_split(z0, a0, ao, boff, jk + 2);
            __builtin_amdgcn_sched_barrier(0);
            split(jk + 1, tail, boff, wc, z1, a1);
        };
        // jb = K0 / 2 is even: the bulk ends on a set-0 split
        int jk = 0;
        for (; jk < jb; jk += 2) pair(jk, false, true);      // every row of the wave at full weight
        for (; jk + 1 <= jk_end; jk += 2) pair(jk, true, true);
        if (jk <= jk_end) pair(jk, true, false);
        since += jk_end + 1;
        if (M::COMP && since >= flush_steps) {
            flush();
            since = 0;
        }
    }
    flush();
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int col = c0 + 16 * c + li;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int kk = K0 + 16 * r + M::drow(lq, e);
                T2 v;
                if constexpr (M::COMP) {
                    v.x = sre[r][c][e] + cre[r][c][e];
                    v.y = sim[r][c][e] + cim[r][c][e];
                } else {
                    v.x = P1[r][c][e] - P2[r][c][e];
                    v.y = P1[r][c][e] + P3[r][c][e];
                }
                if (kk < g.nk && col < g.nc) tout_b[static_cast<long>(kk) * g.nc + col] = v;
            }
        }
}

template <typename T, int RT, int CT, bool PRIO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void pairsum_mfma_kernel(MfmaArgs a)
{
    using T2 = typename vec<T>::v2;
    const Geometry &g = a.g;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int bid = blockIdx.x;
    int b, rg, cg;
    if (a.per_xcd > 0) {
        const int work = (bid % kNumXcd) * a.per_xcd + bid / kNumXcd;
        const int per_b = a.n_rg * a.n_cg;
        if (work >= a.batch * per_b) return;
        b = work / per_b;
        const int rem = work - b * per_b;
        rg = a.n_rg - 1 - rem / a.n_cg;
        cg = rem - (rem / a.n_cg) * a.n_cg;
    } else {
        const int per_rg = a.batch * a.n_cg;
        rg = a.n_rg - 1 - bid / per_rg;
        const int rem = bid - (bid / per_rg) * per_rg;
        b = rem / a.n_cg;
        cg = rem - b * a.n_cg;
    }
    const int c0 = (cg * kWavesPerBlock + wave) * 16 * CT;   // first output column of the wave
    if (c0 >= g.nc) return;
    const long lines = static_cast<long>(g.nk) * g.nc;
    const long plane = static_cast<long>(g.ncw) * g.nkp;
    mfma_tile<T, RT, CT, PRIO>(g, static_cast<const T2 *>(a.zrow) + b * lines,
                         static_cast<const T *>(a.zcol) + b * ALayout<T>::NS * plane, static_cast<const T2 *>(a.wtab),
                         static_cast<T2 *>(a.tout) + b * lines, rg, c0, a.flush_steps);
}

// Persistent pair sum over an uneven work list.  Work items (request, row
// block, column group) sit in eight queues, one per XCD, each a contiguous
// run of the cost-sorted list so that an XCD works on few requests at a time.
// A block first drains the queue of its own XCD (block id mod 8), then steals
// from the others.  The computation of an item does not depend on which block
// runs it, so results are bitwise those of the direct launch.
struct PReq {
    Geometry g;
    const void *zrow;
    const void *zcol;
    void *tsum;
    const void *wtab;
    int n_ctiles;
    int pad;
};
struct PItem {
    int req, kb, cg, pad;
};
struct PersistArgs {
    const PReq *reqs;
    const PItem *items;
    const int *q_begin;   // [kNumXcd + 1]
    int *q_next;          // [kNumXcd] counters, zero at launch
    int flush_terms;
};

template <typename T, int R, bool COMP>
__global__ __launch_bounds__(256) void pairsum_persistent(PersistArgs a)
{
    using T2 = typename vec<T>::v2;
    __shared__ int s_item;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int home = blockIdx.x % kNumXcd;
    int tries = 0;   // meaningful in thread 0 only
    for (;;) {
        if (threadIdx.x == 0) {
            int it = -1;
            while (tries < kNumXcd) {
                const int q = (home + tries) % kNumXcd;
                const int i = a.q_begin[q] + atomicAdd(&a.q_next[q], 1);
                if (i < a.q_begin[q + 1]) {
                    it = i;
                    break;
                }
                ++tries;
            }
            s_item = it;
        }
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it < 0) break;
        const PItem w = a.items[it];
        const PReq rq = a.reqs[w.req];
        const int ct = w.cg * kWavesPerBlock + wave;
        if (ct < rq.n_ctiles)
            pairsum_tile<T, R, COMP>(rq.g, static_cast<const typename vec<T>::v2 *>(rq.zrow),
                                     static_cast<const T *>(rq.zcol),
                                     static_cast<const T2 *>(rq.wtab), static_cast<T2 *>(rq.tsum), w.kb, ct,
                                     a.flush_terms);
    }
}

// The same queues with matrix-core items: (request, row group of 16 RT rows,
// column group of kWavesPerBlock x 16 CT columns).
template <typename T, int RT, int CT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void pairsum_persistent_mfma(PersistArgs a)
{
    using T2 = typename vec<T>::v2;
    __shared__ int s_item;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int home = blockIdx.x % kNumXcd;
    int tries = 0;   // meaningful in thread 0 only
    for (;;) {
        if (threadIdx.x == 0) {
            int it = -1;
            while (tries < kNumXcd) {
                const int q = (home + tries) % kNumXcd;
                const int i = a.q_begin[q] + atomicAdd(&a.q_next[q], 1);
                if (i < a.q_begin[q + 1]) {
                    it = i;
                    break;
                }
                ++tries;
            }
            s_item = it;
        }
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it < 0) break;
        const PItem w = a.items[it];
        const PReq rq = a.reqs[w.req];
        const int c0 = (w.cg * kWavesPerBlock + wave) * 16 * CT;
        if (c0 < rq.g.nc)
            mfma_tile<T, RT, CT, false>(rq.g, static_cast<const T2 *>(rq.zrow), static_cast<const T *>(rq.zcol),
                                 static_cast<const T2 *>(rq.wtab), static_cast<T2 *>(rq.tsum), w.kb, c0,
                                 kMfmaFlushSteps);
    }
}

__global__ void fill_int_kernel(int *p, int n, int v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *p, size_t n, uint32_t v)
{
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------------------
// Stockham inverse DFT in LDS (radix-4 stages, one radix-2 stage when log2 N
// is odd), for `nbatch` transforms of length N stored `ld` apart.  Every stage
// reads its inputs into registers, synchronises, then writes the permuted
// outputs (natural order at the end).  tw[n] = exp(+2 pi i n / N).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ typename vec<T>::v2 cmul(typename vec<T>::v2 a, typename vec<T>::v2 b)
{
    typename vec<T>::v2 r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = fma_(a.x, b.y, a.y * b.x);
    return r;
}

template <typename T, int MAXB>
__device__ void fft_lds(typename vec<T>::v2 *buf, int N, int ld, int nbatch,
                        const typename vec<T>::v2 *__restrict__ tw)
{
    using T2 = typename vec<T>::v2;
    const int nthr = blockDim.x, tid = threadIdx.x;
    int Ns = 1;
    const int q4 = N >> 2;
    while (Ns * 4 <= N) {
        const int total = nbatch * q4;
        const int s = N / (4 * Ns);
        T2 y[MAXB][4];
        int dst[MAXB];
#pragma unroll
        for (int i = 0; i < MAXB; ++i) {
            const int q = tid + i * nthr;
            dst[i] = -1;
            if (q < total) {
                const int f = q / q4, j = q - f * q4;
                T2 *B = buf + static_cast<long>(f) * ld;
                const int k = j & (Ns - 1);
                const T2 x0 = B[j];
                const T2 x1 = cmul<T>(B[j + q4], tw[k * s]);
                const T2 x2 = cmul<T>(B[j + 2 * q4], tw[2 * k * s]);
                const T2 x3 = cmul<T>(B[j + 3 * q4], tw[3 * k * s]);
                const T ar = x0.x + x2.x, ai = x0.y + x2.y;
                const T br = x0.x - x2.x, bi = x0.y - x2.y;
                const T cr = x1.x + x3.x, ci = x1.y + x3.y;
                const T dr = x1.x - x3.x, di = x1.y - x3.y;
                y[i][0].x = ar + cr; y[i][0].y = ai + ci;
                y[i][1].x = br - di; y[i][1].y = bi + dr;   // x0 + i x1 - x2 - i x3
                y[i][2].x = ar - cr; y[i][2].y = ai - ci;
                y[i][3].x = br + di; y[i][3].y = bi - dr;   // x0 - i x1 - x2 + i x3
                dst[i] = f * ld + (j / Ns) * 4 * Ns + k;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MAXB; ++i) {
            if (dst[i] >= 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) buf[dst[i] + r * Ns] = y[i][r];
            }
        }
        __syncthreads();
        Ns *= 4;
    }
    if (Ns < N) {   // one radix-2 stage, Ns == N / 2
        const int q2 = N >> 1;
        const int total = nbatch * q2;
        T2 y[2 * MAXB][2];
        int dst[2 * MAXB];
#pragma unroll
        for (int i = 0; i < 2 * MAXB; ++i) {
            const int q = tid + i * nthr;
            dst[i] = -1;
            if (q < total) {
                const int f = q / q2, j = q - f * q2;
                T2 *B = buf + static_cast<long>(f) * ld;
                const T2 x0 = B[j];
                const T2 x1 = cmul<T>(B[j + q2], tw[j]);
                y[i][0].x = x0.x + x1.x; y[i][0].y = x0.y + x1.y;
                y[i][1].x = x0.x - x1.x; y[i][1].y = x0.y - x1.y;
                dst[i] = f * ld + j;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 2 * MAXB; ++i) {
            if (dst[i] >= 0) {
                buf[dst[i]] = y[i][0];
                buf[dst[i] + q2] = y[i][1];
            }
        }
        __syncthreads();
    }
}

// Amplitudes of Eq. pure and the pair term, per line and realization, in
// FP64 (1 - Sigma cancels near the cap):
//   s_raw = scale * sig, rho = min(1, cap / s_raw), Sigma = rho s_raw,
//   A_pure = 2 sqrt(S dk dw (1 - Sigma)),  A_pair = 2 sqrt(S dk dw rho scale).
// `sig` is the raw (unit-scale) bicoherence sum of the line's pair set; the
// weight table holds sqrt(b2_raw), so sqrt(scale) goes into A_pair.
struct AmpArgs {
    const double *S;          // plan spectrum [nk][nc]
    const double *sig;        // unit-scale raw pair sums [nk][nc]
    const double *scale_b;    // per realization b^2 scale, or null (1)
    const double *const *S_b; // per realization spectrum, or null (plan's)
    double dkdw;
    double cap;
    int pairs;                // 0: no pair sums (zero bicoherence)
    const double *lc;         // per-line complex pair factor c_k (interleaved), or null (1)
    const double *lr;         // per-line complex factor rho_k carried by zrow (interleaved), or null (1)
    const void *tab;          // per-line (A_pure, A_pair) in T at unit scale and the plan's spectrum, or null
};

struct TfftArgs {
    Geometry g;
    int mode;             // 0: assemble from pair sums and phase rows; 1: read C; 2: zero bicoherence,
                          // the phase factors generated here (no phase rows)
    const void *cin;      // mode 1: [B][nk][nc]
    const void *zrow;     // mode 0
    const void *tsum;     // mode 0
    SeedChunk seeds;      // mode 2: seeds of realizations b0 .. b0 + 255 (or seeds_dev)
    const uint64_t *seeds_dev;
    int b0;
    AmpArgs amp;
    const void *wtab;     // [ncw][ncw]
    const void *tw;       // pass twiddles of n_t (fft_schedule)
    void *gout;           // [B][nt / xtw][nk][xtw]: t-transformed rows in tiles of xtw columns
    void *rout;           // n_x == 1 only, or null: the field itself, [B][nt] real (no x-transform)
    int xtw;              // columns per tile of gout (the x-transform's tile width, a power of two)
    FftSched sched;       // length n_t
    int np;               // rows per block (a power of two)
    int rows;             // rows of the launch (realizations x n_kappa)
};

// Coefficient of line (b, kk, c) from its pair sum, phase and amplitudes.
template <typename T>
__device__ __forceinline__ typename vec<T>::v2 assemble_line(const Geometry &g, int b, int kk, int c,
                                                             const typename vec<T>::v2 *zrow,
                                                             const typename vec<T>::v2 *tsum,
                                                             const AmpArgs &amp,
                                                             const typename vec<T>::v2 *wtab)
{
    using T2 = typename vec<T>::v2;
    const long li = static_cast<long>(kk) * g.nc + c;
    const long bi = static_cast<long>(b) * g.nk * g.nc + li;
    T2 t;
    t.x = T(0);
    t.y = T(0);
    if (amp.pairs) t = tsum[bi];
    const int kw = c - (g.nw - 1);
    if (amp.pairs == 1 && ((kk | kw) & 1) == 0) {
        const int hw = kw / 2;
        if (hw > -g.W && hw < g.W) {
            // half of the self pair {(kk/2, kw/2), (kk/2, kw/2)}
            const T2 w = wtab[static_cast<long>(hw + g.W - 1) * g.ncw + (hw + g.W - 1)];
            const T2 zh = zrow[static_cast<long>(b) * g.nk * g.nc + static_cast<long>(kk / 2) * g.nc + hw + g.nw - 1];
            const T2 z2 = cmul<T>(zh, zh);
            const T2 d = cmul<T>(w, z2);
            t.x += T(0.5) * d.x;
            t.y += T(0.5) * d.y;
        }
    }
    if (amp.tab && !amp.scale_b && !amp.S_b) {
        // the same amplitudes, evaluated once per plan
        const T2 pq = static_cast<const T2 *>(amp.tab)[li];
        const T2 z = zrow[bi];
        T2 C;
        C.x = fma_(pq.x, z.x, pq.y * t.x);
        C.y = fma_(pq.x, z.y, pq.y * t.y);
        return C;
    }
    const double *Sp = (amp.S_b && amp.S_b[b]) ? amp.S_b[b] : amp.S;
    const double sc = amp.scale_b ? amp.scale_b[b] : 1.0;
    const double sraw = sc * amp.sig[li];
    const double rho = (amp.cap > 0.0 && sraw > amp.cap) ? amp.cap / sraw : 1.0;
    const double base = Sp[li] * amp.dkdw;
    const double pd = 2.0 * sqrt(base * (1.0 - rho * sraw));
    const double qd = 2.0 * sqrt(base * rho * sc);
    const T2 z = zrow[bi];
    T2 C;
    if (!amp.lc && !amp.lr) {
        const T p = static_cast<T>(pd);
        const T q = static_cast<T>(qd);
        C.x = fma_(p, z.x, q * t.x);
        C.y = fma_(p, z.y, q * t.y);
        return C;
    }
    // complex line factors: pair part times c_k; zrow carries rho_k, which the
    // pure part divides out (its bare phase factor)
    double qr = qd, qi = 0.0, pr = pd, pi = 0.0;
    if (amp.lc) {
        qr = qd * amp.lc[2 * li];
        qi = qd * amp.lc[2 * li + 1];
    }
    if (amp.lr) {
        const double xr = amp.lr[2 * li], xi = amp.lr[2 * li + 1];
        const double m2 = xr * xr + xi * xi;
        pr = m2 > 0.0 ? pd * xr / m2 : 0.0;
        pi = m2 > 0.0 ? -pd * xi / m2 : 0.0;
    }
    const T Pr = static_cast<T>(pr), Pi = static_cast<T>(pi), Qr = static_cast<T>(qr), Qi = static_cast<T>(qi);
    C.x = Pr * z.x - Pi * z.y + Qr * t.x - Qi * t.y;
    C.y = Pr * z.y + Pi * z.x + Qr * t.y + Qi * t.x;
    return C;
}

// ---------------------------------------------------------------------------
// Register-blocked Stockham FFT (inverse, e^{+2 pi i n m / N}) of the t- and
// x-transforms (Section 4.3: the double sum as two batches of 1-D FFTs).
// Every thread holds 16 elements: the 16 / R butterflies of a radix-R pass
// (fft_schedule: radix 16, then one pass of radix 2, 4 or 8).  The first pass
// takes its inputs from a functor (computed or read from global memory, no
// LDS staging), the last hands its outputs to another (written to global
// memory), and the passes in between exchange through LDS (the transform-major
// layout padded by one element every 256 bytes against the bank conflicts of
// the first pass's stride-16 writes).  Twiddles of a pass come from the
// plan's table in global memory, indexed (r - 1) Ns + k with k running over
// the lanes.  Two layouts: transform-major (element n of transform f at
// f N + n, a transform's butterflies on consecutive lanes; the t-transform,
// whose inputs and outputs run along n) and interleaved (at n np + f, the
// transforms on consecutive lanes; the x-transform, whose inputs and outputs
// run along the transforms).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ilog2i(int x) { return __builtin_ctz(static_cast<unsigned>(x)); }

template <typename T2>
__device__ __forceinline__ void idft4(T2 &x0, T2 &x1, T2 &x2, T2 &x3)
{
    const auto ar = x0.x + x2.x, ai = x0.y + x2.y, br = x0.x - x2.x, bi = x0.y - x2.y;
    const auto cr = x1.x + x3.x, ci = x1.y + x3.y, dr = x1.x - x3.x, di = x1.y - x3.y;
    x0.x = ar + cr;
    x0.y = ai + ci;
    x2.x = ar - cr;
    x2.y = ai - ci;
    x1.x = br - di;   // (x0 - x2) + i (x1 - x3)
    x1.y = bi + dr;
    x3.x = br + di;   // (x0 - x2) - i (x1 - x3)
    x3.y = bi - dr;
}

// x * (cr + i ci)
template <typename T, typename T2>
__device__ __forceinline__ T2 cmulc(T2 x, T cr, T ci)
{
    T2 r;
    r.x = x.x * cr - x.y * ci;
    r.y = x.x * ci + x.y * cr;
    return r;
}

// In-register inverse DFT of R points; output m sits at x[idft_pos<R>(m)].
template <int R>
__device__ __forceinline__ constexpr int idft_pos(int m)
{
    return R == 16 ? 4 * (m & 3) + (m >> 2) : m;
}

template <typename T, int R>
__device__ __forceinline__ void idft(typename vec<T>::v2 (&x)[R])
{
    using T2 = typename vec<T>::v2;
    constexpr T h = T(0.70710678118654752440);    // cos(pi/4)
    constexpr T c8 = T(0.92387953251128675613);   // cos(pi/8)
    constexpr T s8 = T(0.38268343236508977173);   // sin(pi/8)
    if constexpr (R == 2) {
        const T2 a = x[0];
        x[0].x = a.x + x[1].x;
        x[0].y = a.y + x[1].y;
        x[1].x = a.x - x[1].x;
        x[1].y = a.y - x[1].y;
    } else if constexpr (R == 4) {
        idft4(x[0], x[1], x[2], x[3]);
    } else if constexpr (R == 8) {
        idft4(x[0], x[2], x[4], x[6]);   // even half: E_m at x[2m]
        idft4(x[1], x[3], x[5], x[7]);   // odd half:  O_m at x[2m + 1]
        T2 o[4];
        o[0] = x[1];
        o[1].x = (x[3].x - x[3].y) * h;   // O_1 e^{i pi/4}
        o[1].y = (x[3].x + x[3].y) * h;
        o[2].x = -x[5].y;                 // O_2 e^{i pi/2}
        o[2].y = x[5].x;
        o[3].x = -(x[7].x + x[7].y) * h;  // O_3 e^{3 i pi/4}
        o[3].y = (x[7].x - x[7].y) * h;
        T2 y[8];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            y[m].x = x[2 * m].x + o[m].x;
            y[m].y = x[2 * m].y + o[m].y;
            y[m + 4].x = x[2 * m].x - o[m].x;
            y[m + 4].y = x[2 * m].y - o[m].y;
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = y[m];
    } else {
        static_assert(R == 16, "radix 2, 4, 8 or 16");
        // n = 4 n1 + n2, m = k1 + 4 k2: four 4-point DFTs over n1, twiddles
        // e^{2 pi i n2 k1 / 16}, four 4-point DFTs over n2
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) idft4(x[n2], x[4 + n2], x[8 + n2], x[12 + n2]);
        x[5] = cmulc(x[5], c8, s8);     // k1 = 1, n2 = 1: e^{i pi/8}
        x[6] = cmulc(x[6], h, h);       //         n2 = 2: e^{i pi/4}
        x[7] = cmulc(x[7], s8, c8);     //         n2 = 3: e^{3 i pi/8}
        x[9] = cmulc(x[9], h, h);       // k1 = 2, n2 = 1: e^{i pi/4}
        {
            const T t = x[10].x;        //         n2 = 2: e^{i pi/2}
            x[10].x = -x[10].y;
            x[10].y = t;
        }
        x[11] = cmulc(x[11], -h, h);    //         n2 = 3: e^{3 i pi/4}
        x[13] = cmulc(x[13], s8, c8);   // k1 = 3, n2 = 1: e^{3 i pi/8}
        x[14] = cmulc(x[14], -h, h);    //         n2 = 2: e^{3 i pi/4}
        x[15] = cmulc(x[15], -c8, -s8); //         n2 = 3: e^{9 i pi/8}
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) idft4(x[4 * k1], x[4 * k1 + 1], x[4 * k1 + 2], x[4 * k1 + 3]);
    }
}

// LDS index of element e in the transform-major layout: one pad element every
// 256 bytes, which puts the stride-16 writes of the first pass on distinct
// banks (the interleaved layout is not padded: its lanes run along the
// transforms).
template <typename T>
__host__ __device__ constexpr int fft_lds_elems(int n)
{
    return n + (n >> (sizeof(T) == 4 ? 5 : 4)) + 1;
}

template <typename T>
__device__ __forceinline__ int lpad(int e)
{
    return e + (e >> (sizeof(T) == 4 ? 5 : 4));
}

// One radix-R pass of span Ns = 2^LG_S over np transforms of length
// N = 2^lg_n: butterfly q = threadIdx.x + i blockDim.x, i < 16 / R, reads
// elements j + r N / R of its transform, twiddles them by
// e^{2 pi i r k / (R Ns)} (k = j mod Ns), and writes output r to
// (j / Ns) R Ns + k + r Ns.
template <typename T, int R, int LG_S, bool INTER, bool FIRST, bool LAST, class In, class Out>
__device__ __forceinline__ void fft_pass(typename vec<T>::v2 *buf, int lg_n, int np, int lg_np,
                                         const typename vec<T>::v2 *__restrict__ tw, const In &in, const Out &out)
{
    using T2 = typename vec<T>::v2;
    constexpr int NB = 16 / R;
    constexpr int LR = R == 16 ? 4 : (R == 8 ? 3 : (R == 4 ? 2 : 1));
    constexpr int Ns = 1 << LG_S;
    constexpr int PS = sizeof(T) == 4 ? 5 : 4;   // pad shift
    const int lg_nb = lg_n - LR;
    const int nb = 1 << lg_nb;
    const int total = np << lg_nb;
    // transform-major reads are linear in r when N / R is a multiple of the pad period
    const bool lin = nb >= (1 << PS);
    const int pnb = nb + (nb >> PS);
    T2 x[NB][R];
    int fq[NB], jq[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int q = threadIdx.x + i * blockDim.x;
        const int f = INTER ? (q & (np - 1)) : (q >> lg_nb);
        const int j = INTER ? (q >> lg_np) : (q & (nb - 1));
        const bool valid = q < total;
        fq[i] = valid ? f : -1;
        jq[i] = j;
        if (valid) {
            if (FIRST) {
#pragma unroll
                for (int r = 0; r < R; ++r) x[i][r] = in(f, j + r * nb);
            } else {
                if (INTER) {
                    const int b0 = (j << lg_np) + f, st = nb << lg_np;
#pragma unroll
                    for (int r = 0; r < R; ++r) x[i][r] = buf[b0 + r * st];
                } else if (lin) {
                    const int b0 = lpad<T>((f << lg_n) + j);
#pragma unroll
                    for (int r = 0; r < R; ++r) x[i][r] = buf[b0 + r * pnb];
                } else {
                    const int b0 = (f << lg_n) + j;
#pragma unroll
                    for (int r = 0; r < R; ++r) x[i][r] = buf[lpad<T>(b0 + r * nb)];
                }
                if (Ns > 1) {
                    const T2 *t = tw + (j & (Ns - 1));
#pragma unroll
                    for (int r = 1; r < R; ++r) x[i][r] = cmul<T>(x[i][r], t[(r - 1) * Ns]);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                x[i][r].x = T(0);
                x[i][r].y = T(0);
            }
        }
        idft<T, R>(x[i]);
    }
    if (!FIRST) __syncthreads();   // every read of the pass before its writes
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if (fq[i] < 0) continue;
        const int f = fq[i], j = jq[i];
        const int d0 = ((j >> LG_S) << (LG_S + LR)) + (j & (Ns - 1));
        if (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) out(f, d0 + r * Ns, x[i][idft_pos<R>(r)]);
        } else if (INTER) {
            const int b0 = (d0 << lg_np) + f;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[b0 + ((r * Ns) << lg_np)] = x[i][idft_pos<R>(r)];
        } else {
            const int e0 = (f << lg_n) + d0;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[lpad<T>(e0 + r * Ns)] = x[i][idft_pos<R>(r)];
        }
    }
    if (!LAST) __syncthreads();
}

template <typename T, int LG_S, bool INTER, bool FIRST, bool LAST, class In, class Out>
__device__ __forceinline__ void fft_pass_r(int R, typename vec<T>::v2 *buf, int lg_n, int np, int lg_np,
                                           const typename vec<T>::v2 *tw, const In &in, const Out &out)
{
    switch (R) {
    case 16: fft_pass<T, 16, LG_S, INTER, FIRST, LAST>(buf, lg_n, np, lg_np, tw, in, out); break;
    case 8: fft_pass<T, 8, LG_S, INTER, FIRST, LAST>(buf, lg_n, np, lg_np, tw, in, out); break;
    case 4: fft_pass<T, 4, LG_S, INTER, FIRST, LAST>(buf, lg_n, np, lg_np, tw, in, out); break;
    default: fft_pass<T, 2, LG_S, INTER, FIRST, LAST>(buf, lg_n, np, lg_np, tw, in, out); break;
    }
}

// np transforms of length s.N (blockDim.x * 16 >= np N elements).  The pass
// spans are 1, 16, 256, 4096 (compile time): radix 16 up to the last pass.
// STAGED: the inputs are already in LDS (transform-major, padded), written by
// the caller before a barrier; the first pass reads them from there.
template <typename T, bool INTER, bool STAGED, class In, class Out>
__device__ __forceinline__ void fft_block(typename vec<T>::v2 *buf, const FftSched &s, int np,
                                          const typename vec<T>::v2 *tw, const In &in, const Out &out)
{
    if (s.npass == 0) {   // N = 1
        for (int f = threadIdx.x; f < np; f += blockDim.x) out(f, 0, STAGED ? buf[lpad<T>(f)] : in(f, 0));
        return;
    }
    const int lg_n = ilog2i(s.N), lg_np = ilog2i(np);
    const int last = s.npass - 1, RL = s.R[last];
    if (last == 0) {
        fft_pass_r<T, 0, INTER, !STAGED, true>(RL, buf, lg_n, np, lg_np, tw, in, out);
        return;
    }
    fft_pass<T, 16, 0, INTER, !STAGED, false>(buf, lg_n, np, lg_np, tw, in, out);
    if (last >= 2) fft_pass<T, 16, 4, INTER, false, false>(buf, lg_n, np, lg_np, tw + s.off[1], in, out);
    if (last >= 3) fft_pass<T, 16, 8, INTER, false, false>(buf, lg_n, np, lg_np, tw + s.off[2], in, out);
    const typename vec<T>::v2 *tl = tw + s.off[last];
    switch (last) {
    case 1: fft_pass_r<T, 4, INTER, false, true>(RL, buf, lg_n, np, lg_np, tl, in, out); break;
    case 2: fft_pass_r<T, 8, INTER, false, true>(RL, buf, lg_n, np, lg_np, tl, in, out); break;
    default: fft_pass_r<T, 12, INTER, false, true>(RL, buf, lg_n, np, lg_np, tl, in, out); break;
    }
}

template <typename T, int MODE, bool ONE_ROW>
__global__ __launch_bounds__(sizeof(T) == 8 ? 512 : 1024) void tfft_kernel(TfftArgs a)
{
    using T2 = typename vec<T>::v2;
    extern __shared__ unsigned char smem_raw[];
    T2 *buf = reinterpret_cast<T2 *>(smem_raw);
    // the functors below capture copies of the arguments they use (a
    // reference to the kernel argument itself would move it to scratch)
    const Geometry g = a.g;
    const int np = ONE_ROW ? 1 : a.np, rows = a.rows;
    const int row0 = blockIdx.x * np;   // rows b * nk + kk of the launch's chunk
    // one-row blocks assembling from pair sums run row-major over (kk, b):
    // consecutive blocks take the same wavenumber row of successive
    // realizations, so its per-line plan data (amplitudes) is read from L2.
    // The other modes run over (b, kk): consecutive blocks write adjacent rows
    // of the tile-major output (measured faster for them).
    const int nbat = rows / g.nk;
    int ku = 0, bu = 0;
    if (ONE_ROW) {
        if (MODE == 0) {
            ku = static_cast<int>(blockIdx.x) / nbat;
            bu = static_cast<int>(blockIdx.x) - ku * nbat;
        } else {
            bu = static_cast<int>(blockIdx.x) / g.nk;
            ku = static_cast<int>(blockIdx.x) - bu * g.nk;
        }
    }
    const int rowu = bu * g.nk + ku;
    // mode 2: the seeds of the block's rows (one row: a scalar; several: after the rows in LDS)
    uint64_t seed0 = 0;
    uint64_t *seed_l = reinterpret_cast<uint64_t *>(buf + fft_lds_elems<T>(np * g.nt));
    // mode 2: the phase-factor table after the rows and their seeds (16-byte aligned)
    double2 *ptab = reinterpret_cast<double2 *>(
        (reinterpret_cast<uintptr_t>(seed_l + (np > 1 ? np : 0)) + 15) & ~static_cast<uintptr_t>(15));
    if (MODE == 2) phase_table_fill(ptab);
    if (MODE == 2) {
        auto seed_of = [](const TfftArgs &x, int row, int nk) -> uint64_t {
            const int b = row / nk;
            return x.seeds_dev ? x.seeds_dev[x.b0 + b] : x.seeds.s[b];
        };
        if (ONE_ROW) {
            seed0 = a.seeds_dev ? a.seeds_dev[a.b0 + bu] : a.seeds.s[bu];
        } else {
            for (int f = threadIdx.x; f < np; f += blockDim.x)
                seed_l[f] = row0 + f < rows ? seed_of(a, row0 + f, g.nk) : 0;
        }
        __syncthreads();   // seeds and phase table
    }
    const AmpArgs amp = a.amp;
    const int lg_n = ilog2i(g.nt);
    if constexpr (MODE == 2) {
        // C = A_pure e^{i phi} of every line of the block's rows, staged in
        // LDS at its bin (k_w, or k_w + n_t below zero), one generator call
        // (four frequencies) per step; the phases are those the phase kernel
        // draws (same words, phase_cs, rounding)
        const int qmin = floor_div4(-(g.nw - 1)), qmax = floor_div4(g.nw - 1);
        const int ng = qmax - qmin + 1;
        for (int u = threadIdx.x; u < np * ng; u += blockDim.x) {
            const int f = u / ng;
            const int q = qmin + (u - f * ng);
            const int row = ONE_ROW ? rowu : row0 + f;
            const bool live = row < rows;
            int b = bu, kk = ku;
            if (!ONE_ROW) {
                b = row / g.nk;
                kk = row - b * g.nk;
            }
            uint32_t w[4] = {0u, 0u, 0u, 0u};
            if (live) phase_words(kk, q, ONE_ROW ? seed0 : seed_l[f], w);
            const double *Sp = (amp.S_b && live && amp.S_b[b]) ? amp.S_b[b] : amp.S;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int kw = 4 * q + j;
                if (kw < -(g.nw - 1) || kw > g.nw - 1) continue;
                T2 C;
                C.x = T(0);
                C.y = T(0);
                if (live) {
                    double sn, cs;
                    phase_cs(w[j], ptab, cs, sn);
                    const long li = static_cast<long>(kk) * g.nc + kw + g.nw - 1;
                    T p;
                    if (amp.tab && !amp.S_b) {
                        p = static_cast<const T2 *>(amp.tab)[li].x;
                    } else {
                        p = static_cast<T>(2.0 * sqrt(Sp[li] * amp.dkdw));
                    }
                    C.x = p * static_cast<T>(cs);
                    C.y = p * static_cast<T>(sn);
                }
                const int n = kw >= 0 ? kw : kw + g.nt;
                buf[lpad<T>((f << lg_n) + n)] = C;
            }
        }
        // the bins between the positive and the negative frequencies
        const int gap = g.nt - 2 * g.nw + 1;
        for (int u = threadIdx.x; u < np * gap; u += blockDim.x) {
            const int f = u / gap;
            T2 z;
            z.x = T(0);
            z.y = T(0);
            buf[lpad<T>((f << lg_n) + g.nw + (u - f * gap))] = z;
        }
        __syncthreads();
    }
    const T2 *zrow = static_cast<const T2 *>(a.zrow);
    const T2 *tsum = static_cast<const T2 *>(a.tsum);
    const T2 *wtab = static_cast<const T2 *>(a.wtab);
    const T2 *cin = static_cast<const T2 *>(a.cin);
    // coefficient of bin n (k_w = n, or n - n_t above the zero gap) of row row0 + f
    auto in = [=](int f, int n) -> T2 {
        T2 C;
        C.x = T(0);
        C.y = T(0);
        const int row = ONE_ROW ? rowu : row0 + f;
        int kw = n;
        if (n >= g.nw) {
            if (n <= g.nt - g.nw || row >= rows) return C;
            kw = n - g.nt;
        } else if (row >= rows) {
            return C;
        }
        int b = bu, kk = ku;
        if (!ONE_ROW) {
            b = row / g.nk;
            kk = row - b * g.nk;
        }
        const int c = kw + g.nw - 1;
        if constexpr (MODE == 2) {
            (void)b;   // staged in LDS above; the first pass reads it from there
        } else if constexpr (MODE == 0) {
            C = assemble_line<T>(g, b, kk, c, zrow, tsum, amp, wtab);
        } else {
            C = cin[static_cast<long>(row) * g.nc + c];
        }
        return C;
    };
    const int xtw = a.xtw, lg_w = ilog2i(xtw);
    T *rout = static_cast<T *>(a.rout);
    T2 *gout = static_cast<T2 *>(a.gout);
    auto out = [=](int f, int n, T2 v) {
        const int row = ONE_ROW ? rowu : row0 + f;
        if (row >= rows) return;
        if (rout) {   // one kappa line and one x point: the x-transform is the real part
            rout[static_cast<long>(row) * g.nt + n] = v.x;
            return;
        }
        // tile-major rows: the x-transform of a tile then reads one contiguous block
        int b = bu, kk = ku;
        if (!ONE_ROW) {
            b = row / g.nk;
            kk = row - b * g.nk;
        }
        const int tile = n >> lg_w;
        gout[static_cast<long>(b) * g.nk * g.nt + (static_cast<long>(tile) * g.nk + kk) * xtw + (n - (tile << lg_w))] = v;
    };
    fft_block<T, false, MODE == 2>(buf, a.sched, np, static_cast<const T2 *>(a.tw), in, out);
}

// (A_pure, A_pair) per line at unit scale: the FP64 expressions of
// assemble_line with scale 1, rounded to T.
template <typename T>
__global__ __launch_bounds__(256) void amp_table_kernel(const double *__restrict__ S, const double *__restrict__ sig,
                                                        double dkdw, double cap, long n,
                                                        typename vec<T>::v2 *__restrict__ out)
{
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double sc = 1.0;
    const double sraw = sc * sig[i];
    const double rho = (cap > 0.0 && sraw > cap) ? cap / sraw : 1.0;
    const double base = S[i] * dkdw;
    typename vec<T>::v2 v;
    v.x = static_cast<T>(2.0 * sqrt(base * (1.0 - rho * sraw)));
    v.y = static_cast<T>(2.0 * sqrt(base * rho * sc));
    out[i] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void assemble_kernel(TfftArgs a, typename vec<T>::v2 *cout)
{
    using T2 = typename vec<T>::v2;
    const Geometry &g = a.g;
    const long per = static_cast<long>(g.nk) * g.nc;
    const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (idx >= per) return;
    const int kk = static_cast<int>(idx / g.nc);
    const int c = static_cast<int>(idx - static_cast<long>(kk) * g.nc);
    cout[static_cast<long>(b) * per + idx] =
        assemble_line<T>(g, b, kk, c, static_cast<const typename vec<T>::v2 *>(a.zrow), static_cast<const T2 *>(a.tsum), a.amp,
                         static_cast<const T2 *>(a.wtab));
}

struct XfftArgs {
    Geometry g;
    FftSched sched;      // length n_x
    int tcols;           // columns (t samples) per block: one tile of gin
    const void *gin;     // [B][nt / tcols][nk][tcols]
    const void *tw;      // pass twiddles of n_x
    void *out;           // [B][nx][nt] real
    void *const *out_b;  // per realization output, or null (out + b * nx * nt)
};

// The x-transform takes the real part, so two columns share one complex
// transform: with a_1, a_2 the columns (non-zero at kk < nk <= nx) and
// y_j[n] = (a_j[n] + conj a_j[nx - n]) / 2 (Hermitian, so its inverse DFT is
// Re IDFT(a_j)), the inverse DFT of z = y_1 + i y_2 holds column 1's field in
// its real part and column 2's in its imaginary part.  One block transforms
// one tile of tcols columns (a contiguous block of gin) in tcols / 2 packed
// transforms, transform f on lane f: the tile's rows are read and the field's
// rows written as runs of tcols consecutive values.
template <typename T>
__global__ __launch_bounds__(sizeof(T) == 8 ? 512 : 1024) void xfft_kernel(XfftArgs a)
{
    using T2 = typename vec<T>::v2;
    extern __shared__ unsigned char smem_raw[];
    T2 *buf = reinterpret_cast<T2 *>(smem_raw);
    const Geometry &g = a.g;
    // tiles in the reverse of the order the t-transform writes them (by
    // realization): the most recently written part of G is read first, while
    // it is still in the Infinity Cache
    const int b = gridDim.y - 1 - blockIdx.y;
    const int tc = a.tcols;
    const int np = (tc + 1) / 2;   // packed transforms (a single column when tc == 1)
    const int mt0 = (gridDim.x - 1 - blockIdx.x) * tc;
    const int N = g.nx;
    const int nk = g.nk;
    const T2 *gin = static_cast<const T2 *>(a.gin) + (static_cast<long>(b) * g.nt + mt0) * nk;
    const bool sparse = 2 * nk <= N;   // a[n] and a[N - n] never both non-zero
    auto col2 = [&](int kk, int f, T2 &a1, T2 &a2) {
        const T2 *p = gin + static_cast<long>(kk) * tc + 2 * f;
        a1 = p[0];
        if (2 * f + 1 < tc) {
            a2 = p[1];
        } else {
            a2.x = T(0);
            a2.y = T(0);
        }
    };
    auto in = [&](int f, int n) -> T2 {
        T2 r;
        r.x = T(0);
        r.y = T(0);
        T2 a1, a2;
        if (sparse) {
            if (n == 0) {
                col2(0, f, a1, a2);
                r.x = a1.x;
                r.y = a2.x;
            } else if (n < nk) {
                col2(n, f, a1, a2);
                r.x = T(0.5) * (a1.x - a2.y);
                r.y = T(0.5) * (a1.y + a2.x);
            } else if (n > N - nk) {
                col2(N - n, f, a1, a2);
                r.x = T(0.5) * (a1.x + a2.y);
                r.y = T(0.5) * (a2.x - a1.y);
            }
            return r;
        }
        // n_x < 2 n_kappa: entry n takes a[n] and conj a[N - n] together
        const int km = (N - n) & (N - 1);
        T2 u1, u2, v1, v2;
        u1.x = u1.y = u2.x = u2.y = v1.x = v1.y = v2.x = v2.y = T(0);
        if (n < nk) col2(n, f, u1, u2);
        if (km < nk) col2(km, f, v1, v2);
        const T y1r = T(0.5) * (u1.x + v1.x), y1i = T(0.5) * (u1.y - v1.y);
        const T y2r = T(0.5) * (u2.x + v2.x), y2i = T(0.5) * (u2.y - v2.y);
        r.x = y1r - y2i;
        r.y = y1i + y2r;
        return r;
    };
    T *outp = a.out_b ? static_cast<T *>(a.out_b[b]) : static_cast<T *>(a.out) + static_cast<long>(b) * g.nx * g.nt;
    // pairs of columns as one store where the field is aligned for it (the
    // usual case: an even tile width and an aligned field)
    const bool vec_out = (reinterpret_cast<uintptr_t>(outp) & (sizeof(T2) - 1)) == 0 && (g.nt & 1) == 0 &&
                         (tc & 1) == 0;
    auto out = [&](int f, int mx, T2 z) {
        T *o = outp + static_cast<long>(mx) * g.nt + mt0 + 2 * f;
        if (vec_out) {
            *reinterpret_cast<T2 *>(o) = z;
        } else {
            o[0] = z.x;
            if (2 * f + 1 < tc) o[1] = z.y;
        }
    };
    fft_block<T, true, false>(buf, a.sched, np, static_cast<const T2 *>(a.tw), in, out);
}

// ---------------------------------------------------------------------------
// Pair sum through an FFT along kappa.
//
// For fixed frequencies (i_w, j_w) the kappa part of the ordered pair sum is a
// linear convolution of two phase columns, so with Z[q][i_w] the length-M DFT
// (M >= 2 N_kappa - 1, zero padded) of column i_w over kappa,
//     ordered sum O[kk][kw] = (1/M) sum_q e^{+2 pi i q kk / M} Y[q][kw],
//     Y[q][kw] = sum_{i_w} W(i_w, kw - i_w) Z[q][i_w] Z[q][kw - i_w],
// and T = O / 2 as in the direct form.  Y pairs (i_w, j_w) and (j_w, i_w) give
// the same term, so the sheared table Wh[i_w][kw] = f W(i_w, kw - i_w) with
// f = 2 (i_w > j_w), 1 (i_w = j_w), 0 (i_w < j_w) sums each unordered
// frequency pair once.  Work per realization: M x (2W - 1)^2 / 2 complex
// terms against N_kappa^2 (2W - 1)^2 / 4 in the direct form.
// ---------------------------------------------------------------------------

// Column DFTs over the rows of a row-major array, one block per tc columns:
// rows [0, in_rows) of columns col0 .. col0 + ncols - 1 are read (the rest of
// the N inputs are zero), transformed and rows [0, out_rows) are written,
// scaled, to columns ocol0 + c of the output.  `tw` is e^{+2 pi i n/N}; the
// forward transform (e^{-2 pi i}) conjugates the input and the output of the
// inverse one.
struct ColfftArgs {
    const void *in;
    long in_bstride;    // elements between realizations
    int in_ld, in_rows, col0;
    void *out;
    long out_bstride;
    int out_ld, out_rows, ocol0;
    int ncols, N, tc;
    int forward;
    const void *tw;
    double scale;
    int tw_lds;         // 1: the twiddles are copied to LDS after the tile
};

template <typename T, int MAXB>
__global__ __launch_bounds__(256) void colfft_kernel(ColfftArgs a)
{
    using T2 = typename vec<T>::v2;
    extern __shared__ unsigned char smem_raw[];
    T2 *buf = reinterpret_cast<T2 *>(smem_raw);
    const int b = blockIdx.y;
    const int c0 = blockIdx.x * a.tc;
    const int tc = min(a.tc, a.ncols - c0);
    const T2 *in = static_cast<const T2 *>(a.in) + b * a.in_bstride;
    for (int n = threadIdx.x; n < a.tc * a.N; n += blockDim.x) {
        const int row = n / a.tc, col = n - row * a.tc;
        T2 v;
        v.x = T(0);
        v.y = T(0);
        if (row < a.in_rows && col < tc) v = in[static_cast<long>(row) * a.in_ld + a.col0 + c0 + col];
        if (a.forward) v.y = -v.y;
        buf[col * a.N + row] = v;
    }
    T2 *twl = buf + a.tc * a.N;
    if (a.tw_lds)
        for (int n = threadIdx.x; n < a.N; n += blockDim.x) twl[n] = static_cast<const T2 *>(a.tw)[n];
    __syncthreads();
    fft_lds<T, MAXB>(buf, a.N, a.N, a.tc, a.tw_lds ? twl : static_cast<const T2 *>(a.tw));
    T2 *out = static_cast<T2 *>(a.out) + b * a.out_bstride;
    const T sc = static_cast<T>(a.scale);
    for (int n = threadIdx.x; n < a.out_rows * tc; n += blockDim.x) {
        const int row = n / tc, col = n - row * tc;
        T2 v = buf[col * a.N + row];
        v.x *= sc;
        v.y *= a.forward ? -sc : sc;
        out[static_cast<long>(row) * a.out_ld + a.ocol0 + c0 + col] = v;
    }
}

// Zero the pair sums of the output columns that no frequency pair reaches.
template <typename T>
__global__ __launch_bounds__(256) void zero_cols_kernel(typename vec<T>::v2 *tsum, int nk, int nc, int c_lo,
                                                        int c_hi)
{
    const long per = static_cast<long>(nk) * nc;
    const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= per) return;
    const int c = static_cast<int>(idx % nc);
    if (c >= c_lo && c <= c_hi) return;
    typename vec<T>::v2 z;
    z.x = T(0);
    z.y = T(0);
    tsum[static_cast<long>(blockIdx.y) * per + idx] = z;
}

// Bispectrum generated per pair inside the kernel, no table: for the
// canonical member (i, j) of an unordered pair (i_kappa > j_kappa, or equal
// and i_w >= j_w), Philox4x32-10 with key `key` and counter
// (i_kappa, i_w, j_kappa, j_w) gives b^2_raw = scale * word0 / 2^32 and
// beta = 2 pi word1 / 2^32.  One thread per output line loops over its pairs
// (self pair in full) and sums in FP64.  Without phases (zrow null) it sums
// b^2_raw per line (plan time); else it writes the unscaled pair sum
// sum sqrt(b^2_raw) e^{i(phi_i + phi_j + beta)}.
// A bispectrum drawn per 4-index pair, just in time (no table).  For the
// canonical member (i, j) of an unordered pair of line k = i + j, with
// m = floor(i_w / 8) and t = i_w - 8 m, Philox4x32-10 (key, counter
// (i_kappa, m, j_kappa, k_w)) holds the pair's 16 bits in word floor(t / 2)
// (high half for even t, low half for odd t): u = the high byte, v = the low
// byte, b_p = sqrt(alpha) u / 2^8 and beta = 2 pi v / 2^8.  One call thus
// serves the eight pairs of a line whose i_w share m.
//
// A wave owns one output row k_kappa and 64 consecutive output columns (one
// per lane); it walks the kappa splits i_kappa >= j_kappa and the partner
// columns in steps of eight (one generator call per lane and step).  z_i is
// the same for every lane (scalar loads), z_j is read at consecutive columns;
// the next step's phase factors are loaded while the generator runs.
// e^{i beta} comes from a 256-entry LDS table (FP64 sincospi, rounded to T).
// FP32 plans sum blocks of 32 steps in FP32 and the blocks in FP64; FP64 plans
// sum in FP64.  The SIGMA form writes the per-line raw sums
// alpha sum_P (u / 2^8)^2 instead (integer sum of u^2, exact).
struct HashPairArgs {
    Geometry g;
    uint64_t key;
    double scale;
    const void *zrow;   // [B][nk][nc] phase factors (pair-sum form)
    void *tsum;         // [B][nk][nc] complex out (pair-sum form)
    double *sig;        // [nk][nc] out (SIGMA form)
    int n_cg;           // column groups of 256 (four waves of 64 columns)
};

__device__ __forceinline__ int floor_div8(int x) { return x >= 0 ? x >> 3 : -((-x + 7) >> 3); }

template <typename T, bool SIGMA>
__global__ __launch_bounds__(256) void pairsum_hash_kernel(HashPairArgs a)
{
    using T2 = typename vec<T>::v2;
    __shared__ T2 tab[256];
    if (!SIGMA) {
        const int m = threadIdx.x;
        double sn, cs;
        sincospi(static_cast<double>(m) * (1.0 / 128.0), &sn, &cs);   // 2 pi m / 256
        tab[m].x = static_cast<T>(cs);
        tab[m].y = static_cast<T>(sn);
        __syncthreads();
    }
    const Geometry &g = a.g;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    const int kk = blockIdx.x / a.n_cg;
    const int cg = blockIdx.x - kk * a.n_cg;
    const int cw0 = (cg * 4 + wave) * 64;             // first column of the wave
    if (cw0 >= g.nc) return;
    const int c = cw0 + lane;
    const bool col_ok = c < g.nc;
    const int kw = c - (g.nw - 1);
    const int Wm1 = g.W - 1;
    // partner range of the lane and of the wave
    const int lo = max(-Wm1, kw - Wm1), hi = min(Wm1, kw + Wm1);
    const int kw_last = min(cw0 + 63, g.nc - 1) - (g.nw - 1);
    const int wlo = max(-Wm1, cw0 - (g.nw - 1) - Wm1), whi = min(Wm1, kw_last + Wm1);
    const int m_lo = floor_div8(wlo), m_hi = floor_div8(whi);
    const long per = static_cast<long>(g.nk) * g.nc;
    if (SIGMA) {
        uint64_t su = 0;
        for (int ik = (kk + 1) >> 1; ik <= kk; ++ik) {
            const int jk = kk - ik;
            for (int m = m_lo; m <= m_hi; ++m) {
                uint32_t w[4];
                philox_words4(static_cast<uint32_t>(ik), static_cast<uint32_t>(m), static_cast<uint32_t>(jk),
                              static_cast<uint32_t>(kw), a.key, w);
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int iw = 8 * m + t;
                    const bool ok = col_ok && iw >= lo && iw <= hi && (ik > jk || 2 * iw >= kw);
                    const uint32_t h = (t & 1) ? (w[t >> 1] & 0xFFFFu) : (w[t >> 1] >> 16);
                    const uint32_t u = ok ? (h >> 8) : 0u;
                    su += u * u;
                }
            }
        }
        if (col_ok) a.sig[static_cast<long>(kk) * g.nc + c] = a.scale * (static_cast<double>(su) * (1.0 / 65536.0));
        return;
    }
    const T2 *z = static_cast<const T2 *>(a.zrow) + static_cast<long>(blockIdx.y) * per;
    // z_j through a buffer resource over this realization's rows: partner
    // columns outside the row read a neighbouring row's (finite) factor and
    // offsets before the first or past the last row read zero; both carry a
    // zero weight
    const brsrc zr = make_brsrc(z, static_cast<unsigned>(per * sizeof(T2)));
    double sr = 0.0, si = 0.0;
    for (int ik = (kk + 1) >> 1; ik <= kk; ++ik) {
        const int jk = kk - ik;
        const T2 *zi_row = z + static_cast<long>(ik) * g.nc + (g.nw - 1);
        // pair (i_w, k_w - i_w) applies to the lane iff lo2 <= i_w <= hi (canonical
        // member: 2 i_w >= k_w when i_kappa = j_kappa); empty for lanes past the row
        const int lo2 = ik > jk ? lo : max(lo, (kw + 1) >> 1);
        const unsigned span = col_ok && hi >= lo2 ? static_cast<unsigned>(hi - lo2) : 0u;
        const int base = col_ok && hi >= lo2 ? lo2 : 0x40000000;
        // byte offset of z_j for i_w = 0 (row j_kappa, column k_w)
        const int jo = (jk * g.nc + (g.nw - 1) + kw) * static_cast<int>(sizeof(T2));
        T2 zi[8], zj[8];
        auto load = [&](int m) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int iw = 8 * m + t;
                zi[t] = zi_row[min(max(iw, -Wm1), Wm1)];
                zj[t] = bload(zr, static_cast<unsigned>(jo - iw * static_cast<int>(sizeof(T2))), 0u, T(0));
            }
        };
        load(m_lo);
        for (int m0 = m_lo; m0 <= m_hi; m0 += 32) {
            const int m1 = min(m_hi, m0 + 31);
            T br = T(0), bi = T(0);
            for (int m = m0; m <= m1; ++m) {
                T2 ci[8], cj[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    ci[t] = zi[t];
                    cj[t] = zj[t];
                }
                load(m + 1);   // clamped or range-checked, so safe past the last step too
                uint32_t w[4];
                philox_words4(static_cast<uint32_t>(ik), static_cast<uint32_t>(m), static_cast<uint32_t>(jk),
                              static_cast<uint32_t>(kw), a.key, w);
                const int d = 8 * m - base;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const bool ok = static_cast<unsigned>(d + t) <= span;
                    const uint32_t h = (t & 1) ? (w[t >> 1] & 0xFFFFu) : (w[t >> 1] >> 16);
                    const T b = ok ? static_cast<T>(h >> 8) : T(0);   // u; the 1/2^8 is applied at the end
                    const T2 e = tab[h & 0xFFu];
                    const T pr = ci[t].x * cj[t].x - ci[t].y * cj[t].y;
                    const T pi = ci[t].x * cj[t].y + ci[t].y * cj[t].x;
                    const T fr = b * e.x, fi = b * e.y;
                    br = fma_(fr, pr, fma_(-fi, pi, br));
                    bi = fma_(fr, pi, fma_(fi, pr, bi));
                }
            }
            sr += static_cast<double>(br);
            si += static_cast<double>(bi);
        }
    }
    if (!col_ok) return;
    const long idx = static_cast<long>(kk) * g.nc + c;
    const double sa = sqrt(a.scale) * (1.0 / 256.0);
    T2 o;
    o.x = static_cast<T>(sa * sr);
    o.y = static_cast<T>(sa * si);
    static_cast<T2 *>(a.tsum)[static_cast<long>(blockIdx.y) * per + idx] = o;
}

// Rank-one weights W(i_w, j_w) = g_i g_j (separable bicoherence, beta = 0):
// the weighted frequency autoconvolution of a DFT row is a plain linear
// autoconvolution of y = g Z, done as a forward FFT of length L >= 2(2W-1) - 1,
// a squaring and an inverse FFT, all in LDS (one block per row).  The forward
// transform is the inverse one on the conjugate; F(y)^2 = conj(conj(F(y))^2).
// Output column cc holds k_w = kw0 + cc, i.e. index k_w + 2W - 2 of the
// convolution, scaled by 1/L.
struct RowconvArgs {
    const void *Z;      // [rows][2W - 1] phase DFTs along kappa
    void *Y;            // [rows][nca]
    const void *gw;     // [2W - 1] g = sqrt(g2), path precision
    const void *tw;     // [L] exp(+2 pi i n / L)
    int W, nca, kw0, L;
    int tw_lds;         // 1: the twiddles are copied to LDS after the row
};

template <typename T, int MAXB>
__global__ __launch_bounds__(1024) void rowconv_kernel(RowconvArgs a)
{
    using T2 = typename vec<T>::v2;
    extern __shared__ unsigned char smem_raw[];
    T2 *buf = reinterpret_cast<T2 *>(smem_raw);
    const int ncw = 2 * a.W - 1;
    const long row = blockIdx.x;
    const T2 *z = static_cast<const T2 *>(a.Z) + row * ncw;
    const T *gw = static_cast<const T *>(a.gw);
    for (int n = threadIdx.x; n < a.L; n += blockDim.x) {
        T2 v;
        v.x = T(0);
        v.y = T(0);
        if (n < ncw) {
            const T2 x = z[n];
            v.x = gw[n] * x.x;
            v.y = -gw[n] * x.y;
        }
        buf[n] = v;
    }
    T2 *twl = buf + a.L;
    if (a.tw_lds)
        for (int n = threadIdx.x; n < a.L; n += blockDim.x) twl[n] = static_cast<const T2 *>(a.tw)[n];
    const T2 *tw = a.tw_lds ? twl : static_cast<const T2 *>(a.tw);
    __syncthreads();
    fft_lds<T, MAXB>(buf, a.L, a.L, 1, tw);
    for (int n = threadIdx.x; n < a.L; n += blockDim.x) {
        const T2 f = buf[n];
        T2 v;
        v.x = f.x * f.x - f.y * f.y;
        v.y = T(-2) * f.x * f.y;
        buf[n] = v;
    }
    __syncthreads();
    fft_lds<T, MAXB>(buf, a.L, a.L, 1, tw);
    T2 *y = static_cast<T2 *>(a.Y) + row * a.nca;
    const T sc = T(1) / static_cast<T>(a.L);
    for (int cc = threadIdx.x; cc < a.nca; cc += blockDim.x) {
        T2 v = buf[a.kw0 + cc + 2 * a.W - 2];
        v.x *= sc;
        v.y *= sc;
        y[cc] = v;
    }
}

// Sheared half table Wh[ic][cc] = f W(i_w, kw - i_w) over the active output
// columns cc (kw = kw0 + cc), zero outside the support; `pad` rows of zeros
// follow the table.
template <typename T>
__global__ __launch_bounds__(256) void wsh_kernel(const typename vec<T>::v2 *__restrict__ wt, int W, int nca,
                                                  int kw0, int pad_rows, typename vec<T>::v2 *__restrict__ wh)
{
    const int ncw = 2 * W - 1;
    const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<long>(ncw + pad_rows) * nca) return;
    const int ic = static_cast<int>(idx / nca), cc = static_cast<int>(idx - static_cast<long>(ic) * nca);
    typename vec<T>::v2 v;
    v.x = T(0);
    v.y = T(0);
    if (ic < ncw) {
        const int iw = ic - (W - 1), jw = kw0 + cc - iw;
        if (jw > -W && jw < W && iw >= jw) {
            v = wt[static_cast<long>(ic) * ncw + (jw + W - 1)];
            if (iw > jw) {
                v.x *= T(2);
                v.y *= T(2);
            }
        }
    }
    wh[idx] = v;
}

struct YpairArgs {
    const void *Z;      // [B][M][ncw] phase DFTs along kappa
    void *Y;            // [B][M][nca]
    const void *wh;     // [wh_rows][nca] sheared half table, zero rows after row ncw - 1
    int M, W, nca, kw0;
    int batch, n_qtiles, n_ctiles, per_xcd;
    int one_sided;      // partners i_w <= k_omega only (both partners >= 0)
};

// Staged form of the frequency autoconvolution.  A wave owns 64 consecutive
// output columns (one per lane) and R DFT rows q, and walks the partner
// frequencies i_w in chunks of C steps.  The b operand Z[q][kw - i_w] of lane
// l at step i_w is element e = e0 + l - i_w of row q, so a chunk reads a
// window of 64 + C - 1 elements per row; the window and the chunk's a
// operands Z[q][i_w] (the same for all lanes) are staged in the wave's own
// slice of LDS with coalesced global loads -- no barrier: the wave alone
// writes and reads its slice.  The weight row W_h[i_w][.] is read from global
// memory once per step for all R rows, two steps ahead.  Steps past the last
// partner meet zero weights (zero rows after the table, or pairs outside the
// support).  Per term: t = a b (4 ops), acc += w t (4 FMAs).
constexpr int kY2Rows = 8;      // DFT rows per wave
constexpr int kY2Chunk = 32;    // steps per staged window
constexpr int kY2Unroll = 4;

template <typename T, int R, int C>
__global__ __launch_bounds__(256) void ypair2_kernel(YpairArgs a)
{
    using T2 = typename vec<T>::v2;
    constexpr int LW = 64 + C;   // staged elements per row (64 + C - 1 used)
    static_assert((R * LW) % 64 == 0 && (C * R) % 64 == 0 && C % kY2Unroll == 0, "staging shape");
    extern __shared__ unsigned char smem_raw[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    T2 *ldsb = reinterpret_cast<T2 *>(smem_raw) + wave * (R * LW + C * R);
    T2 *ldsa = ldsb + R * LW;
    // a block: one column tile, kWavesPerBlock consecutive q tiles (one per
    // wave), so that its waves read the same weight rows at about the same time
    const int bid = blockIdx.x;
    const int work = (bid % kNumXcd) * a.per_xcd + bid / kNumXcd;
    const int n_qgroups = (a.n_qtiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per_b = n_qgroups * a.n_ctiles;
    if (work >= a.batch * per_b) return;
    const int b = work / per_b;
    const int rem = work - b * per_b;
    const int qg = rem / a.n_ctiles;
    const int ct = rem - qg * a.n_ctiles;
    const int qt = qg * kWavesPerBlock + wave;
    if (qt >= a.n_qtiles) return;
    const int cc0 = ct * 64;
    const int W = a.W, ncw = 2 * W - 1, q0 = qt * R;
    const T2 *Zb = static_cast<const T2 *>(a.Z) + static_cast<long>(b) * a.M * ncw;
    const int kw_lo = a.kw0 + cc0;
    const int kw_hi = a.kw0 + min(cc0 + 64, a.nca) - 1;
    const int iw_lo = max(-W + 1, (kw_lo + 1) >> 1);
    const int iw_hi = min(W - 1, a.one_sided ? kw_hi : kw_hi + W - 1);
    const int nchunk = __builtin_amdgcn_readfirstlane(iw_hi >= iw_lo ? (iw_hi - iw_lo + C) / C : 0);
    const gptr<T2> wcol = as_global(static_cast<const T2 *>(a.wh)) + cc0 + lane;
    const long wstride = a.nca;

    T accr[R], acci[R], sumr[R], sumi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) accr[r] = acci[r] = sumr[r] = sumi[r] = T(0);

    for (int ch = 0; ch < nchunk; ++ch) {
        const int iwc = iw_lo + ch * C;
        // b window: lane l at chunk step s reads index l + C - 1 - s of row r
        const int e_lo = kw_lo + W - 1 - (iwc + C - 1);
#pragma unroll
        for (int i = 0; i < R * LW / 64; ++i) {
            const int idx = i * 64 + lane;
            const int r = idx / LW, x = idx - r * LW;
            const int e = e_lo + x;
            T2 v;
            v.x = T(0);
            v.y = T(0);
            if (e >= 0 && e < ncw) v = Zb[static_cast<long>(min(q0 + r, a.M - 1)) * ncw + e];
            ldsb[r * LW + x] = v;
        }
        // a operands of the chunk, [s][r]
#pragma unroll
        for (int i = 0; i < C * R / 64; ++i) {
            const int idx = i * 64 + lane;
            const int st = idx / R, r = idx - st * R;
            const int ic = iwc + st + W - 1;
            T2 v;
            v.x = T(0);
            v.y = T(0);
            if (ic < ncw) v = Zb[static_cast<long>(min(q0 + r, a.M - 1)) * ncw + ic];
            ldsa[st * R + r] = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int ic0 = iwc + W - 1;
        T2 w0 = wcol[static_cast<long>(ic0) * wstride];
        T2 w1 = wcol[static_cast<long>(ic0 + 1) * wstride];
        for (int s0 = 0; s0 < C; s0 += kY2Unroll) {
#pragma unroll
            for (int u = 0; u < kY2Unroll; ++u) {
                const int s = s0 + u;
                const T2 w2 = wcol[static_cast<long>(ic0 + s + 2) * wstride];
                const int x = lane + C - 1 - s;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const T2 av = ldsa[s * R + r];
                    const T2 bv = ldsb[r * LW + x];
                    const T tr = fma_(av.x, bv.x, -av.y * bv.y);
                    const T ti = fma_(av.x, bv.y, av.y * bv.x);
                    accr[r] = fma_(w0.x, tr, accr[r]);
                    accr[r] = fma_(-w0.y, ti, accr[r]);
                    acci[r] = fma_(w0.x, ti, acci[r]);
                    acci[r] = fma_(w0.y, tr, acci[r]);
                }
                w0 = w1;
                w1 = w2;
            }
        }
        // the slice is rewritten by the next chunk only after these reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (ch & 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                sumr[r] += accr[r];
                sumi[r] += acci[r];
                accr[r] = acci[r] = T(0);
            }
        }
    }
    T2 *Y = static_cast<T2 *>(a.Y) + static_cast<long>(b) * a.M * a.nca;
    const int cc = cc0 + lane;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (cc < a.nca && q0 + r < a.M) {
            T2 v;
            v.x = sumr[r] + accr[r];
            v.y = sumi[r] + acci[r];
            Y[static_cast<long>(q0 + r) * a.nca + cc] = v;
        }
    }
}

// Pair weight table W[i][j] = sqrt(b2_raw(i, j)) exp(i beta(i, j)) over the
// support |i_w|, |j_w| < W (index i_w + W - 1), computed in FP64 and stored in
// the path precision.  b2_raw = g2[i] g2[j] (separable) or b2[i][j] (dense);
// beta from Philox (counter (max, min, 1, 0), key beta_seed), a table, or 0.
template <typename T>
__global__ __launch_bounds__(256) void wtable_kernel(int W, int b2_kind, const double *__restrict__ g2,
                                                     const double *__restrict__ b2, int beta_mode,
                                                     const uint32_t *__restrict__ beta_tab, uint64_t beta_seed,
                                                     typename vec<T>::v2 *__restrict__ wt)
{
    const int ncw = 2 * W - 1;
    const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<long>(ncw) * ncw) return;
    const int i = static_cast<int>(idx / ncw), j = static_cast<int>(idx - static_cast<long>(i) * ncw);
    double v = 0.0;
    if (b2_kind == SRM3_BISPEC_SEPARABLE) v = g2[i] * g2[j];
    else if (b2_kind == SRM3_BISPEC_DENSE) v = b2[idx];
    uint32_t beta = 0u;
    if (b2_kind != SRM3_BISPEC_NONE) {
        if (beta_mode == SRM3_BETA_SEEDED) {
            const int iw = i - (W - 1), jw = j - (W - 1);
            const int hi = iw >= jw ? iw : jw, lo = iw >= jw ? jw : iw;
            beta = philox_word0(static_cast<uint32_t>(hi), static_cast<uint32_t>(lo), 1u, 0u, beta_seed);
        } else if (beta_mode == SRM3_BETA_TABLE) {
            beta = beta_tab[idx];
        }
    }
    double sn, cs;
    sincospi(static_cast<double>(beta) * (1.0 / 2147483648.0), &sn, &cs);
    const double m = sqrt(v);
    typename vec<T>::v2 o;
    o.x = static_cast<T>(m * cs);
    o.y = static_cast<T>(m * sn);
    wt[idx] = o;
}

// Spectrum on the lines from the Kaimal frequency spectrum times the exact
// Fourier transform of the Davenport coherence (the wind-field example of
// Section 5, in the workload normalisation), FP64; S(., 0) = 0.
__global__ __launch_bounds__(256) void spectrum_kernel(int nk, int nw, double dk, double dw, double u_star,
                                                       double z, double U, double lam, double *S)
{
    const int nc = 2 * nw - 1;
    const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<long>(nk) * nc) return;
    const int kk = static_cast<int>(idx / nc);
    const int kw = static_cast<int>(idx - static_cast<long>(kk) * nc) - (nw - 1);
    double v = 0.0;
    if (kw != 0) {
        const double two_pi = 6.283185307179586476925286766559;
        const double w = fabs(static_cast<double>(kw)) * dw;
        const double f = w / two_pi;
        const double sw = 200.0 * u_star * u_star * (z / U) / pow(1.0 + 50.0 * f * z / U, 5.0 / 3.0);
        const double a = lam * w / (two_pi * U);
        const double kap = kk * dk;
        v = sw * (a / 3.14159265358979323846264338327950288) / (a * a + kap * kap);
    }
    S[idx] = v;
}

constexpr int kFftMaxB = 4;

int fft_threads(int butterflies)
{
    int t = (butterflies + kFftMaxB - 1) / kFftMaxB;
    t = ((t + 63) / 64) * 64;
    if (t < 64) t = 64;
    if (t > 1024) t = 1024;
    return t;
}

}  // namespace

int pairsum_rows_per_wave(int nk, int precision)
{
    const int cap = 8;   // FP32: 4 waves per SIMD at R = 8 beat 2 at R = 16; FP64: 3 waves
    int r = 2;
    while (r * 2 <= cap && r * 2 <= nk) r *= 2;
    return r;
}

size_t workspace_bytes(const Geometry &g, int precision, int batch)
{
    const size_t e = precision == SRM3_FP64 ? 8 : 4;
    const size_t lines = static_cast<size_t>(g.nk) * g.nc;
    auto al = [](size_t x) { return (x + 255) & ~static_cast<size_t>(255); };
    return al(batch * lines * 2 * e) + al(static_cast<size_t>(batch) * g.ncw * g.nkp * a_slots(precision) * e) +
           al(batch * lines * 2 * e) + al(static_cast<size_t>(batch) * g.nk * g.nt * 2 * e);
}

Workspace carve_workspace(const Geometry &g, int precision, int batch, void *base)
{
    const size_t e = precision == SRM3_FP64 ? 8 : 4;
    const size_t lines = static_cast<size_t>(g.nk) * g.nc;
    auto al = [](size_t x) { return (x + 255) & ~static_cast<size_t>(255); };
    char *p = static_cast<char *>(base);
    Workspace w;
    w.zrow = p;
    p += al(batch * lines * 2 * e);
    w.zcol = p;
    p += al(static_cast<size_t>(batch) * g.ncw * g.nkp * a_slots(precision) * e);
    w.tsum = p;
    p += al(batch * lines * 2 * e);
    w.g = p;
    return w;
}

template <typename T, int TR>
static void launch_phase_tiles(const Geometry &g, const SeedChunk &sc, const uint64_t *seeds_dev, int b0, int nb,
                               const Workspace &ws, const double *lr, hipStream_t st)
{
    // tiles of 64 frequencies from the multiple of 4 at or below -(n_omega - 1)
    const int kwb = 4 * floor_div4(-(g.nw - 1));
    const unsigned gx = static_cast<unsigned>((g.nw - kwb + 63) / 64), gy = static_cast<unsigned>((g.nkp + TR - 1) / TR);
    phase_kernel<T, TR><<<dim3(gx, gy, nb), 256, 0, st>>>(sc, seeds_dev, b0, g,
                                                          static_cast<typename vec<T>::v2 *>(ws.zrow),
                                                          static_cast<T *>(ws.zcol), lr);
}

template <typename T>
static hipError_t phases_t(const Geometry &g, const uint64_t *seeds, const uint64_t *seeds_dev, int batch,
                           const Workspace &ws, const double *lr, hipStream_t st)
{
    // seeds travel as kernel arguments in chunks, or are read from the device
    const int chunk = seeds_dev ? 65535 : kMaxSeedsPerLaunch;
    for (int b0 = 0; b0 < batch; b0 += chunk) {
        const int nb = std::min(chunk, batch - b0);
        SeedChunk sc{};
        if (!seeds_dev)
            for (int i = 0; i < nb; ++i) sc.s[i] = seeds[b0 + i];
        if (!ws.zcol) {
            const long ng = floor_div4(g.nw - 1) - floor_div4(-(g.nw - 1)) + 1;
            const long calls = static_cast<long>(g.nk) * ng;
            phase_rows_kernel<T><<<dim3(static_cast<unsigned>((calls + kPhaseRowCalls - 1) / kPhaseRowCalls), nb),
                                   256, 0, st>>>(sc, seeds_dev, b0, g, static_cast<typename vec<T>::v2 *>(ws.zrow),
                                                 lr);
        } else if (g.nkp <= 16) {
            launch_phase_tiles<T, 16>(g, sc, seeds_dev, b0, nb, ws, lr, st);
        } else {
            launch_phase_tiles<T, sizeof(T) == 8 ? 32 : 64>(g, sc, seeds_dev, b0, nb, ws, lr, st);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_phases(const Geometry &g, int precision, const uint64_t *seeds, const uint64_t *seeds_dev,
                         int batch, const Workspace &ws, const double *lr, hipStream_t st)
{
    return precision == SRM3_FP64 ? phases_t<double>(g, seeds, seeds_dev, batch, ws, lr, st)
                                  : phases_t<float>(g, seeds, seeds_dev, batch, ws, lr, st);
}

template <typename T, int R, bool COMP>
static hipError_t pairsum_t(const Geometry &g, const void *wtab, int batch, const Workspace &ws,
                            hipStream_t st)
{
    PairsumArgs a;
    a.zrow = ws.zrow;
    a.zcol = ws.zcol;
    a.wtab = wtab;
    a.tout = ws.tsum;
    a.g = g;
    a.batch = batch;
    a.n_rowblocks = g.nkp / R;
    a.n_ctiles = (g.nc + 63) / 64;
    a.n_cgroups = (a.n_ctiles + kWavesPerBlock - 1) / kWavesPerBlock;
    a.flush_terms = kFlushTerms;
    const long work = static_cast<long>(a.n_rowblocks) * batch * a.n_cgroups;
    a.per_xcd = batch >= kNumXcd ? static_cast<int>((work + kNumXcd - 1) / kNumXcd) : 0;
    const long blocks = a.per_xcd > 0 ? static_cast<long>(a.per_xcd) * kNumXcd : work;
    pairsum_kernel<T, R, COMP><<<dim3(static_cast<unsigned>(blocks)), 64 * kWavesPerBlock, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_pairsum(const Geometry &g, int precision, const void *wtab, int batch,
                          const Workspace &ws, hipStream_t st)
{
    if (precision == SRM3_FP64) {
        switch (g.R) {
        case 2: return pairsum_t<double, 2, false>(g, wtab, batch, ws, st);
        case 4: return pairsum_t<double, 4, false>(g, wtab, batch, ws, st);
        case 8: return pairsum_t<double, 8, false>(g, wtab, batch, ws, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (g.R) {
    case 2: return pairsum_t<float, 2, true>(g, wtab, batch, ws, st);
    case 4: return pairsum_t<float, 4, true>(g, wtab, batch, ws, st);
    case 8: return pairsum_t<float, 8, true>(g, wtab, batch, ws, st);
    case 16: return pairsum_t<float, 16, true>(g, wtab, batch, ws, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int RT, int CT>
static hipError_t pairsum_mfma_t(const Geometry &g, const void *wtab, int batch, const Workspace &ws, hipStream_t st)
{
    MfmaArgs a;
    a.zrow = ws.zrow;
    a.zcol = ws.zcol;
    a.wtab = wtab;
    a.tout = ws.tsum;
    a.g = g;
    a.batch = batch;
    a.n_rg = (g.nk + 16 * RT - 1) / (16 * RT);
    const int n_ct = (g.nc + 16 * CT - 1) / (16 * CT);
    a.n_cg = (n_ct + kWavesPerBlock - 1) / kWavesPerBlock;
    a.flush_steps = kMfmaFlushSteps;
    const long work = static_cast<long>(a.n_rg) * batch * a.n_cg;
    a.per_xcd = batch >= kNumXcd ? static_cast<int>((work + kNumXcd - 1) / kNumXcd) : 0;
    const long blocks = a.per_xcd > 0 ? static_cast<long>(a.per_xcd) * kNumXcd : work;
    // raised MFMA priority pays where every SIMD runs many waves over the
    // launch (256x1024 x 64 and 512x8192 x 16: 1.2-1.4 % faster) and costs
    // small launches (the bridge example's 4 blocks per CU: 10 % slower)
    if (blocks >= kMfmaPrioBlocks)
        pairsum_mfma_kernel<T, RT, CT, true><<<dim3(static_cast<unsigned>(blocks)), 64 * kWavesPerBlock, 0, st>>>(a);
    else
        pairsum_mfma_kernel<T, RT, CT, false><<<dim3(static_cast<unsigned>(blocks)), 64 * kWavesPerBlock, 0, st>>>(a);
    return hipGetLastError();
}

// Tile shapes of the matrix-core pair sum: 16 x 16 MFMA tiles per wave,
// RT along kappa x CT along the frequency.  Shape 0 is the default.
MfmaShape mfma_shape(int precision, int id)
{
    static const MfmaShape f32[kMfmaShapes] = {{2, 2}, {2, 1}, {1, 2}};
    static const MfmaShape f64[kMfmaShapes] = {{2, 2}, {2, 1}, {1, 2}};
    if (id < 0 || id >= kMfmaShapes) id = 0;
    return precision == SRM3_FP64 ? f64[id] : f32[id];
}

hipError_t launch_pairsum_mfma(const Geometry &g, int precision, int shape, const void *wtab, int batch,
                               const Workspace &ws, hipStream_t st)
{
    if (precision == SRM3_FP64) {
        switch (shape) {
        case 1: return pairsum_mfma_t<double, 2, 1>(g, wtab, batch, ws, st);
        case 2: return pairsum_mfma_t<double, 1, 2>(g, wtab, batch, ws, st);
        default: return pairsum_mfma_t<double, 2, 2>(g, wtab, batch, ws, st);
        }
    }
    switch (shape) {
    case 1: return pairsum_mfma_t<float, 2, 1>(g, wtab, batch, ws, st);
    case 2: return pairsum_mfma_t<float, 1, 2>(g, wtab, batch, ws, st);
    default: return pairsum_mfma_t<float, 2, 2>(g, wtab, batch, ws, st);
    }
}

template <typename T>
static hipError_t pairsum_hash_t(const Geometry &g, uint64_t key, double scale, int batch, const Workspace *ws,
                                 double *sig, hipStream_t st)
{
    HashPairArgs a{};
    a.g = g;
    a.key = key;
    a.scale = scale;
    a.zrow = ws ? ws->zrow : nullptr;
    a.tsum = ws ? ws->tsum : nullptr;
    a.sig = sig;
    a.n_cg = (g.nc + 255) / 256;
    const long per = static_cast<long>(g.nk) * g.nc;
    const unsigned gx = static_cast<unsigned>(static_cast<long>(a.n_cg) * g.nk);
    hipError_t e = hipSuccess;
    for (int b0 = 0; b0 < (ws ? batch : 1); b0 += 65535) {
        const int nb = ws ? std::min(65535, batch - b0) : 1;
        HashPairArgs c = a;
        if (ws) {
            c.zrow = static_cast<const typename vec<T>::v2 *>(ws->zrow) + static_cast<long>(b0) * per;
            c.tsum = static_cast<typename vec<T>::v2 *>(ws->tsum) + static_cast<long>(b0) * per;
        }
        if (ws)
            pairsum_hash_kernel<T, false><<<dim3(gx, nb), 256, 0, st>>>(c);
        else
            pairsum_hash_kernel<T, true><<<dim3(gx, nb), 256, 0, st>>>(c);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return e;
}

hipError_t launch_pairsum_hash(const Geometry &g, int precision, uint64_t key, double scale, int batch,
                               const Workspace *ws, double *sig, hipStream_t st)
{
    return precision == SRM3_FP64 ? pairsum_hash_t<double>(g, key, scale, batch, ws, sig, st)
                                  : pairsum_hash_t<float>(g, key, scale, batch, ws, sig, st);
}

template <typename T, int RT, int CT>
static hipError_t persistent_mfma_t(const void *reqs, const void *items, const int *q_begin, int *q_next,
                                    int nblocks, hipStream_t st)
{
    fill_int_kernel<<<1, 64, 0, st>>>(q_next, kNumXcd, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    PersistArgs a;
    a.reqs = static_cast<const PReq *>(reqs);
    a.items = static_cast<const PItem *>(items);
    a.q_begin = q_begin;
    a.q_next = q_next;
    a.flush_terms = kFlushTerms;
    pairsum_persistent_mfma<T, RT, CT><<<dim3(static_cast<unsigned>(nblocks)), 64 * kWavesPerBlock, 0, st>>>(a);
    return hipGetLastError();
}

template <typename T, int R, bool COMP>
static hipError_t persistent_t(const void *reqs, const void *items, const int *q_begin, int *q_next, int nblocks,
                               hipStream_t st)
{
    fill_int_kernel<<<1, 64, 0, st>>>(q_next, kNumXcd, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    PersistArgs a;
    a.reqs = static_cast<const PReq *>(reqs);
    a.items = static_cast<const PItem *>(items);
    a.q_begin = q_begin;
    a.q_next = q_next;
    a.flush_terms = kFlushTerms;
    pairsum_persistent<T, R, COMP><<<dim3(static_cast<unsigned>(nblocks)), 64 * kWavesPerBlock, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_pairsum_persistent(int precision, int R, const void *reqs, const void *items, const int *q_begin,
                                     int *q_next, int nblocks, hipStream_t st, bool mfma, int shape)
{
    if (mfma) {
        if (precision == SRM3_FP64) {
            switch (shape) {
            case 1: return persistent_mfma_t<double, 2, 1>(reqs, items, q_begin, q_next, nblocks, st);
            case 2: return persistent_mfma_t<double, 1, 2>(reqs, items, q_begin, q_next, nblocks, st);
            default: return persistent_mfma_t<double, 2, 2>(reqs, items, q_begin, q_next, nblocks, st);
            }
        }
        switch (shape) {
        case 1: return persistent_mfma_t<float, 2, 1>(reqs, items, q_begin, q_next, nblocks, st);
        case 2: return persistent_mfma_t<float, 1, 2>(reqs, items, q_begin, q_next, nblocks, st);
        default: return persistent_mfma_t<float, 2, 2>(reqs, items, q_begin, q_next, nblocks, st);
        }
    }
    if (precision == SRM3_FP64) {
        switch (R) {
        case 2: return persistent_t<double, 2, false>(reqs, items, q_begin, q_next, nblocks, st);
        case 4: return persistent_t<double, 4, false>(reqs, items, q_begin, q_next, nblocks, st);
        case 8: return persistent_t<double, 8, false>(reqs, items, q_begin, q_next, nblocks, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (R) {
    case 2: return persistent_t<float, 2, true>(reqs, items, q_begin, q_next, nblocks, st);
    case 4: return persistent_t<float, 4, true>(reqs, items, q_begin, q_next, nblocks, st);
    case 8: return persistent_t<float, 8, true>(reqs, items, q_begin, q_next, nblocks, st);
    case 16: return persistent_t<float, 16, true>(reqs, items, q_begin, q_next, nblocks, st);
    default: return hipErrorInvalidValue;
    }
}

size_t persistent_req_bytes() { return sizeof(PReq); }
int mfma_rows_per_group(int precision, int shape) { return 16 * mfma_shape(precision, shape).rt; }
int mfma_cols_per_group(int precision, int shape) { return 16 * mfma_shape(precision, shape).ct * kWavesPerBlock; }
size_t persistent_item_bytes() { return sizeof(PItem); }

void fill_persistent_req(void *dst, const Geometry &g, const void *zrow, const void *zcol, void *tsum,
                         const void *wtab)
{
    PReq r{};
    r.g = g;
    r.zrow = zrow;
    r.zcol = zcol;
    r.tsum = tsum;
    r.wtab = wtab;
    r.n_ctiles = (g.nc + 63) / 64;
    std::memcpy(dst, &r, sizeof r);
}

void fill_persistent_item(void *dst, int req, int kb, int cg)
{
    PItem it{req, kb, cg, 0};
    std::memcpy(dst, &it, sizeof it);
}

int waves_per_block() { return kWavesPerBlock; }

hipError_t launch_fill_u32(void *p, size_t words, uint32_t v, hipStream_t st)
{
    if (words == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((words + 255) / 256, 8192);
    fill_u32_kernel<<<dim3(static_cast<unsigned>(blocks)), 256, 0, st>>>(static_cast<uint32_t *>(p), words, v);
    return hipGetLastError();
}

// Columns per tile of the t-transformed rows = the x-transform's tile width:
// 64 KB of packed transforms (nx complex values per pair of columns), at most
// n_t.  Both launchers take it from here, so the two layouts agree.
// Elements of one block of the register-blocked FFT: 16 per thread, at most
// 1024 threads (512 for FP64), 128 KB of LDS.
template <typename T>
constexpr int fft_block_elems()
{
    return sizeof(T) == 8 ? 8192 : 16384;
}

// Columns per block of the x-transform, which is also the tile width of the
// t-transform's output: two columns per packed transform, as many transforms
// as fill a block (at most 32), never more than n_t.  A power of two.  Both
// launchers take it from here, so the two layouts agree.
template <typename T>
static int xfft_cols(const Geometry &g)
{
    int np = fft_block_elems<T>() / g.nx;
    if (np > 32) np = 32;
    if (np < 1) np = 1;
    int tc = 2 * np;
    if (tc > g.nt) tc = g.nt;
    return tc;
}

static int fft_block_threads(long elems)
{
    long t = (elems + 15) / 16;
    t = ((t + 63) / 64) * 64;
    return static_cast<int>(std::max(64L, std::min(1024L, t)));
}

template <typename T>
static hipError_t tfft_t(const Geometry &g, int mode, const void *cin, const AmpRef &amp, const void *wtab,
                         const void *tw, int batch, const Workspace &ws, void *rout, const uint64_t *seeds,
                         hipStream_t st)
{
    using T2 = typename vec<T>::v2;
    TfftArgs a;
    a.rout = (g.nx == 1 && g.nk == 1) ? rout : nullptr;
    a.g = g;
    a.mode = mode;
    a.cin = cin;
    a.zrow = ws.zrow;
    a.tsum = ws.tsum;
    a.seeds_dev = nullptr;
    a.b0 = 0;
    a.amp = AmpArgs{amp.S, amp.sig, amp.scale_b, amp.S_b, amp.dkdw, amp.cap, amp.pairs, amp.lc, amp.lr, amp.tab};
    a.wtab = wtab;
    a.tw = tw;
    a.gout = ws.g;
    a.xtw = xfft_cols<T>(g);
    a.sched = fft_schedule(g.nt);
    // short rows share a block (1024 elements per block, at most 64 rows)
    a.np = g.nt >= 1024 ? 1 : std::min(64, 1024 / g.nt);
    const int thr = fft_block_threads(static_cast<long>(a.np) * g.nt);
    // rows (padded), then (several rows per block) their seeds, then (mode 2)
    // the phase-factor table, 16-byte aligned
    const size_t lds = static_cast<size_t>(fft_lds_elems<T>(a.np * g.nt)) * sizeof(T2) +
                       (a.np > 1 ? a.np * sizeof(uint64_t) : 0) + (mode == 2 ? 256 * sizeof(double2) + 16 : 0);
    // mode 2 with host seeds: kernel-argument chunks of realizations (the
    // per-realization spectrum and scale arrays are not used in this mode)
    const int chunk = mode == 2 ? kMaxSeedsPerLaunch : batch;
    for (int b0 = 0; b0 < batch; b0 += chunk) {
        const int nb = std::min(chunk, batch - b0);
        TfftArgs c = a;
        c.rows = nb * g.nk;
        if (mode == 2) {
            for (int i = 0; i < nb; ++i) c.seeds.s[i] = seeds[b0 + i];
            c.gout = static_cast<T2 *>(ws.g) + static_cast<long>(b0) * g.nk * g.nt;
            if (c.rout) c.rout = static_cast<T *>(rout) + static_cast<long>(b0) * g.nt;
        }
        const unsigned blocks = static_cast<unsigned>((c.rows + a.np - 1) / a.np);
        const bool one = a.np == 1;
        if (mode == 2)
            one ? tfft_kernel<T, 2, true><<<dim3(blocks), thr, lds, st>>>(c)
                : tfft_kernel<T, 2, false><<<dim3(blocks), thr, lds, st>>>(c);
        else if (mode == 0)
            one ? tfft_kernel<T, 0, true><<<dim3(blocks), thr, lds, st>>>(c)
                : tfft_kernel<T, 0, false><<<dim3(blocks), thr, lds, st>>>(c);
        else
            one ? tfft_kernel<T, 1, true><<<dim3(blocks), thr, lds, st>>>(c)
                : tfft_kernel<T, 1, false><<<dim3(blocks), thr, lds, st>>>(c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_amp_table(int precision, long n, const double *S, const double *sig, double dkdw, double cap,
                            void *out, hipStream_t st)
{
    const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
    if (precision == SRM3_FP64)
        amp_table_kernel<double><<<blocks, 256, 0, st>>>(S, sig, dkdw, cap, n, static_cast<double2 *>(out));
    else
        amp_table_kernel<float><<<blocks, 256, 0, st>>>(S, sig, dkdw, cap, n, static_cast<float2 *>(out));
    return hipGetLastError();
}

hipError_t launch_tfft(const Geometry &g, int precision, int mode, const void *cin, const AmpRef &amp,
                       const void *wtab, const void *tw, int batch, const Workspace &ws, hipStream_t st, void *rout,
                       const uint64_t *seeds)
{
    if (mode == 2 && !seeds) return hipErrorInvalidValue;
    return precision == SRM3_FP64 ? tfft_t<double>(g, mode, cin, amp, wtab, tw, batch, ws, rout, seeds, st)
                                  : tfft_t<float>(g, mode, cin, amp, wtab, tw, batch, ws, rout, seeds, st);
}

template <typename T>
static hipError_t assemble_t(const Geometry &g, const AmpRef &amp, const void *wtab, int batch,
                             const Workspace &ws, void *cout, hipStream_t st)
{
    TfftArgs a{};
    a.g = g;
    a.zrow = ws.zrow;
    a.tsum = ws.tsum;
    a.amp = AmpArgs{amp.S, amp.sig, amp.scale_b, amp.S_b, amp.dkdw, amp.cap, amp.pairs, amp.lc, amp.lr, amp.tab};
    a.wtab = wtab;
    const long per = static_cast<long>(g.nk) * g.nc;
    assemble_kernel<T><<<dim3(static_cast<unsigned>((per + 255) / 256), batch), 256, 0, st>>>(
        a, static_cast<typename vec<T>::v2 *>(cout));
    return hipGetLastError();
}

hipError_t launch_assemble(const Geometry &g, int precision, const AmpRef &amp, const void *wtab, int batch,
                           const Workspace &ws, void *cout, hipStream_t st)
{
    return precision == SRM3_FP64 ? assemble_t<double>(g, amp, wtab, batch, ws, cout, st)
                                  : assemble_t<float>(g, amp, wtab, batch, ws, cout, st);
}

template <typename T>
static hipError_t xfft_t(const Geometry &g, const void *tw, int batch, const Workspace &ws, void *out,
                         void *const *out_b, hipStream_t st)
{
    XfftArgs a;
    a.g = g;
    a.sched = fft_schedule(g.nx);
    const int tc = xfft_cols<T>(g);
    const int np = (tc + 1) / 2;
    a.tcols = tc;
    a.gin = ws.g;
    a.tw = tw;
    a.out = out;
    a.out_b = out_b;
    const int thr = fft_block_threads(static_cast<long>(np) * g.nx);
    const size_t lds = static_cast<size_t>(np) * g.nx * sizeof(typename vec<T>::v2);
    xfft_kernel<T><<<dim3(static_cast<unsigned>(g.nt / tc), batch), thr, lds, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_xfft(const Geometry &g, int precision, const void *tw, int batch, const Workspace &ws,
                       void *out, void *const *out_b, hipStream_t st)
{
    return precision == SRM3_FP64 ? xfft_t<double>(g, tw, batch, ws, out, out_b, st)
                                  : xfft_t<float>(g, tw, batch, ws, out, out_b, st);
}

// ---- pair sum through an FFT along kappa ----

KfftGeom kfft_geometry(const Geometry &g, bool one_sided)
{
    KfftGeom k{};
    int M = 1;
    while (M < 2 * g.nk - 1) M *= 2;
    k.M = M;
    k.one_sided = one_sided ? 1 : 0;
    // output frequencies that a pair of support frequencies reaches
    const int kw_lo = one_sided ? 0 : std::max(-(g.nw - 1), -(2 * g.W - 2));
    const int kw_hi = std::min(g.nw - 1, 2 * g.W - 2);
    k.kw0 = kw_lo;
    k.c_lo = kw_lo + g.nw - 1;
    k.nca = kw_hi - kw_lo + 1;
    // zero rows after the table: the weight rows read up to C + 1 steps past
    // the last partner, and the ragged last column tile (< 64 columns past a
    // row's end)
    k.wh_rows = g.ncw + kY2Chunk + 2 + (64 + k.nca - 1) / k.nca;
    return k;
}

size_t kfft_workspace_bytes(const Geometry &g, const KfftGeom &k, int precision, int batch)
{
    const size_t e2 = precision == SRM3_FP64 ? 16 : 8;
    auto al = [](size_t x) { return (x + 255) & ~static_cast<size_t>(255); };
    return al(static_cast<size_t>(batch) * k.M * g.ncw * e2) + al(static_cast<size_t>(batch) * k.M * k.nca * e2);
}

KfftWorkspace carve_kfft(const Geometry &g, const KfftGeom &k, int precision, int batch, void *base)
{
    const size_t e2 = precision == SRM3_FP64 ? 16 : 8;
    auto al = [](size_t x) { return (x + 255) & ~static_cast<size_t>(255); };
    KfftWorkspace w;
    w.Z = base;
    w.Y = static_cast<char *>(base) + al(static_cast<size_t>(batch) * k.M * g.ncw * e2);
    return w;
}

bool kfft_supported(const Geometry &, const KfftGeom &k, int, std::string *why)
{
    // one column transform of length M fits the column-DFT kernel's LDS
    if (k.M > 4096) {
        if (why) *why = "n_kappa above 2048";
        return false;
    }
    return true;
}

template <typename T>
static hipError_t wsh_t(const void *wt, const Geometry &g, const KfftGeom &k, void *wh, hipStream_t st)
{
    const long n = static_cast<long>(k.wh_rows) * k.nca;
    wsh_kernel<T><<<dim3(static_cast<unsigned>((n + 255) / 256)), 256, 0, st>>>(
        static_cast<const typename vec<T>::v2 *>(wt), g.W, k.nca, k.kw0, k.wh_rows - g.ncw,
        static_cast<typename vec<T>::v2 *>(wh));
    return hipGetLastError();
}

hipError_t launch_wsh(int precision, const void *wt, const Geometry &g, const KfftGeom &k, void *wh, hipStream_t st)
{
    return precision == SRM3_FP64 ? wsh_t<double>(wt, g, k, wh, st) : wsh_t<float>(wt, g, k, wh, st);
}

template <typename T>
static hipError_t colfft_t(ColfftArgs a, int batch, hipStream_t st)
{
    using T2 = typename vec<T>::v2;
    a.tc = std::max(1, static_cast<int>(32768 / (static_cast<long>(a.N) * sizeof(T2))));
    const dim3 grid(static_cast<unsigned>((a.ncols + a.tc - 1) / a.tc), static_cast<unsigned>(batch));
    size_t lds = static_cast<size_t>(a.tc) * a.N * sizeof(T2);
    a.tw_lds = lds + a.N * sizeof(T2) <= 131072 ? 1 : 0;
    if (a.tw_lds) lds += a.N * sizeof(T2);
    colfft_kernel<T, 4><<<grid, 256, lds, st>>>(a);
    return hipGetLastError();
}

template <typename T>
static hipError_t kfft_pairsum_t(const Geometry &g, const KfftGeom &k, const KfftTables &tab, int batch,
                                 const Workspace &ws, const KfftWorkspace &kw, hipStream_t st)
{
    const void *wh = tab.wh, *tw_i = tab.tw_k;
    using T2 = typename vec<T>::v2;
    hipError_t e;
    for (int b0 = 0; b0 < batch; b0 += 65535) {
        const int nb = std::min(65535, batch - b0);
        // forward DFT along kappa of the support columns
        ColfftArgs f{};
        f.in = static_cast<const T2 *>(ws.zrow) + static_cast<long>(b0) * g.nk * g.nc;
        f.in_bstride = static_cast<long>(g.nk) * g.nc;
        f.in_ld = g.nc;
        f.in_rows = g.nk;
        f.col0 = g.nw - g.W;
        f.out = static_cast<T2 *>(kw.Z) + static_cast<long>(b0) * k.M * g.ncw;
        f.out_bstride = static_cast<long>(k.M) * g.ncw;
        f.out_ld = g.ncw;
        f.out_rows = k.M;
        f.ocol0 = 0;
        f.ncols = g.ncw;
        f.N = k.M;
        f.forward = 1;
        f.tw = tw_i;
        f.scale = 1.0;
        if ((e = colfft_t<T>(f, nb, st)) != hipSuccess) return e;
    }
    if (k.L > 0) {
        // rank-one weights: FFT autoconvolution of every (realization, q) row
        RowconvArgs r{};
        r.Z = kw.Z;
        r.Y = kw.Y;
        r.gw = tab.gw;
        r.tw = tab.tw_l;
        r.W = g.W;
        r.nca = k.nca;
        r.kw0 = k.kw0;
        r.L = k.L;
        const long rows = static_cast<long>(batch) * k.M;
        const int thr = fft_threads(k.L / 2);
        size_t lds = static_cast<size_t>(k.L) * sizeof(T2);
        r.tw_lds = 2 * lds <= 131072 ? 1 : 0;
        if (r.tw_lds) lds *= 2;
        for (long r0 = 0; r0 < rows; r0 += 1L << 30) {
            const long nr = std::min(rows - r0, 1L << 30);
            RowconvArgs rr = r;
            rr.Z = static_cast<const T2 *>(kw.Z) + r0 * g.ncw;
            rr.Y = static_cast<T2 *>(kw.Y) + r0 * k.nca;
            rowconv_kernel<T, kFftMaxB><<<dim3(static_cast<unsigned>(nr)), thr, lds, st>>>(rr);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    } else {
    // weighted frequency autoconvolution per kappa frequency q
    YpairArgs y{};
    y.Z = kw.Z;
    y.Y = kw.Y;
    y.wh = wh;
    y.M = k.M;
    y.W = g.W;
    y.nca = k.nca;
    y.kw0 = k.kw0;
    y.batch = batch;
    y.one_sided = k.one_sided;
    if (k.M == 1) {
        // one kappa line: the realizations are the rows ([B][1][.] == [B][.])
        y.M = batch;
        y.batch = 1;
    }
    y.n_qtiles = (y.M + kY2Rows - 1) / kY2Rows;
    y.n_ctiles = (k.nca + 63) / 64;
    const long blocks = static_cast<long>(y.batch) * ((y.n_qtiles + kWavesPerBlock - 1) / kWavesPerBlock) * y.n_ctiles;
    y.per_xcd = static_cast<int>((blocks + kNumXcd - 1) / kNumXcd);
    const size_t lds = static_cast<size_t>(kWavesPerBlock) * (kY2Rows * (64 + kY2Chunk) + kY2Chunk * kY2Rows) *
                       sizeof(T2);
    ypair2_kernel<T, kY2Rows, kY2Chunk><<<dim3(static_cast<unsigned>(static_cast<long>(y.per_xcd) * kNumXcd)),
                                         64 * kWavesPerBlock, lds, st>>>(y);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (int b0 = 0; b0 < batch; b0 += 65535) {
        const int nb = std::min(65535, batch - b0);
        // inverse DFT along kappa, first n_kappa rows, halved: T = O / 2
        ColfftArgs v{};
        v.in = static_cast<const T2 *>(kw.Y) + static_cast<long>(b0) * k.M * k.nca;
        v.in_bstride = static_cast<long>(k.M) * k.nca;
        v.in_ld = k.nca;
        v.in_rows = k.M;
        v.col0 = 0;
        v.out = static_cast<T2 *>(ws.tsum) + static_cast<long>(b0) * g.nk * g.nc;
        v.out_bstride = static_cast<long>(g.nk) * g.nc;
        v.out_ld = g.nc;
        v.out_rows = g.nk;
        v.ocol0 = k.c_lo;
        v.ncols = k.nca;
        v.N = k.M;
        v.forward = 0;
        v.tw = tw_i;
        v.scale = 0.5 / k.M;
        if ((e = colfft_t<T>(v, nb, st)) != hipSuccess) return e;
        if (k.nca < g.nc) {
            const long per = static_cast<long>(g.nk) * g.nc;
            zero_cols_kernel<T><<<dim3(static_cast<unsigned>((per + 255) / 256), static_cast<unsigned>(nb)), 256, 0,
                                  st>>>(static_cast<T2 *>(ws.tsum) + static_cast<long>(b0) * per, g.nk, g.nc,
                                        k.c_lo, k.c_lo + k.nca - 1);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_kfft_pairsum(int precision, const Geometry &g, const KfftGeom &k, const KfftTables &t, int batch,
                               const Workspace &ws, const KfftWorkspace &kw, hipStream_t st)
{
    return precision == SRM3_FP64 ? kfft_pairsum_t<double>(g, k, t, batch, ws, kw, st)
                                  : kfft_pairsum_t<float>(g, k, t, batch, ws, kw, st);
}

double kfft_terms(const Geometry &g, const KfftGeom &k)
{
    if (k.L > 0) {
        // two length-L transforms (L/2 log2 L butterflies each) and L squarings per row
        int lg = 0;
        while ((1 << lg) < k.L) ++lg;
        return static_cast<double>(k.M) * (static_cast<double>(k.L) * lg + k.L);
    }
    // complex terms of the frequency autoconvolution per realization: for each
    // q, the unordered support pairs (i_w >= j_w) of every active output
    double t = 0;
    for (int kw = k.kw0; kw < k.kw0 + k.nca; ++kw) {
        int lo = std::max(-(g.W - 1), kw - (g.W - 1)), hi = std::min(g.W - 1, kw + (g.W - 1));
        if (k.one_sided) hi = std::min(hi, kw);   // both partners >= 0
        const int half_lo = std::max(lo, (kw + 1) >> 1);
        if (hi >= half_lo) t += hi - half_lo + 1;
    }
    return t * k.M;
}

// Allow the transform kernels the 128 KB of LDS a length-16384 FP32 (8192
// FP64) transform needs.  Called once when a plan is built, never during a
// stream capture.
template <typename T>
static hipError_t prepare_t()
{
    const int lds = 131072;
    // the transforms' padded rows take up to 139 KB (of the 160 KB of a workgroup)
    const void *tk[] = {reinterpret_cast<const void *>(&tfft_kernel<T, 0, true>),
                        reinterpret_cast<const void *>(&tfft_kernel<T, 0, false>),
                        reinterpret_cast<const void *>(&tfft_kernel<T, 1, true>),
                        reinterpret_cast<const void *>(&tfft_kernel<T, 1, false>),
                        reinterpret_cast<const void *>(&tfft_kernel<T, 2, true>),
                        reinterpret_cast<const void *>(&tfft_kernel<T, 2, false>)};
    hipError_t e = hipSuccess;
    for (const void *k : tk)
        if ((e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 163840)) != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&rowconv_kernel<T, kFftMaxB>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&colfft_kernel<T, kFftMaxB>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&xfft_kernel<T>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
}

hipError_t prepare_transforms(int precision)
{
    return precision == SRM3_FP64 ? prepare_t<double>() : prepare_t<float>();
}

hipError_t launch_wtable(int precision, int W, int b2_kind, const double *g2, const double *b2, int beta_mode,
                        const uint32_t *beta_tab, uint64_t beta_seed, void *wt, hipStream_t st)
{
    const long n = static_cast<long>(2 * W - 1) * (2 * W - 1);
    const dim3 grid(static_cast<unsigned>((n + 255) / 256));
    if (precision == SRM3_FP64)
        wtable_kernel<double><<<grid, 256, 0, st>>>(W, b2_kind, g2, b2, beta_mode, beta_tab, beta_seed,
                                                    static_cast<double2 *>(wt));
    else
        wtable_kernel<float><<<grid, 256, 0, st>>>(W, b2_kind, g2, b2, beta_mode, beta_tab, beta_seed,
                                                   static_cast<float2 *>(wt));
    return hipGetLastError();
}

hipError_t launch_spectrum(int nk, int nw, double dk, double dw, double u_star, double z, double U, double lam,
                           double *S, hipStream_t st)
{
    const long n = static_cast<long>(nk) * (2 * nw - 1);
    spectrum_kernel<<<dim3(static_cast<unsigned>((n + 255) / 256)), 256, 0, st>>>(nk, nw, dk, dw, u_star, z, U,
                                                                                   lam, S);
    return hipGetLastError();
}

}  // namespace srm3
