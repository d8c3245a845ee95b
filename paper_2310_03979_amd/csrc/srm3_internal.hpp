// Internal declarations of the srm3 HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "srm3.h"

namespace srm3 {

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11):
// ten rounds of two 32x32 -> 64-bit multiplies mixed with a Weyl key schedule.
// Only the first output word is used.  Host and device share this definition.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint64_t key)
{
    uint32_t k0 = static_cast<uint32_t>(key), k1 = static_cast<uint32_t>(key >> 32);
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c0;
}

template <typename T> struct vec;
template <> struct vec<float> { using v2 = float2; using v4 = float4; };
template <> struct vec<double> { using v2 = double2; using v4 = double4; };

constexpr int kMaxSeedsPerLaunch = 32;
struct SeedChunk {
    uint64_t s[kMaxSeedsPerLaunch];
};

// Geometry shared by the kernels of one plan.
struct Geometry {
    int nk, nw, W;      // lines n_kappa x (2 nw - 1); pair support |omega| < W
    int nc, ncw;        // 2 nw - 1, 2 W - 1
    int nx, nt;         // field
    int R;              // output rows per wave in the pair sum
    int nkp;            // n_kappa rounded up to a multiple of R
};

// Device workspace of one generate call (views into the plan's buffer).
struct Workspace {
    void *zrow;   // [B][nk][nc] complex phase factors, row-major over lines
    void *zcol;   // [B][3][ncw][nkp] planes (re + im, re, im), kappa-contiguous per support column
    void *tsum;   // [B][nk][nc] complex pair sums
    void *g;      // [B][nk][nt] complex, after the t-transform
};

size_t workspace_bytes(const Geometry &g, int precision, int batch);
Workspace carve_workspace(const Geometry &g, int precision, int batch, void *base);

// Inputs of the FP64 amplitude computation done on the device (see
// assemble_line): plan spectrum, unit-scale raw pair sums, optional
// per-realization b^2 scales and spectra (device arrays indexed by the
// realization within a launch).
struct AmpRef {
    const double *S;
    const double *sig;
    const double *scale_b;
    const double *const *S_b;
    double dkdw;
    double cap;
};

// Kernel launchers (stream-ordered, return the launch status).
hipError_t launch_phases(const Geometry &g, int precision, const uint64_t *seeds, const uint64_t *seeds_dev,
                         int batch, const Workspace &ws, hipStream_t st);
hipError_t launch_pairsum(const Geometry &g, int precision, const void *wtab, int batch,
                          const Workspace &ws, hipStream_t st);
// Persistent pair sum over a device work list (all requests share R).
hipError_t launch_pairsum_persistent(int precision, int R, const void *reqs, const void *items, const int *q_begin,
                                     int *q_next, int nblocks, hipStream_t st);
size_t persistent_req_bytes();
size_t persistent_item_bytes();
void fill_persistent_req(void *dst, const Geometry &g, const void *zrow, const void *zcol, void *tsum,
                         const void *wtab);
void fill_persistent_item(void *dst, int req, int kb, int cg);
int waves_per_block();
constexpr int kXcds = 8;
// mode 0: assemble C from pair sums and phases; mode 1: read C from `cin`.
hipError_t launch_tfft(const Geometry &g, int precision, int mode, const void *cin, const AmpRef &amp,
                       const void *wtab, const void *tw, int batch, const Workspace &ws, hipStream_t st);
hipError_t launch_assemble(const Geometry &g, int precision, const AmpRef &amp, const void *wtab, int batch,
                           const Workspace &ws, void *cout, hipStream_t st);
hipError_t launch_xfft(const Geometry &g, int precision, const void *tw, int batch, const Workspace &ws,
                       void *out, void *const *out_b, hipStream_t st);
hipError_t launch_spectrum(int nk, int nw, double dk, double dw, double u_star, double z, double U, double lam,
                           double *S, hipStream_t st);

int pairsum_rows_per_wave(int nk, int precision);
hipError_t prepare_transforms(int precision);

}  // namespace srm3
