// Shared definitions of the coarse-operator library (device and host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "coarse.h"

namespace coarse {

// ---------------------------------------------------------------------------
// Geometry, passed to kernels by value.
// ---------------------------------------------------------------------------
struct Geom {
    int L[4];
    int V;
    int nb;
    int np;
    int self_p;            // index of the zero displacement, -1 if absent
    int8_t off[81][4];
};

__device__ __forceinline__ void site_coords(const Geom &g, int s, int c[4]) {
    c[0] = s % g.L[0];
    s /= g.L[0];
    c[1] = s % g.L[1];
    s /= g.L[1];
    c[2] = s % g.L[2];
    c[3] = s / g.L[2];
}

// Index of x + sign*delta_p (periodic), x given by coordinates.
__device__ __forceinline__ int displaced(const Geom &g, const int c[4], int p, int sign) {
    int y[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        int v = c[mu] + sign * (int)g.off[p][mu];
        v += (v < 0) ? g.L[mu] : 0;
        v -= (v >= g.L[mu]) ? g.L[mu] : 0;
        y[mu] = v;
    }
    return y[0] + g.L[0] * (y[1] + g.L[1] * (y[2] + g.L[2] * y[3]));
}

// ---------------------------------------------------------------------------
// Packed link layouts.
//
// C64 "tiled" layout (nbasis % 8 == 0): a block A_p(x) is nb x nb complex; its
// real embedding A'[i][k'] with k' = 2j + h (h: 0 = Re, 1 = Im) is stored in
// chunks of 16 k'-columns; inside a chunk the rows come in 16-row tiles and
// a tile is laid out [q][row][u] with k' = 16c + 4u + q, so that lane
// t = q*16 + row of a wave reads the 4 floats it feeds to 4 consecutive
// 16x16x4 MFMA steps with one 16-byte load and the 64 lanes read 1 KB
// contiguously. Partial row tiles (nb % 16 == 8) are stored without padding.
// Other nbasis: natural row-major order.
//
// 16-bit layout (BF16/FP16, nbasis % 16 == 0): k' is split in steps of 32;
// inside a step a 16-row tile is [q][row][e] with k' = 32 st + 8q + e, so that
// lane t = q*16 + row reads the 8 values of one 16x16x32 MFMA operand with
// one 16-byte load (4 consecutive complex entries of row i).
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ bool tiled_c64(int nb) { return (nb % 8) == 0; }

// Float offset of the complex entry (i, j), component comp, inside one block of
// the 3M layout (nb % 16 == 0): chunk c = j / 8 of eight columns, 16-row tile
// mt; the tile's 16-byte entry (il, q) holds (Re, Im) of columns 8c + q and
// 8c + 4 + q of row 16 mt + il, entries ordered [il / 4][q][il % 4]. The
// forward kernel's lane (il, q) reads entry (il, q) (a wave reads the whole
// 1 KiB tile); the adjoint's k-step reads rows 4s..4s + 3 of all eight columns
// of a chunk, which this order makes 256 contiguous bytes (two whole lines).
__host__ __device__ __forceinline__ int c64_3m_block_offset(int nb, int i, int j, int comp) {
    int c = j >> 3, half = (j >> 2) & 1, q = j & 3;
    int mt = i >> 4, il = i & 15;
    return (c * nb + 16 * mt) * 16 + ((il >> 2) * 16 + q * 4 + (il & 3)) * 4 + 2 * half + comp;
}

// Float offset of A'[i][kp] inside one c64 block.
__host__ __device__ __forceinline__ int c64_block_offset(int nb, int i, int kp) {
    if (!tiled_c64(nb)) return i * 2 * nb + kp;
    int c = kp >> 4, u = (kp >> 2) & 3, q = kp & 3;
    int mt = i >> 4, il = i & 15;
    int rows = nb - 16 * mt;
    rows = rows < 16 ? rows : 16;
    return (c * nb + 16 * mt) * 16 + (q * rows + il) * 4 + u;
}

// Element offset of A'[i][kp] inside one 16-bit block.
__host__ __device__ __forceinline__ int h16_block_offset(int nb, int i, int kp) {
    int st = kp >> 5, q = (kp >> 3) & 3, e = kp & 7;
    int mt = i >> 4, il = i & 15;
    return ((st * (nb >> 4) + mt) * 64 + (q * 16 + il)) * 8 + e;
}

// Byte layout of a 16-bit packed buffer: [links 16-bit][self c64 tiled][scales]
struct LowpLayout {
    size_t links_bytes, self_off, self_bytes, scale_off, total;
};

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

inline LowpLayout lowp_layout(int V, int np, int nb, bool has_self) {
    LowpLayout l;
    l.links_bytes = (size_t)V * np * nb * nb * 2 * 2;
    l.self_off = align256(l.links_bytes);
    l.self_bytes = has_self ? (size_t)V * nb * nb * 8 : 0;
    l.scale_off = align256(l.self_off + l.self_bytes);
    l.total = l.scale_off + (size_t)V * np * 4;
    return l;
}

// ---------------------------------------------------------------------------
// Explicit LDS pointers: selecting between LDS buffers through generic
// pointers can make the compiler fall back to flat accesses, and every flat
// access waits for all outstanding global loads.
// ---------------------------------------------------------------------------
// Global address space: pointers typed with it compile to global (not flat)
// memory instructions, which do not wait on LDS traffic.
#define GLOBAL_AS __attribute__((address_space(1)))

#define LDS_AS __attribute__((address_space(3)))
template <typename T>
__device__ __forceinline__ LDS_AS T *lds_ptr(void *p) {
    return (LDS_AS T *)(p);
}

// ---------------------------------------------------------------------------
// MFMA operand types
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mfma16x16x4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16x16x4(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Rounding helpers shared by the pack and apply kernels.
// ---------------------------------------------------------------------------
// 2^ceil(log2 m) for m > 0, 1 for m == 0 (or NaN).
__device__ __forceinline__ float pow2_ceil(float m) {
    if (!(m > 0.f)) return 1.f;
    int e;
    float mant = frexpf(m, &e);
    if (mant == 0.5f) e -= 1;
    return ldexpf(1.f, e);
}

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// float -> IEEE half bits, round to nearest even (hardware conversion).
__device__ __forceinline__ uint16_t to_f16_bits(float f) {
    _Float16 h = (_Float16)f;
    return __builtin_bit_cast(uint16_t, h);
}

__device__ __forceinline__ float bf16_bits_to_float(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ float f16_bits_to_float(uint16_t b) {
    return (float)__builtin_bit_cast(_Float16, b);
}

// ---------------------------------------------------------------------------
// Host-side error plumbing
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();
int32_t hip_fail(hipError_t e, const char *what);

#define COARSE_HIP(call)                                   \
    do {                                                   \
        hipError_t _e = (call);                            \
        if (_e != hipSuccess) return hip_fail(_e, #call);  \
    } while (0)

// Validate a geometry and fill the device-side struct. Returns CG_OK or an error.
int32_t make_geom(const coarse_geom *g, Geom *out);
int32_t check_nrhs(int32_t nrhs);

}  // namespace coarse
