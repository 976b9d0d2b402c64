// Shared device-side definitions of the QAP swarm library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qap {

constexpr int kWave = 64;
constexpr int kMaxN = 256;

// Best-ever record of an instance (device memory).
struct BestRec {
    long long goal;
    int iter, swarm, member;
    int pad;
    uint8_t perm[kMaxN];
};

// Per-swarm minimum of the current goals of one iteration.
struct SwarmMin {
    long long goal;
    int member;
    int pad;
};

// Everything a kernel needs to know about one instance.  Device pointers.
// Particle k of the instance is member k % S of swarm k / S.
struct InstDesc {
    int n;          // problem size
    int npad;       // n rounded up to a multiple of 32 (MFMA tiles)
    int m, S, P;    // swarms, members per swarm, particles
    float c1, c2, c3, vmax;
    int norm;       // S_v: 0 raw, 1 column-normalised
    int depth;      // SecondTarget depth
    int sx;         // S_x procedure: 0 SecondTarget, 1 PickColumn
    int ls;         // best-improvement pair exchanges per particle-iteration (0: none)
    int migrate, migr_d, period;
    int sym;        // F and D both symmetric
    int zd;         // F and D both have a zero diagonal
    int path;       // 1 int8 MFMA, 2 int32, 3 byte-split int8 MFMA
    int split;      // path 3: bit 0 F split into two planes, bit 1 D split
    uint64_t seed;
    int swarm_base; // index of this descriptor's first swarm in the instance (random streams, records)
    // instance data
    const int* F32;         // [n][n]
    const int* D32;         // [n][n]
    const int8_t* F8;       // [npad][npad] zero padded (int8 path) : F
    const int8_t* D8;       // [npad][npad] : D
    const int8_t* FT8;      // [npad][npad] : F^T
    const int8_t* DT8;      // [npad][npad] : D^T
    // path 3: F8 / D8 hold the low planes (M mod 128 where split, else M),
    // FH8 / DH8 the high planes floor(M / 128) of the split matrices
    const int8_t* FH8;      // [npad][npad]
    const int8_t* DH8;      // [npad][npad]
    // particle state; index [k] by particle, two buffers selected by iteration parity
    // V is kept column-scaled: V[r][c] = fl(U[r][c] * Vinv[c]) with U the
    // unnormalised S_v output and Vinv the reciprocal column norm (1 for raw
    // S_v).  Applying the scale on read gives the same binary32 value as
    // storing the normalised matrix, and lets the velocity pass stream.
    float* V[2];            // [P][n][n] U, row = location, column = facility
    float* Vinv[2];         // [P][n]    column scale
    uint8_t* X[2];          // [P][n]   p[i] = location of facility i
    uint8_t* PL;            // [P][n]
    long long* goal;        // [P]
    long long* goalPL;      // [P]
    uint8_t* PG;            // [m][n]
    long long* goalPG;      // [m]
    SwarmMin* smin;         // [m]
    BestRec* best;          // [1]
    int* iter;              // [1] completed iterations
    int* order;             // [m] migration ranking scratch
    uint8_t* Xnew;          // [P][n] SecondTarget output (per-stage engine)
    int* scratch;           // per-block contraction scratch (per-stage engine)
};

// A pointer read from device memory (a descriptor in a device table) is
// generic to the compiler, so accesses through it become flat instructions
// (64-bit addresses in vector registers, and waits shared with LDS).  Every
// pointer of a descriptor is device global memory: accesses through gl(p)
// are global instructions.
template <class T>
using global_t = __attribute__((address_space(1))) T;

template <class T>
__device__ __forceinline__ global_t<T>* gl(T* p)
{
    return (global_t<T>*)p;
}

// Buffer b (0 or 1) of a double-buffered member, chosen by a select rather
// than an index: a descriptor held in registers then stays in registers.
template <class T>
__device__ __forceinline__ T* buf(T* const (&a)[2], int b)
{
    return b ? a[1] : a[0];
}

// ---------------------------------------------------------------- wave ops
// The lane id goes through an empty asm so that values derived from it are
// formed where used rather than hoisted out of a long loop (where they would
// hold vector registers for its whole length).
__device__ __forceinline__ int lane_id()
{
    int l = (int)__lane_id();
    asm volatile("" : "+v"(l));
    return l;
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROW_MASK,
                                                      0xF, false));
}

// Maximum over the 64 lanes, returned to every lane (uniform).
__device__ __forceinline__ float wave_max(float v)
{
    v = fmaxf(v, dpp_f32<0xB1>(v));        // quad_perm [1,0,3,2]
    v = fmaxf(v, dpp_f32<0x4E>(v));        // quad_perm [2,3,0,1]
    v = fmaxf(v, dpp_f32<0x141>(v));       // row_half_mirror
    v = fmaxf(v, dpp_f32<0x140>(v));       // row_mirror: every lane holds its row's max
    v = fmaxf(v, dpp_f32<0x142, 0xA>(v));  // row_bcast15 into rows 1, 3
    v = fmaxf(v, dpp_f32<0x143, 0xC>(v));  // row_bcast31 into rows 2, 3
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// DPP move of a 32-bit value; lanes whose row is masked off, or whose source lies
// outside the row, receive `old`.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ int dpp_i32(int old, int v)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROW_MASK, 0xF, false);
}

// Sum over the 64 lanes, returned to every lane (uniform).  Same row steps as
// wave_max, with 0 entering from masked rows.
__device__ __forceinline__ int wave_sum_i32(int v)
{
    v += dpp_i32<0xB1>(0, v);
    v += dpp_i32<0x4E>(0, v);
    v += dpp_i32<0x141>(0, v);
    v += dpp_i32<0x140>(0, v);
    v += dpp_i32<0x142, 0xA>(0, v);
    v += dpp_i32<0x143, 0xC>(0, v);
    return __builtin_amdgcn_readlane(v, 63);
}

// Inclusive prefix sum over the lanes in lane order: row_shr 1, 2, 4, 8 inside
// each row of 16, then the row totals by row_bcast15 / row_bcast31.
__device__ __forceinline__ int wave_incl_scan_i32(int v)
{
    v += dpp_i32<0x111>(0, v);
    v += dpp_i32<0x112>(0, v);
    v += dpp_i32<0x114>(0, v);
    v += dpp_i32<0x118>(0, v);
    v += dpp_i32<0x142, 0xA>(0, v);
    v += dpp_i32<0x143, 0xC>(0, v);
    return v;
}

__device__ __forceinline__ long long wave_sum_i64(long long v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ long long dpp_i64(long long v)
{
    const int lo = dpp_i32<CTRL, ROW_MASK>((int)v, (int)v);
    const int hi = dpp_i32<CTRL, ROW_MASK>((int)(v >> 32), (int)(v >> 32));
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Minimum over the 64 lanes, returned to every lane (uniform).
__device__ __forceinline__ long long wave_min_i64(long long v)
{
    long long o;
    o = dpp_i64<0xB1>(v); v = o < v ? o : v;
    o = dpp_i64<0x4E>(v); v = o < v ? o : v;
    o = dpp_i64<0x141>(v); v = o < v ? o : v;
    o = dpp_i64<0x140>(v); v = o < v ? o : v;
    o = dpp_i64<0x142, 0xA>(v); v = o < v ? o : v;
    o = dpp_i64<0x143, 0xC>(v); v = o < v ? o : v;
    const int lo = __builtin_amdgcn_readlane((int)v, 63), hi = __builtin_amdgcn_readlane((int)(v >> 32), 63);
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ int readlane_i32(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ float readlane_f32(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ uint64_t ballot64(bool p) { return (uint64_t)__ballot(p); }

// Lexicographic (delta, a, b) minimum over the wave; result uniform.
__device__ __forceinline__ void wave_argmin_pair(long long& d, int& a, int& b)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const long long d2 = __shfl_xor(d, off, kWave);
        const int a2 = __shfl_xor(a, off, kWave);
        const int b2 = __shfl_xor(b, off, kWave);
        const bool take = (d2 < d) || (d2 == d && (a2 < a || (a2 == a && b2 < b)));
        if (take) { d = d2; a = a2; b = b2; }
    }
}

}  // namespace qap
