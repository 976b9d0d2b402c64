// Fused engine: the whole particle iteration in one kernel, one wave64 per
// particle, F and D staged in LDS as int8, the pair-exchange contraction on
// gfx950 int8 MFMA (v_mfma_i32_32x32x32_i8, int32 accumulation).
//
// Per particle (wave):
//  A. stream V(t) once, lane = column (facility), the lane's columns l, l + 64,
//     ... taken through each batch of rows in turn (each load a 256-byte row
//     segment): the velocity update of eq. (velocity) with the S_v clamp, the
//     column norm (stored as a column scale applied on the next read), the
//     store of V(t+1) into the other buffer, and the SecondTarget column caches
//     (max key, Z-cell key).  The at most three cells per column touched by
//     the attraction terms (rows of X, P^L, P^G) are corrected right after
//     the batch that holds them.
//  B. SecondTarget (Alg. 1) on X(t) + V(t), rescans reading V(t) from L2.
//  C. A = F . Dp^T and A^T = Dp . F^T (Dp[y][k] = D[p_y][p_k]) tile by tile
//     on MFMA; goal = trace(A); for every pair x < y
//       delta = 2 (A_xy + A_yx - A_xx - A_yy)
//               + (2 f_xy - f_xx - f_yy)(2 Dp_xy - Dp_xx - Dp_yy)        (F, D symmetric)
//     or, in general, with B = F^T . Dp' on (F^T, D^T):
//       delta = A_xy + A_yx + B_xy + B_yx - (A_xx + B_xx) - (A_yy + B_yy) - kappa + lambda;
//     the lexicographically first minimum (delta, x, y) is applied if < 0.
//  D. X(t+1), goal, P^L.
#include "dword.hpp"
#include "kernels.hpp"
#include "second_target.hpp"

namespace qap {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

namespace {

constexpr int kWaves = 4;  // particles (waves) per workgroup of the evaluation kernels

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS row stride of the n x n int8 matrices: 16 bytes of padding put the 16-byte
// fragments of 8 consecutive rows in 8 distinct 4-bank groups (conflict-free
// ds_read_b128).
template <int NP>
constexpr int lds_stride() { return NP + 16; }

// D and D^T are only gathered byte-wise (and read at single cells), which
// padding does not help: they keep the unpadded stride.
template <int NP>
constexpr int lds_stride_d() { return NP; }

// 16 bytes Mt[p[kb + j]][py], j = 0..15, packed little-endian into 4 ints:
// with Mt the transpose of M this is M[py][p[kb + j]].  For a fixed j every
// lane of a half-wave reads the same row (kb does not depend on the lane) at
// its own column, which spreads the byte reads over the banks; reading row py
// of M instead would send all 32 lanes to one bank.
template <int LS>
__device__ __forceinline__ v4i gather16(const int8_t* Mt, int py, const uint8_t* p, int kb)
{
    const v4i pk = *reinterpret_cast<const v4i*>(p + kb);
    const uint8_t* col = reinterpret_cast<const uint8_t*>(Mt) + py;
    v4i out;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t word = (uint32_t)pk[w];
        uint32_t r = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) r |= (uint32_t)col[((word >> (8 * b)) & 0xffu) * LS] << (8 * b);
        out[w] = (int)r;
    }
    return out;
}

template <int LS>
__device__ __forceinline__ v4i frag16(const int8_t* M, int row, int kb)
{
    return *reinterpret_cast<const v4i*>(M + row * LS + kb);
}

__device__ __forceinline__ v16i mfma32(v4i a, v4i b, v16i c)
{
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// acc element i of lane l in a 32x32 tile: row 8(i/4) + 4(l/32) + i%4, column l%32
__device__ __forceinline__ int tile_row(int i, int h) { return 8 * (i >> 2) + 4 * h + (i & 3); }

// Row info per index x: p_x and the diagonal term dA_x (A_xx when F and D are
// symmetric, else A_xx + B_xx); f_xx and Dp_xx are read from the matrices.
struct RowInfo {
    int p, da;
};

// Stage C for one permutation held in LDS (sp, NP bytes, entries >= n are 0).
// Returns the goal; bestkey = (delta << 16) | (x << 8) | y of the first
// minimum pair (LLONG_MAX if n < 2).  If dout != NULL every delta is written.
template <int NP, bool SYM, bool ZD>
__device__ void goal_delta_mfma(int n, const int8_t* sF, const int8_t* sD, const int8_t* sFT, const int8_t* sDT,
                                const uint8_t* sp, RowInfo* sri, bool want_pairs, long long* dout, long long& goal,
                                long long& bestkey)
{
    constexpr int T = NP / 32, LS = lds_stride<NP>(), LSD = lds_stride_d<NP>();
    const int l = lane_id(), h = l >> 5, lc = l & 31;
    // Dp (and Dp' for the general case) fragments for every (block, K chunk):
    // Dp[y][k] = D[p_y][p_k] = D^T[p_k][p_y], Dp'[y][k] = D^T[p_y][p_k] = D[p_k][p_y]
    v4i dp[T][T];
    v4i dpt[SYM ? 1 : T][SYM ? 1 : T];
#pragma unroll
    for (int b = 0; b < T; ++b) {
        const int y = 32 * b + lc;
        const int py = y < n ? (int)sp[y] : 0;
#pragma unroll
        for (int kc = 0; kc < T; ++kc) {
            dp[b][kc] = y < n ? gather16<LSD>(SYM ? sD : sDT, py, sp, 32 * kc + 16 * h) : v4i{0, 0, 0, 0};
            if constexpr (!SYM) dpt[b][kc] = y < n ? gather16<LSD>(sD, py, sp, 32 * kc + 16 * h) : v4i{0, 0, 0, 0};
        }
    }
    // diagonal terms: A_xx = sum_k F[x][k] Dp[x][k] (and B_xx) as a dot product of
    // the lane's own fragments (4 int8 products per instruction), the two half-waves'
    // K halves added across; row info, goal = trace(A); int8 entries and n <= 160
    // bound |goal| by 160^2 * 127^2 < 2^31
    int gsum = 0;
#pragma unroll
    for (int a = 0; a < T; ++a) {
        int da = 0, db = 0;
#pragma unroll
        for (int kc = 0; kc < T; ++kc) {
            const v4i f = frag16<LS>(sF, 32 * a + lc, 32 * kc + 16 * h);
#pragma unroll
            for (int w = 0; w < 4; ++w) da = __builtin_amdgcn_sdot4(f[w], dp[a][kc][w], da, false);
            if constexpr (!SYM) {
                const v4i g = frag16<LS>(sFT, 32 * a + lc, 32 * kc + 16 * h);
#pragma unroll
                for (int w = 0; w < 4; ++w) db = __builtin_amdgcn_sdot4(g[w], dpt[a][kc][w], db, false);
            }
        }
        da += __shfl_xor(da, 32, kWave);
        if constexpr (!SYM) db += __shfl_xor(db, 32, kWave);
        if (h == 0) {
            const int x = 32 * a + lc;
            if (x < n) {
                gsum += da;
                const int px = sp[x];
                RowInfo ri;
                ri.p = px;
                ri.da = SYM ? da : da + db;
                sri[x] = ri;
            }
        }
    }
    goal = wave_sum_i32(gsum);
    bestkey = LLONG_MAX;
    if (!want_pairs) return;
    wave_sync();
    // all tiles a <= b
#pragma unroll
    for (int a = 0; a < T; ++a) {
#pragma unroll
        for (int b = a; b < T; ++b) {
            const int y = 32 * b + lc;
            // symmetric F, D: A holds A + A^T on the tile (the deltas need only the sum)
            v16i A = {}, AT = {}, B = {}, BT = {};
#pragma unroll
            for (int kc = 0; kc < T; ++kc) {
                const v4i fa = frag16<LS>(sF, 32 * a + lc, 32 * kc + 16 * h);
                const v4i fb = frag16<LS>(sF, 32 * b + lc, 32 * kc + 16 * h);
                A = mfma32(fa, dp[b][kc], A);            // A[x][y]  = sum_k F[x][k] Dp[y][k]
                if constexpr (SYM)
                    A = mfma32(dp[a][kc], fb, A);        // + A^T[x][y] = sum_k Dp[x][k] F[y][k] = A[y][x]
                else
                    AT = mfma32(dp[a][kc], fb, AT);
                if constexpr (!SYM) {
                    const v4i ga = frag16<LS>(sFT, 32 * a + lc, 32 * kc + 16 * h);
                    const v4i gb = frag16<LS>(sFT, 32 * b + lc, 32 * kc + 16 * h);
                    B = mfma32(ga, dpt[b][kc], B);
                    BT = mfma32(dpt[a][kc], gb, BT);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            if (y >= n) continue;
            const RowInfo cy = sri[y];
            const int cyf = (SYM && ZD) ? 0 : sF[y * (LS + 1)];             // f_yy
            const int cyd = (SYM && ZD) ? 0 : sD[__umul24(cy.p, LSD + 1)];  // Dp_yy
            // lane rows x = 32a + 4h + xo(i), xo(i) = 8(i/4) + i%4, increasing in i:
            // the first strict minimum over i is the lexicographic (delta, x) minimum
            const RowInfo* rxb = sri + 32 * a + 4 * h;
            const int8_t* fxb = sF + (32 * a + 4 * h) * LS + y;
            const int8_t* fyb = sF + y * LS + 32 * a + 4 * h;
            // ZD: the minimum is taken over hdel = (A_xy + A_yx - A_xx) + 2 f_xy Dp_xy,
            // delta = 2 (hdel - A_yy): increasing in hdel, so the same first minimum.
            // The minimum is kept as one int, delta * 16 + i (|delta| < 2^26 for int8
            // entries and n <= 160): the smallest delta, then the first element.
            int tkey = INT_MAX;
            // the row info of the next element is read while this one is
            // evaluated: the D read indexed by p_x then waits for one LDS round
            // trip per element instead of two
            RowInfo rxn = rxb[0];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int xo = 8 * (i >> 2) + (i & 3);
                const RowInfo rx = rxn;
                if (i + 1 < 16) rxn = rxb[8 * ((i + 1) >> 2) + ((i + 1) & 3)];
                if (a == b && 32 * a + 4 * h + xo >= y) {  // diagonal tiles: x < y only
                    __builtin_amdgcn_sched_barrier(0);
                    continue;
                }
                const int fxy = fxb[xo * LS];
                const int dxy = sD[__umul24(rx.p, LSD) + cy.p];  // 24-bit multiply: p < 256
                int del;
                if constexpr (SYM && ZD) {
                    del = A[i] - rx.da + 2 * fxy * dxy;
                } else if constexpr (SYM) {
                    const int rxf = sF[(32 * a + 4 * h + xo) * (LS + 1)], rxd = sD[__umul24(rx.p, LSD + 1)];
                    del = 2 * (A[i] - rx.da - cy.da) + (2 * fxy - rxf - cyf) * (2 * dxy - rxd - cyd);
                } else {
                    const int fyx = fyb[xo];
                    const int dyx = sD[__umul24(cy.p, LSD) + rx.p];
                    const int faa = sF[(32 * a + 4 * h + xo) * (LS + 1)], fbb = cyf;
                    const int daa = sD[__umul24(rx.p, LSD + 1)], dbb = cyd;
                    const int kap = (faa - fyx) * (dyx - daa) + (fxy - fbb) * (dbb - dxy) + (faa - fxy) * (dxy - daa) +
                                    (fyx - fbb) * (dbb - dyx);
                    const int lam = (faa - fbb) * (dbb - daa) + (fxy - fyx) * (dyx - dxy);
                    del = A[i] + AT[i] + B[i] + BT[i] - rx.da - cy.da - kap + lam;
                }
                if (dout) {
                    const int x = 32 * a + 4 * h + xo;
                    const int full = (SYM && ZD) ? 2 * (del - cy.da) : del;
                    dout[(size_t)x * n + y] = full;
                    dout[(size_t)y * n + x] = full;
                }
                tkey = min(tkey, (int)((uint32_t)del << 4) | i);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (tkey != INT_MAX) {
                int tmin = tkey >> 4;
                const int ti = tkey & 15;
                if constexpr (SYM && ZD) tmin = 2 * (tmin - cy.da);
                // (delta, x, y) as one ordered 64-bit key: delta * 2^16 + x * 2^8 + y
                const int x = 32 * a + 4 * h + 8 * (ti >> 2) + (ti & 3);
                const long long key = ((long long)tmin << 16) | (x << 8) | y;
                bestkey = key < bestkey ? key : bestkey;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    bestkey = wave_min_i64(bestkey);
}

template <int NP, bool SYM>
__device__ __forceinline__ void load_instance_lds(const InstDesc& d, int8_t* sF, int8_t* sD, int8_t* sFT, int8_t* sDT)
{
    constexpr int LS = lds_stride<NP>(), LSD = lds_stride_d<NP>(), RV = NP / 16;  // 16-byte chunks per row
    global_t<const v4i>* F = reinterpret_cast<global_t<const v4i>*>(gl(d.F8));
    global_t<const v4i>* D = reinterpret_cast<global_t<const v4i>*>(gl(d.D8));
    for (int i = threadIdx.x; i < NP * RV; i += blockDim.x) {
        const int o = (i / RV) * LS + 16 * (i % RV), od = (i / RV) * LSD + 16 * (i % RV);
        *reinterpret_cast<v4i*>(sF + o) = F[i];
        *reinterpret_cast<v4i*>(sD + od) = D[i];
        if constexpr (!SYM) {
            *reinterpret_cast<v4i*>(sFT + o) = reinterpret_cast<global_t<const v4i>*>(gl(d.FT8))[i];
            *reinterpret_cast<v4i*>(sDT + od) = reinterpret_cast<global_t<const v4i>*>(gl(d.DT8))[i];
        }
    }
}

// Clamp to [-vmax, vmax] (S_v); values are finite, so med3 is the clamp.
__device__ __forceinline__ float clampv(float t, float vmax) { return __builtin_amdgcn_fmed3f(t, -vmax, vmax); }

// Rows of X, P^L and P^G in one column and their attraction terms (velocity
// equation) as double words: row xr gets ox = s2 ax + s3 bx (ax, bx in
// {-1, 0}), row lr (!= xr) ol = s2 + s3 bl (bl in {0, 1}), row gr (!= xr, lr)
// s3; every other row none.  s2 = c2 r2 and s3 = c3 r3 are exact double words
// (two_prod), their sum within 3u^2 of exact.
struct Attract {
    int xr, lr, gr;
    DW ox, ol;
};

// An attraction cell: c1 x + o with c1 x an exact double word, added to o by
// the accurate double-word sum and rounded once to binary32, then clamped
// (S_v).  Rounding c1 x, c2 r2 and c3 r3 separately before the terms cancel
// could leave an error that is large next to the result; this way the result
// is within about one unit of 2^-24 of the exact value, relative to itself.
__device__ __forceinline__ float attract_cell(float c1, float x, DW o, float vmax)
{
    return clampv(dw_add(two_prod(c1, x), o).hi, vmax);
}

// Buffer resource over one particle's n x n matrix (raw, 32-bit elements):
// row offsets go to the scalar offset, the lane's column to the vector one.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t matrix_rsrc(const float* p, int n)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, 4 * n * n, 0x00020000);
}

__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}

// The attraction cells among rows [lo, hi) of column c: ex, el, eg are the
// raw V(t) values at rows xr, lr, gr (read only where the row is in range).
// Each is stored after the plain value of the same cell by the same lane
// (program order) and replaces that value in the column sum (a double word:
// the attraction value added, the plain one taken off, both without loss).
// X: whether the X-row cell is handled here too (else it was stored already).
template <bool X>
__device__ __forceinline__ void fix_cells(__amdgpu_buffer_rsrc_t rq, uint32_t col, uint32_t rowb, int lo, int hi,
                                          const Attract& at, float ex, float el, float eg, float sc, float c1,
                                          DW s3, float vmax, DW& sum, float& vx)
{
    if (X && at.xr >= lo && at.xr < hi) {
        const float x = __fmul_rn(ex, sc);
        vx = x;
        // no attraction term (rows of X, P^L and P^G equal): the plain value
        // stands (a re-store would cost a partial write of its line)
        if (at.ox.hi != 0.0f) {
            const float t = attract_cell(c1, x, at.ox, vmax);
            sum = dw_add_f(dw_add_f(sum, fabsf(t)), -fabsf(clampv(__fmul_rn(c1, x), vmax)));
            bstore(rq, col + __umul24(at.xr, rowb), 0u, t);
        }
    }
    if (at.lr != at.xr && at.lr >= lo && at.lr < hi) {
        const float x = __fmul_rn(el, sc);
        const float t = attract_cell(c1, x, at.ol, vmax);
        sum = dw_add_f(dw_add_f(sum, fabsf(t)), -fabsf(clampv(__fmul_rn(c1, x), vmax)));
        bstore(rq, col + __umul24(at.lr, rowb), 0u, t);
    }
    if (at.gr != at.xr && at.gr != at.lr && at.gr >= lo && at.gr < hi) {
        const float x = __fmul_rn(eg, sc);
        const float t = attract_cell(c1, x, s3, vmax);
        sum = dw_add_f(dw_add_f(sum, fabsf(t)), -fabsf(clampv(__fmul_rn(c1, x), vmax)));
        bstore(rq, col + __umul24(at.gr, rowb), 0u, t);
    }
}

// Running top two of a column: m1 = max, m2 = runner-up (the middle of m1,
// m2 and x), u1 = position of the first strict rise of m1 (values finite).
// Written as compare/select so that the compiler neither canonicalises nor
// materialises the position: u is a small inline constant.
__device__ __forceinline__ void top2(float x, int u, float& m1, int& u1, float& m2)
{
    const bool le = x <= m1;
    u1 = le ? u1 : u;
    m2 = __builtin_amdgcn_fmed3f(m1, m2, x);
    m1 = le ? m1 : x;
}

// The state of one column in the velocity pass: its attraction rows and
// which of them differ (packed: X row, P^L row, P^G row in bytes 0-2; bit 24
// P^L row != X row, bit 25 P^G row != X row, bit 26 P^L row == P^G row), the
// scale of V(t), the sum of |.| of the new column so far (a double word), the
// largest V(t) value m1 (first row r1), its runner-up m2, and vx = V(t) at the
// X row.
struct ColStream {
    uint32_t rows;
    float sc;
    DW sum;
    float m1, m2, vx;
    int r1;
};

// The attraction rows and terms of a column (velocity equation) from its
// packed rows and the particle's s2 = c2 r2, s3 = c3 r3 and s23 = s2 + s3:
// ox = -(s2 if the P^L row differs) - (s3 if the P^G row differs),
// ol = s2 (+ s3 if the P^G row is the P^L row).
__device__ __forceinline__ Attract unpack_attract(uint32_t rows, DW s2, DW s3, DW s23)
{
    Attract at;
    at.xr = (int)(rows & 0xffu);
    at.lr = (int)((rows >> 8) & 0xffu);
    at.gr = (int)((rows >> 16) & 0xffu);
    const bool nl = (rows >> 24) & 1u, ng = (rows >> 25) & 1u;
    const DW o = nl && ng ? s23 : nl ? s2 : ng ? s3 : DW{0.0f, 0.0f};
    at.ox = dw_neg(o);
    at.ol = (rows >> 26) & 1u ? s23 : s2;
    return at;
}

// Rows [r0, min(r0 + B, n)) of the column at byte offset col of the velocity
// pass over one particle's V(t) (rp) into V(t+1) before the column norm (rq).
// The batch is summed in binary32 as four interleaved partial sums of B / 4,
// then added to the column's double word with the attraction-cell
// corrections, without loss: the column sum, rounded once at the end, has a
// relative error of at most 9 units of 2^-24 at any n (B = 32; 5 at B = 16),
// where one binary32 running sum could reach n - 1.  The B loads of a batch
// are issued together, and the attraction cells of the batch are read with it
// and fixed right after it.
// TAIL: the last rows, fewer than B (row indices clamped to the matrix, the
// rows past n skipped by uniform branches).
// FOLDX: the X-row cell by a select (at npad >= 128, where it costs no
// registers), else re-stored like the others.
template <int B, bool FOLDX, bool TAIL>
__device__ __forceinline__ void stream_batch(__amdgpu_buffer_rsrc_t rp, __amdgpu_buffer_rsrc_t rq, uint32_t col,
                                             uint32_t rowb, int n, int r0, float c1, DW s2, DW s3, DW s23,
                                             float vmax, ColStream& cs)
{
    const Attract at = unpack_attract(cs.rows, s2, s3, s23);
    const int hi = TAIL ? n : r0 + B;
    float v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) v[u] = bload(rp, col, (uint32_t)(TAIL ? min(r0 + u, n - 1) : r0 + u) * rowb);
    // attraction rows of this batch (row r0 stands in for absent ones: same lines)
    const float ex = bload(rp, col + __umul24(at.xr >= r0 && at.xr < hi ? at.xr : r0, rowb), 0u);
    const float el = bload(rp, col + __umul24(at.lr >= r0 && at.lr < hi ? at.lr : r0, rowb), 0u);
    const float eg = bload(rp, col + __umul24(at.gr >= r0 && at.gr < hi ? at.gr : r0, rowb), 0u);
    // the X-row cell (one in every column) takes its attraction value by a
    // select before the row's single store; the P^L and P^G cells (which
    // equal the X row or each other more and more often late in a run) are
    // re-stored after the batch: a second store to a line just written
    // leaves L2 as a partial write of its own, and three selects per row
    // would cost the registers of a wave per SIMD
    const float tx = attract_cell(c1, __fmul_rn(ex, cs.sc), at.ox, vmax);
    const int dx = FOLDX ? at.xr - r0 : -1;
    if (FOLDX && dx >= 0 && dx < B) cs.vx = __fmul_rn(ex, cs.sc);
    const float mb = cs.m1;
    int u1 = 0;
    float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // rows u = 0, 1, 2, 3 mod 4
#pragma unroll
    for (int u = 0; u < B; ++u) {
        if (!TAIL || u < n - r0) {
            const float x = __fmul_rn(v[u], cs.sc);
            top2(x, u, cs.m1, u1, cs.m2);
            float t = clampv(__fmul_rn(c1, x), vmax);
            if constexpr (FOLDX) t = u == dx ? tx : t;
            bstore(rq, col, (uint32_t)(r0 + u) * rowb, t);
            part[u & 3] = __fadd_rn(part[u & 3], fabsf(t));
        }
    }
    cs.sum = dw_add_f(cs.sum, __fadd_rn(__fadd_rn(part[0], part[1]), __fadd_rn(part[2], part[3])));
    cs.r1 = cs.m1 != mb ? r0 + u1 : cs.r1;  // the maximum rose in this batch
    fix_cells<!FOLDX>(rq, col, rowb, r0, hi, at, ex, el, eg, cs.sc, c1, s3, vmax, cs.sum, cs.vx);
}

}  // namespace

// ------------------------------------------------------------------ fused step
// Stages A and B of particle k (one wave): V(t+1) and its column scale
// written, X(t+1) of SecondTarget (before the exchanges) left in pw, whose
// entries n .. NP-1 are zeroed.  Returns the parity of the current buffers.
template <int NP, int CPL>
__device__ __forceinline__ int velocity_and_target(const InstDesc& d, int k, uint8_t* pw, StLds<CPL>* sl)
{
    const int l = lane_id();
    const int n = d.n;
    const int tprev = *gl(d.iter);
    const uint32_t tau = (uint32_t)tprev + 1u;
    const int cur = tprev & 1;
    const int gs = k / d.S;  // swarm within this descriptor; g: within the instance
    const uint32_t g = (uint32_t)(gs + d.swarm_base), s = (uint32_t)(k % d.S);
    global_t<const float>* Vp = gl(buf(d.V, cur)) + (size_t)k * n * n;
    float* Vq = buf(d.V, cur ^ 1) + (size_t)k * n * n;  // buffer stores
    global_t<const uint8_t>* Xk = gl(buf(d.X, cur)) + (size_t)k * n;
    const Philox4 rb = philox4x32_10(0u, tau, s, g, (uint32_t)d.seed, (uint32_t)(d.seed >> 32));
    // c2 r2, c3 r3 (exact double words) and their sum: the attraction terms
    const DW s2 = two_prod(d.c2, unit_float(rb.w[0]));
    const DW s3 = two_prod(d.c3, unit_float(rb.w[1]));
    const DW s23 = dw_add(s2, s3);
    const float c1 = d.c1, vmax = d.vmax;

    // ---- A. velocity stream + SecondTarget caches
    global_t<const float>* Sp = gl(buf(d.Vinv, cur)) + (size_t)k * n;
    global_t<float>* Sq = gl(buf(d.Vinv, cur ^ 1)) + (size_t)k * n;
    const __amdgpu_buffer_rsrc_t rp = matrix_rsrc((const float*)Vp, n), rq = matrix_rsrc(Vq, n);
    StState<CPL> st;
    st.rowbits = 0;
#pragma unroll
    for (int j = 0; j < CPL; ++j)
        if (l + kWave * j < n) st.rowbits |= 1u << j;
    // The lane's columns l, l + 64, ...  Rows are n floats, unpadded, so the
    // line holding the end of one row and the start of the next is shared by
    // the lane's columns: with several columns per lane the pass runs over
    // batches of 16 rows, each batch through every column before the next, so
    // that such a line is fetched once (a pass per column over the whole
    // matrix fetched it twice, the second time after eviction).  16-row
    // batches keep two columns' state within the registers of one 32-row
    // batch.  With one column per lane a row is one load: batches of 32.
    ColStream cs[CPL];
#pragma unroll
    for (int kk = 0; kk < CPL; ++kk) {
        const int c = l + kWave * kk;
        ColStream& z = cs[kk];
        z.m1 = -INFINITY; z.m2 = -INFINITY; z.vx = 0.0f; z.r1 = -1;
        z.sum = DW{0.0f, 0.0f};
        z.rows = 0u;
        z.sc = 1.0f;
        if (c < n) {
            const uint32_t xr = Xk[c], lr = gl(d.PL)[(size_t)k * n + c], gr = gl(d.PG)[(size_t)gs * n + c];
            z.rows = xr | lr << 8 | gr << 16 | (uint32_t)(lr != xr) << 24 | (uint32_t)(gr != xr) << 25 |
                     (uint32_t)(lr == gr) << 26;
            z.sc = Sp[c];
        }
    }
    constexpr bool FOLDX = NP >= 128;
    const uint32_t rowb = 4u * (uint32_t)n;
    if constexpr (CPL == 1) {
        if (l < n) {
            int r0 = 0;
            for (; r0 + 32 <= n; r0 += 32)
                stream_batch<32, FOLDX, false>(rp, rq, 4u * l, rowb, n, r0, c1, s2, s3, s23, vmax, cs[0]);
            if (r0 < n) stream_batch<32, FOLDX, true>(rp, rq, 4u * l, rowb, n, r0, c1, s2, s3, s23, vmax, cs[0]);
        }
    } else {
        constexpr int RB = 16;
        int r0 = 0;
        for (; r0 + RB <= n; r0 += RB) {
#pragma unroll
            for (int kk = 0; kk < CPL; ++kk) {
                if (l + kWave * kk < n)
                    stream_batch<RB, FOLDX, false>(rp, rq, 4u * (uint32_t)(l + kWave * kk), rowb, n, r0, c1, s2, s3,
                                                   s23, vmax, cs[kk]);
                __builtin_amdgcn_sched_barrier(0);  // one column's batch at a time
            }
        }
        if (r0 < n) {
#pragma unroll
            for (int kk = 0; kk < CPL; ++kk) {
                if (l + kWave * kk < n)
                    stream_batch<RB, FOLDX, true>(rp, rq, 4u * (uint32_t)(l + kWave * kk), rowb, n, r0, c1, s2, s3,
                                                  s23, vmax, cs[kk]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
#pragma unroll
    for (int kk = 0; kk < CPL; ++kk) {
        const int c = l + kWave * kk;
        const bool on = c < n;
        const ColStream& z = cs[kk];
        const int xr = (int)(z.rows & 0xffu);
        const float m1 = z.m1, m2 = z.m2;
        const int r1 = z.r1;
        if (on) {
            const float sum = __fadd_rn(z.sum.hi, z.sum.lo);
            Sq[c] = (d.norm && sum > 0.0f) ? __fdiv_rn(1.0f, sum) : 1.0f;
        }
        // SecondTarget cache of the non-Z keys: exact (value, row, count 1)
        // when the column maximum is unique and off the Z row; the runner-up
        // value bounds it when the maximum sits on the Z row
        if (on && r1 != xr && m2 < m1) {
            st.nzv[kk] = m1; st.nzr[kk] = r1; st.nzc[kk] = 1; st.stale[kk] = false;
        } else {
            st.nzv[kk] = on ? (r1 == xr ? m2 : m1) : -INFINITY;
            st.nzr[kk] = -1; st.nzc[kk] = 0; st.stale[kk] = on;
        }
        st.cal[kk] = on;
        st.zal[kk] = on;
        st.zr[kk] = on ? xr : -1;
        st.zk[kk] = on ? 1.0f + z.vx : -INFINITY;
    }

    // ---- B. SecondTarget
    for (int j = n + l; j < NP; j += kWave) pw[j] = 0;
    st_select<CPL>(n, d.depth, Vp, Sp, st, pw, sl, d.seed, tau, s, g);
    wave_sync();
    return cur;
}

// Stage C: up to d.ls best-improvement exchanges on pw.  contract(goal, key)
// evaluates pw: its goal and the key (delta << 16 | a << 8 | b) of the first
// minimum pair.  Each exchange found while more are allowed is made in place
// and the deltas recomputed; the last allowed one is returned in (ba, bb), with
// goal including it (ba = -1 if none).
template <class Contract>
__device__ __forceinline__ void exchanges(const InstDesc& d, uint8_t* pw, Contract contract, long long& goal,
                                          int& ba, int& bb)
{
    long long key;
    int swaps = 0;
    for (;;) {
        contract(goal, key);
        if (d.ls <= swaps + 1 || key == LLONG_MAX || (key >> 16) >= 0) break;
        if (lane_id() == 0) {
            const int a = (int)((key >> 8) & 0xff), b = (int)(key & 0xff);
            const uint8_t t = pw[a];
            pw[a] = pw[b];
            pw[b] = t;
        }
        wave_sync();
        ++swaps;
    }
    ba = -1;
    bb = -1;
    if (d.ls > swaps && key != LLONG_MAX) {
        const long long del = key >> 16;
        if (del < 0) {
            ba = (int)((key >> 8) & 0xff);
            bb = (int)(key & 0xff);
            goal += del;
        }
    }
}

// Stage D: X(t+1) (pw with a, b exchanged), goal, P^L.
__device__ __forceinline__ void write_particle(const InstDesc& d, int k, int cur, const uint8_t* pw, long long goal,
                                               int ba, int bb)
{
    const int n = d.n, l = lane_id();
    global_t<uint8_t>* Xo = gl(buf(d.X, cur ^ 1)) + (size_t)k * n;
    global_t<uint8_t>* PL = gl(d.PL);
    global_t<long long>* gpl = gl(d.goalPL);
    const bool improve = goal < gpl[k];
    for (int j = l; j < n; j += kWave) {
        uint8_t v = pw[j];
        if (j == ba) v = pw[bb];
        if (j == bb) v = pw[ba];
        Xo[j] = v;
        if (improve) PL[(size_t)k * n + j] = v;
    }
    if (l == 0) {
        gl(d.goal)[k] = goal;
        if (improve) gpl[k] = goal;
    }
}

template <int NP>
constexpr int cols_per_lane() { return NP <= 64 ? 1 : NP <= 128 ? 2 : 4; }

// WPB particles (waves) per workgroup, sharing one LDS copy of F and D (see
// fused_wpb).  TABLE: workgroup b steps particles blkmap[b].y ..
// + WPB - 1 of instance descs[blkmap[b].x] (its pointers marked global where
// they are used, see gl); otherwise workgroup b steps particles WPB b .. of
// the instance passed as `one` (a kernel argument, whose pointers the
// compiler knows to be global).
// One workgroup of k_fused_step: particles first .. first + WPB - 1 of d.
template <int NP, bool SYM, bool ZD, int WPB>
__device__ __forceinline__ void fused_step_block(const InstDesc& d, int first)
{
    constexpr int CPL = cols_per_lane<NP>();  // column slots per lane
    __shared__ __attribute__((aligned(16))) int8_t sF[NP * lds_stride<NP>()];
    __shared__ __attribute__((aligned(16))) int8_t sD[NP * lds_stride_d<NP>()];
    __shared__ __attribute__((aligned(16))) int8_t sFT[SYM ? 16 : NP * lds_stride<NP>()];
    __shared__ __attribute__((aligned(16))) int8_t sDT[SYM ? 16 : NP * lds_stride_d<NP>()];
    __shared__ __attribute__((aligned(16))) uint8_t sp[WPB][NP];
    // per wave: the selection scratch of stage B, then the row info of stage C
    union WaveScratch {
        StLds<CPL> st;
        RowInfo ri[NP];
    };
    __shared__ WaveScratch sws[WPB];
    load_instance_lds<NP, SYM>(d, sF, sD, sFT, sDT);
    __syncthreads();

    // wave index made explicitly uniform: every per-particle address lives in scalar registers
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int k = first + w;
    if (k >= d.P) return;
    uint8_t* pw = sp[w];
    const int cur = velocity_and_target<NP, CPL>(d, k, pw, &sws[w].st);
    long long goal;
    int ba, bb;
    exchanges(d, pw, [&](long long& g, long long& key) {
        goal_delta_mfma<NP, SYM, ZD>(d.n, sF, sD, sFT, sDT, pw, sws[w].ri, d.ls != 0, nullptr, g, key);
    }, goal, ba, bb);
    write_particle(d, k, cur, pw, goal, ba, bb);
}

// Waves per SIMD the register allocation is held to (amdgpu_waves_per_eu).
// Without it the compiler set 16 accumulation registers aside for the MFMA
// results of the symmetric kernels on top of their VGPRs, which cost the
// npad-96 kernels a wave per SIMD; with it those results stay in VGPRs.  The
// general (asymmetric) kernels keep their 64 accumulation registers.
template <int NP, bool SYM, bool ZD>
constexpr int fused_min_waves() { return !SYM ? 1 : NP <= 96 ? 5 : NP == 128 ? 4 : 3; }

template <int NP, bool SYM, bool ZD, bool TABLE, int WPB>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(fused_min_waves<NP, SYM, ZD>())))
void k_fused_step(InstDesc one, const InstDesc* __restrict__ descs,
                                                         const int2* __restrict__ blkmap)
{
    if constexpr (TABLE) {
        const int2 bm = blkmap[blockIdx.x];
        fused_step_block<NP, SYM, ZD, WPB>(descs[__builtin_amdgcn_readfirstlane(bm.x)],
                                           __builtin_amdgcn_readfirstlane(bm.y));
    } else {
        fused_step_block<NP, SYM, ZD, WPB>(one, (int)blockIdx.x * WPB);
    }
}

// ------------------------------------------------------------------ wide step
// Byte-split contraction for symmetric instances whose F or D leave the int8
// range.  Each matrix M that needs it is split as M = 128 M_hi + M_lo with
// M_lo in [0, 127] and M_hi = floor(M / 128) in [-128, 127] (|M| <= 16383); a
// matrix that fits int8 keeps its value in the low plane.  Every product of
// planes is an exact int8 MFMA, and the products are combined by Horner's rule
// in int32: A = 128 (128 A_hh + A_hl + A_lh) + A_ll.
//
// Two equal ways to form A = F . Dp^T: (form 0) F rows direct from LDS and
// Dp[y][k] = D[p_y][p_k] gathered; (form 1) D rows p_x direct and
// Fq[y][l] = F[y][q_l] gathered, q = p^-1, since A[x][y] = sum_l F[x][q_l]
// D[p_y][l].  The gathered operand is held in registers for every block; form
// 1 is taken when only D is split, so that the held operand stays one plane.
// Both matrices split (SPLIT 3) holds two planes: twice the registers.
// SPLIT, the split pattern, is a template parameter (bit 0: F split, bit 1: D
// split), so the plane reads of the pair scan carry no branches.
// For symmetric F and D the deltas use A_xy + A_yx only, which both forms
// accumulate in one tile.

// Row info of the wide path: f_xx, Dp_xx and the diagonal sum 2 A_xx.
struct RowW {
    short f, dp;
    int da;
};

template <int NP, int CPL>
struct WideWaveLds {
    uint8_t p[NP];
    uint8_t q[NP];
    union {
        StLds<CPL> st;   // stage B
        RowW ri[NP];     // stage C
    } u;
};

// Byte planes of the wide path in LDS, NP rows of lds_stride bytes each.
// Both matrices split: F low, F high, D low, D high.  One matrix split: three
// planes, the split matrix's low and high planes first, then the other
// matrix's low plane.  The high plane of a split matrix lies one plane after
// its low plane.
template <int SPLIT>
constexpr int wide_planes() { return SPLIT == 3 ? 4 : 3; }

// Offsets of F's and D's low planes.
template <int NP, int SPLIT>
constexpr int wide_f_off() { return SPLIT == 2 ? 2 * NP * lds_stride<NP>() : 0; }
template <int NP, int SPLIT>
constexpr int wide_d_off() { return SPLIT == 2 ? 0 : 2 * NP * lds_stride<NP>(); }

template <int NP, int SPLIT>
__device__ __forceinline__ void load_wide_lds(const InstDesc& d, int8_t* pl)
{
    constexpr int LS = lds_stride<NP>(), PS = NP * LS, RV = NP / 16;
    int8_t* fl = pl + wide_f_off<NP, SPLIT>();
    int8_t* dl = pl + wide_d_off<NP, SPLIT>();
    global_t<const v4i>* src[4] = {reinterpret_cast<global_t<const v4i>*>(gl(d.F8)), reinterpret_cast<global_t<const v4i>*>(gl(d.FH8)),
                                   reinterpret_cast<global_t<const v4i>*>(gl(d.D8)), reinterpret_cast<global_t<const v4i>*>(gl(d.DH8))};
    int8_t* dst[4] = {fl, fl + PS, dl, dl + PS};
    constexpr bool on[4] = {true, (SPLIT & 1) != 0, true, (SPLIT & 2) != 0};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        if (!on[m]) continue;
        for (int i = threadIdx.x; i < NP * RV; i += blockDim.x)
            *reinterpret_cast<v4i*>(dst[m] + (i / RV) * LS + 16 * (i % RV)) = src[m][i];
    }
}

// Entry off of a matrix from its low plane (and, if SPLIT, the high plane PS
// bytes on).
template <int PS, bool SPLIT>
__device__ __forceinline__ int wide_val(const int8_t* lo, int off)
{
    int v = lo[off];
    if constexpr (SPLIT) v += 128 * (int)lo[off + PS];
    return v;
}

// Stage C of the wide path for one permutation sp (NP bytes, zero beyond n);
// sq receives q = p^-1 when form 1 is used.  Same results as goal_delta_mfma.
// SPLIT must equal the instance's split pattern.
template <int NP, bool ZD, int SPLIT>
__device__ void goal_delta_wide(int n, const int8_t* pl, const uint8_t* sp, uint8_t* sq, RowW* sri,
                                bool want_pairs, long long* dout, long long& goal, long long& bestkey)
{
    constexpr int T = NP / 32, LS = lds_stride<NP>(), PS = NP * LS;
    constexpr bool HS = SPLIT == 3;
    const int l = lane_id(), h = l >> 5, lc = l & 31;
    constexpr bool fs = (SPLIT & 1) != 0, ds = (SPLIT & 2) != 0;
    constexpr bool form = SPLIT == 2;
    const int8_t* fl = pl + wide_f_off<NP, SPLIT>();  // F, low plane (high plane PS bytes on)
    const int8_t* dl = pl + wide_d_off<NP, SPLIT>();  // D, likewise
    const int8_t* hl = form ? fl : dl;  // held (gathered) operand, low plane
    const int8_t* hh = hl + PS;
    const int8_t* rl = form ? dl : fl;  // direct operand, low plane
    const int8_t* rh = rl + PS;
    constexpr bool hs = HS;
    constexpr bool rs = form || fs;
    if constexpr (form) {
        for (int j = l; j < NP; j += kWave) {
            if (j < n) sq[sp[j]] = (uint8_t)j;
            else sq[j] = 0;
        }
        wave_sync();
    }
    const uint8_t* idx = form ? sq : sp;
    constexpr int TH = HS ? T : 1;
    v4i Hl[T][T], Hh[TH][TH];
#pragma unroll
    for (int b = 0; b < T; ++b) {
        const int y = 32 * b + lc;
        const int gy = y < n ? (form ? y : (int)sp[y]) : 0;
#pragma unroll
        for (int kc = 0; kc < T; ++kc) {
            Hl[b][kc] = y < n ? gather16<LS>(hl, gy, idx, 32 * kc + 16 * h) : v4i{0, 0, 0, 0};
            if constexpr (HS) Hh[b][kc] = y < n ? gather16<LS>(hh, gy, idx, 32 * kc + 16 * h) : v4i{0, 0, 0, 0};
        }
    }
    // direct operand row of lane index x
    auto drow = [&](int x) { return form ? (int)sp[x] : x; };
    // diagonal tiles: A_xx -> row info; goal = trace(A) in 64 bits
    long long gsum = 0;
#pragma unroll
    for (int a = 0; a < T; ++a) {
        const int ra = drow(32 * a + lc);
        v16i acc = {};
        if constexpr (HS) {
#pragma unroll
            for (int kc = 0; kc < T; ++kc) acc = mfma32(frag16<LS>(rh, ra, 32 * kc + 16 * h), Hh[a][kc], acc);
            acc *= 128;
        }
        if constexpr (rs) {
#pragma unroll
            for (int kc = 0; kc < T; ++kc) acc = mfma32(frag16<LS>(rh, ra, 32 * kc + 16 * h), Hl[a][kc], acc);
        }
        if constexpr (HS) {
#pragma unroll
            for (int kc = 0; kc < T; ++kc) acc = mfma32(frag16<LS>(rl, ra, 32 * kc + 16 * h), Hh[a][kc], acc);
        }
        if constexpr (rs || hs) acc *= 128;
#pragma unroll
        for (int kc = 0; kc < T; ++kc) acc = mfma32(frag16<LS>(rl, ra, 32 * kc + 16 * h), Hl[a][kc], acc);
        if (h == ((lc >> 2) & 1)) {
            const int want = 4 * (lc >> 3) + (lc & 3);
            int da = 0;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (i == want) da = acc[i];
            const int x = 32 * a + lc;
            if (x < n) {
                gsum += da;
                const int px = sp[x];
                RowW ri;
                ri.f = (short)wide_val<PS, fs>(fl, x * LS + x);
                ri.dp = (short)wide_val<PS, ds>(dl, px * LS + px);
                ri.da = 2 * da;
                sri[x] = ri;
            }
        }
    }
    goal = wave_sum_i64(gsum);
    bestkey = LLONG_MAX;
    if (!want_pairs) return;
    wave_sync();
#pragma unroll
    for (int a = 0; a < T; ++a) {
#pragma unroll
        for (int b = a; b < T; ++b) {
            const int y = 32 * b + lc;
            const int ra = drow(32 * a + lc), rb = drow(y);
            // acc = A + A^T on the tile (x in block a, y in block b)
            v16i acc = {};
            if constexpr (HS) {
#pragma unroll
                for (int kc = 0; kc < T; ++kc) {
                    acc = mfma32(frag16<LS>(rh, ra, 32 * kc + 16 * h), Hh[b][kc], acc);
                    acc = mfma32(Hh[a][kc], frag16<LS>(rh, rb, 32 * kc + 16 * h), acc);
                }
                acc *= 128;
            }
            if constexpr (rs) {
#pragma unroll
                for (int kc = 0; kc < T; ++kc) {
                    acc = mfma32(frag16<LS>(rh, ra, 32 * kc + 16 * h), Hl[b][kc], acc);
                    acc = mfma32(Hl[a][kc], frag16<LS>(rh, rb, 32 * kc + 16 * h), acc);
                }
            }
            if constexpr (HS) {
#pragma unroll
                for (int kc = 0; kc < T; ++kc) {
                    acc = mfma32(frag16<LS>(rl, ra, 32 * kc + 16 * h), Hh[b][kc], acc);
                    acc = mfma32(Hh[a][kc], frag16<LS>(rl, rb, 32 * kc + 16 * h), acc);
                }
            }
            if constexpr (rs || hs) acc *= 128;
#pragma unroll
            for (int kc = 0; kc < T; ++kc) {
                acc = mfma32(frag16<LS>(rl, ra, 32 * kc + 16 * h), Hl[b][kc], acc);
                acc = mfma32(Hl[a][kc], frag16<LS>(rl, rb, 32 * kc + 16 * h), acc);
            }
            __builtin_amdgcn_sched_barrier(0);
            if (y >= n) continue;
            const RowW cy = sri[y];
            const int py = sp[y];
            int tmin = INT_MAX, ti = 0;
            // the next element's row info and p_x are read while this one is
            // evaluated (one LDS round trip per element instead of two)
            RowW rxn = sri[32 * a + 4 * h];
            int pxn = sp[32 * a + 4 * h];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int xo = 8 * (i >> 2) + (i & 3);
                const int x = 32 * a + 4 * h + xo;
                const RowW rx = rxn;
                const int px = pxn;
                if (i + 1 < 16) {
                    const int xn = 32 * a + 4 * h + 8 * ((i + 1) >> 2) + ((i + 1) & 3);
                    rxn = sri[xn];
                    pxn = sp[xn];
                }
                if (a == b && x >= y) {  // diagonal tiles: x < y only
                    __builtin_amdgcn_sched_barrier(0);
                    continue;
                }
                const int fxy = wide_val<PS, fs>(fl, x * LS + y);
                const int dxy = wide_val<PS, ds>(dl, __umul24(px, LS) + py);
                const int base = 2 * acc[i] - rx.da - cy.da;
                int del;
                if constexpr (ZD)
                    del = base + 4 * fxy * dxy;
                else
                    del = base + (2 * fxy - rx.f - cy.f) * (2 * dxy - rx.dp - cy.dp);
                if (dout) {
                    dout[(size_t)x * n + y] = del;
                    dout[(size_t)y * n + x] = del;
                }
                const bool lt = del < tmin;
                tmin = lt ? del : tmin;
                ti = lt ? i : ti;
                // keep the running (minimum, index) pair in registers: otherwise
                // the compiler keeps all 16 deltas to recover the index at the end
                asm volatile("" : "+v"(tmin), "+v"(ti));
                __builtin_amdgcn_sched_barrier(0);
            }
            if (tmin != INT_MAX) {
                const int x = 32 * a + 4 * h + 8 * (ti >> 2) + (ti & 3);
                const long long key = ((long long)tmin << 16) | (x << 8) | y;
                bestkey = key < bestkey ? key : bestkey;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    bestkey = wave_min_i64(bestkey);
}

template <int NP, bool ZD, int SPLIT, int WPB>
__device__ __forceinline__ void fused_wide_block(const InstDesc& d, int first)
{
    constexpr int CPL = cols_per_lane<NP>();
    __shared__ __attribute__((aligned(16))) int8_t spl[wide_planes<SPLIT>() * NP * lds_stride<NP>()];
    __shared__ __attribute__((aligned(16))) WideWaveLds<NP, CPL> sw[WPB];
    load_wide_lds<NP, SPLIT>(d, spl);
    __syncthreads();

    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int k = first + w;
    if (k >= d.P) return;
    uint8_t* pw = sw[w].p;
    const int cur = velocity_and_target<NP, CPL>(d, k, pw, &sw[w].u.st);
    wave_sync();  // stage B's scratch is reused for the row info
    long long goal;
    int ba, bb;
    exchanges(d, pw, [&](long long& g, long long& key) {
        goal_delta_wide<NP, ZD, SPLIT>(d.n, spl, pw, sw[w].q, sw[w].u.ri, d.ls != 0, nullptr, g, key);
    }, goal, ba, bb);
    write_particle(d, k, cur, pw, goal, ba, bb);
}

// Waves per SIMD the register allocation of the byte-split kernels is held to
// (as for k_fused_step).
template <int NP, bool ZD, int SPLIT, int WPB>
constexpr int wide_min_waves()
{
    return SPLIT == 3 ? (NP <= 32 ? 5 : NP == 64 ? 4 : NP == 96 ? 3 : 2)
                      : (NP <= 64 ? 5 : NP == 96 ? 4 : NP == 128 ? (WPB == 8 ? 4 : 3) : 2);
}

template <int NP, bool ZD, int SPLIT, bool TABLE, int WPB>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(wide_min_waves<NP, ZD, SPLIT, WPB>())))
void k_fused_wide(InstDesc one, const InstDesc* __restrict__ descs,
                                                         const int2* __restrict__ blkmap)
{
    if constexpr (TABLE) {
        const int2 bm = blkmap[blockIdx.x];
        fused_wide_block<NP, ZD, SPLIT, WPB>(descs[__builtin_amdgcn_readfirstlane(bm.x)],
                                             __builtin_amdgcn_readfirstlane(bm.y));
    } else {
        fused_wide_block<NP, ZD, SPLIT, WPB>(one, (int)blockIdx.x * WPB);
    }
}

// ------------------------------------------------------------------ eval
template <int NP, bool SYM, bool ZD>
__global__ __launch_bounds__(256) void k_eval_mfma(InstDesc d, const uint8_t* __restrict__ perms, int count,
                                                   long long* __restrict__ goals, long long* __restrict__ deltas)
{
    __shared__ __attribute__((aligned(16))) int8_t sF[NP * lds_stride<NP>()];
    __shared__ __attribute__((aligned(16))) int8_t sD[NP * lds_stride_d<NP>()];
    __shared__ __attribute__((aligned(16))) int8_t sFT[SYM ? 16 : NP * lds_stride<NP>()];
    __shared__ __attribute__((aligned(16))) int8_t sDT[SYM ? 16 : NP * lds_stride_d<NP>()];
    __shared__ __attribute__((aligned(16))) uint8_t sp[kWaves][NP];
    __shared__ RowInfo sri[kWaves][NP];
    load_instance_lds<NP, SYM>(d, sF, sD, sFT, sDT);
    __syncthreads();
    const int w = threadIdx.x / kWave, l = lane_id();
    const int e = blockIdx.x * kWaves + w;
    if (e >= count) return;
    const int n = d.n;
    uint8_t* pw = sp[w];
    for (int j = l; j < NP; j += kWave) pw[j] = j < n ? perms[(size_t)e * n + j] : 0;
    wave_sync();
    long long* dout = deltas ? deltas + (size_t)e * n * n : nullptr;
    long long goal, key;
    goal_delta_mfma<NP, SYM, ZD>(n, sF, sD, sFT, sDT, pw, sri[w], dout != nullptr, dout, goal, key);
    if (dout)
        for (int j = l; j < n; j += kWave) dout[(size_t)j * n + j] = 0;
    if (l == 0) goals[e] = goal;
}

template <int NP, bool ZD, int SPLIT>
__global__ __launch_bounds__(256) void k_eval_wide(InstDesc d, const uint8_t* __restrict__ perms, int count,
                                                   long long* __restrict__ goals, long long* __restrict__ deltas)
{
    constexpr int CPL = cols_per_lane<NP>();
    __shared__ __attribute__((aligned(16))) int8_t spl[wide_planes<SPLIT>() * NP * lds_stride<NP>()];
    __shared__ __attribute__((aligned(16))) WideWaveLds<NP, CPL> sw[kWaves];
    load_wide_lds<NP, SPLIT>(d, spl);
    __syncthreads();
    const int w = threadIdx.x / kWave, l = lane_id();
    const int e = blockIdx.x * kWaves + w;
    if (e >= count) return;
    const int n = d.n;
    uint8_t* pw = sw[w].p;
    for (int j = l; j < NP; j += kWave) pw[j] = j < n ? perms[(size_t)e * n + j] : 0;
    wave_sync();
    long long* dout = deltas ? deltas + (size_t)e * n * n : nullptr;
    long long goal, key;
    goal_delta_wide<NP, ZD, SPLIT>(n, spl, pw, sw[w].q, sw[w].u.ri, dout != nullptr, dout, goal, key);
    if (dout)
        for (int j = l; j < n; j += kWave) dout[(size_t)j * n + j] = 0;
    if (l == 0) goals[e] = goal;
}

// ------------------------------------------------------------------ launchers
// Contraction variants: int8 general (F or D not symmetric), int8 symmetric,
// int8 symmetric with zero diagonals, and the byte-split symmetric ones (WIDE =
// the split pattern: 1 F split, 2 D split, 3 both; both split at npad 160 would
// not fit the register file and is left to the int32 path).
template <int NP, int WIDE, bool SYM, bool ZD>
static hipError_t fused_launch_one(const InstDesc* one, const InstDesc* descs, const int2* blkmap, int blocks,
                                   hipStream_t st)
{
    constexpr int WPB = fused_wpb(NP, WIDE, SYM, ZD);
    const dim3 grid((unsigned)blocks), block(WPB * kWave);
    if constexpr (WIDE == 3 && NP > 128) {
        return hipErrorNotSupported;
    } else if constexpr (WIDE != 0) {
        if (one)
            hipLaunchKernelGGL((k_fused_wide<NP, ZD, WIDE, false, WPB>), grid, block, 0, st, *one, descs, blkmap);
        else
            hipLaunchKernelGGL((k_fused_wide<NP, ZD, WIDE, true, WPB>), grid, block, 0, st, InstDesc{}, descs,
                               blkmap);
    } else {
        if (one)
            hipLaunchKernelGGL((k_fused_step<NP, SYM, ZD, false, WPB>), grid, block, 0, st, *one, descs, blkmap);
        else
            hipLaunchKernelGGL((k_fused_step<NP, SYM, ZD, true, WPB>), grid, block, 0, st, InstDesc{}, descs, blkmap);
    }
    return hipGetLastError();
}

template <int WIDE, bool SYM, bool ZD>
static hipError_t fused_launch_np(int npad, const InstDesc* one, const InstDesc* descs, const int2* blkmap,
                                  int blocks, hipStream_t st)
{
    switch (npad) {
    case 32: return fused_launch_one<32, WIDE, SYM, ZD>(one, descs, blkmap, blocks, st);
    case 64: return fused_launch_one<64, WIDE, SYM, ZD>(one, descs, blkmap, blocks, st);
    case 96: return fused_launch_one<96, WIDE, SYM, ZD>(one, descs, blkmap, blocks, st);
    case 128: return fused_launch_one<128, WIDE, SYM, ZD>(one, descs, blkmap, blocks, st);
    case 160: return fused_launch_one<160, WIDE, SYM, ZD>(one, descs, blkmap, blocks, st);
    default: return hipErrorNotSupported;
    }
}

bool split_supported(int npad, int split) { return npad <= 160 && (split != 3 || npad <= 128); }

int fused_particles_per_block(int npad, int wide, bool sym, bool zd) { return fused_wpb(npad, wide, sym, zd); }

bool fused_supported(const InstDesc& d)
{
    return (d.path == 1 || (d.path == 3 && d.sym && split_supported(d.npad, d.split))) && d.npad <= 160 && d.sx == 0;
}

hipError_t launch_fused_class(int npad, int wide, bool sym, bool zd, const InstDesc* one, const InstDesc* descs,
                              const int2* blkmap, int blocks, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    if (wide != 0 && !sym) return hipErrorNotSupported;
    if (wide == 1)
        return zd ? fused_launch_np<1, true, true>(npad, one, descs, blkmap, blocks, st)
                  : fused_launch_np<1, true, false>(npad, one, descs, blkmap, blocks, st);
    if (wide == 2)
        return zd ? fused_launch_np<2, true, true>(npad, one, descs, blkmap, blocks, st)
                  : fused_launch_np<2, true, false>(npad, one, descs, blkmap, blocks, st);
    if (wide == 3)
        return zd ? fused_launch_np<3, true, true>(npad, one, descs, blkmap, blocks, st)
                  : fused_launch_np<3, true, false>(npad, one, descs, blkmap, blocks, st);
    return !sym ? fused_launch_np<0, false, false>(npad, one, descs, blkmap, blocks, st)
                : zd ? fused_launch_np<0, true, true>(npad, one, descs, blkmap, blocks, st)
                     : fused_launch_np<0, true, false>(npad, one, descs, blkmap, blocks, st);
}

template <int NP, int WIDE, bool SYM, bool ZD>
static void eval_launch_one(const InstDesc& d, const uint8_t* perms, int count, long long* goals, long long* deltas,
                            hipStream_t st)
{
    const dim3 grid((unsigned)((count + kWaves - 1) / kWaves)), block(kWaves * kWave);
    if constexpr (WIDE == 3 && NP > 128)
        return;  // not reached: split_supported
    else if constexpr (WIDE != 0)
        hipLaunchKernelGGL((k_eval_wide<NP, ZD, WIDE>), grid, block, 0, st, d, perms, count, goals, deltas);
    else
        hipLaunchKernelGGL((k_eval_mfma<NP, SYM, ZD>), grid, block, 0, st, d, perms, count, goals, deltas);
}

template <int WIDE, bool SYM, bool ZD>
static hipError_t eval_launch_np(const InstDesc& d, const uint8_t* perms, int count, long long* goals,
                                 long long* deltas, hipStream_t st)
{
    switch (d.npad) {
    case 32: eval_launch_one<32, WIDE, SYM, ZD>(d, perms, count, goals, deltas, st); break;
    case 64: eval_launch_one<64, WIDE, SYM, ZD>(d, perms, count, goals, deltas, st); break;
    case 96: eval_launch_one<96, WIDE, SYM, ZD>(d, perms, count, goals, deltas, st); break;
    case 128: eval_launch_one<128, WIDE, SYM, ZD>(d, perms, count, goals, deltas, st); break;
    case 160: eval_launch_one<160, WIDE, SYM, ZD>(d, perms, count, goals, deltas, st); break;
    default: return hipErrorNotSupported;
    }
    return hipGetLastError();
}

hipError_t launch_eval_mfma(const InstDesc& d, const uint8_t* perms, int count, long long* goals, long long* deltas,
                            hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    if (d.path == 3) {
        if (!d.sym || !split_supported(d.npad, d.split)) return hipErrorNotSupported;
        switch (d.split) {
        case 1: return d.zd ? eval_launch_np<1, true, true>(d, perms, count, goals, deltas, st)
                            : eval_launch_np<1, true, false>(d, perms, count, goals, deltas, st);
        case 2: return d.zd ? eval_launch_np<2, true, true>(d, perms, count, goals, deltas, st)
                            : eval_launch_np<2, true, false>(d, perms, count, goals, deltas, st);
        case 3: return d.zd ? eval_launch_np<3, true, true>(d, perms, count, goals, deltas, st)
                            : eval_launch_np<3, true, false>(d, perms, count, goals, deltas, st);
        default: return hipErrorNotSupported;
        }
    }
    return !d.sym ? eval_launch_np<0, false, false>(d, perms, count, goals, deltas, st)
                  : d.zd ? eval_launch_np<0, true, true>(d, perms, count, goals, deltas, st)
                         : eval_launch_np<0, true, false>(d, perms, count, goals, deltas, st);
}

}  // namespace qap
