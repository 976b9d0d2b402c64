// Per-stage kernels: initialisation, and the per-stage ("plain") engine that
// launches one kernel per step of the iteration with an int32 contraction for
// the pair-exchange deltas.  The swarm-best and finish kernels are shared by
// both engines.
#include "dword.hpp"
#include "kernels.hpp"
#include "second_target.hpp"

namespace qap {

// ------------------------------------------------------------------ init
// X(0): Fisher-Yates shuffle of the identity, one lane per particle
// (for i = n-1 .. 1 swap p[i] with p[bounded(word_{n-1-i}, i+1)], t = 0).
__global__ void k_init_perm(InstDesc d)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.P) return;
    const uint32_t g = (uint32_t)(k / d.S + d.swarm_base), s = (uint32_t)(k % d.S);
    const int n = d.n;
    uint8_t* x = d.X[0] + (size_t)k * n;
    for (int j = 0; j < n; ++j) x[j] = (uint8_t)j;
    for (int e = 0; e <= n - 2; ++e) {
        const int i = n - 1 - e;
        const int j = (int)bounded_u32(stream_word(d.seed, (uint32_t)e, 0, s, g), (uint32_t)(i + 1));
        const uint8_t t = x[i];
        x[i] = x[j];
        x[j] = t;
    }
    for (int j = 0; j < n; ++j) d.PL[(size_t)k * n + j] = x[j];
}

// V(0)_rc = vmax (2u - 1), then S_v; one thread per (particle, column).  The
// column's L1 norm is accumulated as a double word (no loss per addition) and
// rounded once, as in the velocity pass.
__global__ void k_init_vel(InstDesc d)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = d.n;
    if (idx >= (long long)d.P * n) return;
    const int k = (int)(idx / n), c = (int)(idx % n);
    const uint32_t g = (uint32_t)(k / d.S + d.swarm_base), s = (uint32_t)(k % d.S);
    float* V = d.V[0] + (size_t)k * n * n;
    DW sum{0.0f, 0.0f};
    for (int r = 0; r < n; ++r) {
        const float u = unit_float(stream_word(d.seed, 256u + (uint32_t)(r * n + c), 0, s, g));
        float t = __fmul_rn(d.vmax, __fsub_rn(__fmul_rn(2.0f, u), 1.0f));
        t = fminf(fmaxf(t, -d.vmax), d.vmax);
        V[(size_t)r * n + c] = t;
        sum = dw_add_f(sum, fabsf(t));
    }
    const float tot = __fadd_rn(sum.hi, sum.lo);
    d.Vinv[0][(size_t)k * n + c] = (d.norm && tot > 0.0f) ? __fdiv_rn(1.0f, tot) : 1.0f;
}

// ------------------------------------------------------------------ velocity
// eq. (velocity): V(t+1) = S_v(c1 V + c2 r2 (P^L - X) + c3 r3 (P^G - X)) at
// state t, one thread per (particle, column), one pass: the unnormalised
// values and the column scale are stored.
__global__ void k_velocity(InstDesc d)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = d.n;
    if (idx >= (long long)d.P * n) return;
    const int k = (int)(idx / n), c = (int)(idx % n);
    const int tprev = *d.iter;
    const uint32_t tau = (uint32_t)tprev + 1u;
    const int cur = tprev & 1;
    const int gl = k / d.S;  // swarm within this descriptor; g: within the instance
    const uint32_t g = (uint32_t)(gl + d.swarm_base), s = (uint32_t)(k % d.S);
    const Philox4 rb = philox4x32_10(0u, tau, s, g, (uint32_t)d.seed, (uint32_t)(d.seed >> 32));
    // c2 r2, c3 r3 and c1 x are exact double words: an attraction cell
    // c1 x + s2 a + s3 b (a, b in {-1, 0, 1} of one sign) is summed by the
    // accurate double-word addition and rounded once (the terms can cancel);
    // the column sum is accumulated as a double word and rounded once
    const DW s2 = two_prod(d.c2, unit_float(rb.w[0]));
    const DW s3 = two_prod(d.c3, unit_float(rb.w[1]));
    const DW s23 = dw_add(s2, s3);
    const int x = d.X[cur][(size_t)k * n + c];
    const int pl = d.PL[(size_t)k * n + c];
    const int pg = d.PG[(size_t)gl * n + c];
    const float* Vc = d.V[cur] + (size_t)k * n * n;
    const float sc = d.Vinv[cur][(size_t)k * n + c];
    float* Vn = d.V[cur ^ 1] + (size_t)k * n * n;
    DW sum{0.0f, 0.0f};
    for (int r = 0; r < n; ++r) {
        const int a = (r == pl) - (r == x), b = (r == pg) - (r == x);
        const float v = __fmul_rn(Vc[(size_t)r * n + c], sc);
        float t;
        if (a | b) {
            const DW o = (a && b) ? s23 : a ? s2 : s3;
            t = dw_add(two_prod(d.c1, v), (a + b) < 0 ? dw_neg(o) : o).hi;
        } else {
            t = __fmul_rn(d.c1, v);
        }
        t = fminf(fmaxf(t, -d.vmax), d.vmax);
        sum = dw_add_f(sum, fabsf(t));
        Vn[(size_t)r * n + c] = t;
    }
    const float tot = __fadd_rn(sum.hi, sum.lo);
    d.Vinv[cur ^ 1][(size_t)k * n + c] = (d.norm && tot > 0.0f) ? __fdiv_rn(1.0f, tot) : 1.0f;
}

// ------------------------------------------------------------------ S_x
// S_x = SecondTarget of particle k at state tprev (buffers of parity tprev & 1,
// random stream of iteration tprev + 1) into out [n]; one wave.
template <int CPL>
__device__ __forceinline__ void second_target_particle(const InstDesc& d, int k, int tprev, uint8_t* out,
                                                       StLds<CPL>* sl)
{
    const int n = d.n;
    const int cur = tprev & 1;
    const uint32_t g = (uint32_t)(k / d.S + d.swarm_base), s = (uint32_t)(k % d.S);
    const float* V = d.V[cur] + (size_t)k * n * n;
    const float* Vs = d.Vinv[cur] + (size_t)k * n;
    StState<CPL> st;
    st_init_scan<CPL>(n, V, Vs, d.X[cur] + (size_t)k * n, st);
    st_select<CPL>(n, d.depth, V, Vs, st, out, sl, d.seed, (uint32_t)tprev + 1u, s, g);
}

template <int CPL>
__global__ __launch_bounds__(256) void k_second_target(InstDesc d)
{
    __shared__ StLds<CPL> slds[4];
    const int wave = (int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
    if (wave >= d.P) return;
    second_target_particle<CPL>(d, wave, *d.iter, d.Xnew + (size_t)wave * d.n, &slds[threadIdx.x / kWave]);
}

// S_x = PickColumn, one wave per particle: the visit order (Fisher-Yates on
// stream elements 4 + n + j, drawn in parallel by the lanes and applied by
// lane 0 in LDS), then per visited column the largest key over the rows left
// (a wave maximum over lane-owned rows), equal keys to the k-th such row with
// k = bounded(stream element 4 + visit, count).  Particle k at state tprev
// into out [n]; swords, order: LDS of this wave.
template <int CPL>
__device__ __forceinline__ void pick_column_particle(const InstDesc& d, int k, int tprev, uint8_t* out,
                                                     uint32_t* w, uint8_t* order)
{
    const int l = lane_id();
    const int n = d.n;
    const int cur = tprev & 1;
    const uint32_t tau = (uint32_t)tprev + 1u;
    const uint32_t g = (uint32_t)(k / d.S + d.swarm_base), s = (uint32_t)(k % d.S);
    const float* V = d.V[cur] + (size_t)k * n * n;
    const float* Vs = d.Vinv[cur] + (size_t)k * n;
    const uint8_t* z = d.X[cur] + (size_t)k * n;
    for (int j = l; j < n - 1; j += kWave) w[j] = stream_word(d.seed, 4u + (uint32_t)(n + j), tau, s, g);
    for (int c = l; c < n; c += kWave) order[c] = (uint8_t)c;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (l == 0)
        for (int i = n - 1; i >= 1; --i) {
            const uint32_t jj = bounded_u32(w[n - 1 - i], (uint32_t)(i + 1));
            const uint8_t t = order[i];
            order[i] = order[jj];
            order[jj] = t;
        }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    unsigned rowbits = 0;
#pragma unroll
    for (int j = 0; j < CPL; ++j)
        if (l + kWave * j < n) rowbits |= 1u << j;
    for (int v = 0; v < n; ++v) {
        const int c = order[v];
        const int zc = z[c];
        const float sc = Vs[c];
        float key[CPL];
        float best = -INFINITY;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            const int r = l + kWave * j;
            key[j] = -INFINITY;
            if ((rowbits >> j) & 1u) {
                const float x = __fmul_rn(V[(size_t)r * n + c], sc);
                key[j] = r == zc ? 1.0f + x : x;
            }
            best = fmaxf(best, key[j]);
        }
        const float m = wave_max(best);
        uint64_t bal[CPL];
        int count = 0;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            bal[j] = ballot64(((rowbits >> j) & 1u) && key[j] == m);
            count += __popcll(bal[j]);
        }
        int kk = count > 1 ? (int)bounded_u32(stream_word(d.seed, 4u + (uint32_t)v, tau, s, g), (uint32_t)count) : 0;
        int sel = -1;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            if (sel >= 0) continue;
            const int pc = __popcll(bal[j]);
            if (kk < pc) {
                uint64_t b = bal[j];
                for (int q = 0; q < kk; ++q) b &= b - 1;  // drop the kk lowest set bits
                sel = kWave * j + __ffsll((long long)b) - 1;
            } else {
                kk -= pc;
            }
        }
        if (sel < 0 || sel >= n) sel = 0;  // unreachable: the column has an alive row
        if (l == 0) out[c] = (uint8_t)sel;
        if (l == (sel & (kWave - 1))) rowbits &= ~(1u << (sel >> 6));
    }
}


template <int CPL>
__global__ __launch_bounds__(256) void k_pick_column(InstDesc d)
{
    __shared__ uint32_t swords[4][kMaxN];
    __shared__ uint8_t sorder[4][kMaxN];
    const int wl = (int)(threadIdx.x / kWave);
    const int wave = (int)(blockIdx.x * (blockDim.x / kWave)) + wl;
    if (wave >= d.P) return;
    pick_column_particle<CPL>(d, wave, *d.iter, d.Xnew + (size_t)wave * d.n, swords[wl], sorder[wl]);
}

// S_x output of one particle k at state tprev (one wave): the permutation the
// step from tprev to tprev + 1 selected before its pair exchanges, recomputed
// from the buffers of state tprev (which that step only read).
template <int CPL>
__global__ __launch_bounds__(64) void k_sx_probe(InstDesc d, int k, int tprev, uint8_t* out)
{
    __shared__ StLds<CPL> sl;
    __shared__ uint32_t swords[kMaxN];
    __shared__ uint8_t sorder[kMaxN];
    if (d.sx == 1)
        pick_column_particle<CPL>(d, k, tprev, out, swords, sorder);
    else
        second_target_particle<CPL>(d, k, tprev, out, &sl);
}

template __global__ void k_second_target<1>(InstDesc);
template __global__ void k_second_target<2>(InstDesc);
template __global__ void k_second_target<4>(InstDesc);
template __global__ void k_pick_column<1>(InstDesc);
template __global__ void k_pick_column<2>(InstDesc);
template __global__ void k_pick_column<4>(InstDesc);
template __global__ void k_sx_probe<1>(InstDesc, int, int, uint8_t*);
template __global__ void k_sx_probe<2>(InstDesc, int, int, uint8_t*);
template __global__ void k_sx_probe<4>(InstDesc, int, int, uint8_t*);

// ------------------------------------------------------------------ goal + deltas (int32)
// One workgroup (256 threads) per particle.  A = F . Dp^T with Dp[y][k] =
// D[p_y][p_k] (and, for non-symmetric data, B = F^T . Dp' with D^T) is
// accumulated in int32 by a 64x64-tiled LDS GEMM into a per-workgroup global
// scratch, then every pair (a, b), a < b, gets
//   delta = (A_ab + A_ba - A_aa - A_bb) + (B_ab + B_ba - B_aa - B_bb) - kappa + lambda
// (B = A when F and D are symmetric), with the corrections for the terms the
// sums count wrongly (k = a or b):
//   kappa  = (f_aa-f_ba)(Dp_ba-Dp_aa) + (f_ab-f_bb)(Dp_bb-Dp_ab)
//          + (f_aa-f_ab)(Dp_ab-Dp_aa) + (f_ba-f_bb)(Dp_bb-Dp_ba)
//   lambda = (f_aa-f_bb)(Dp_bb-Dp_aa) + (f_ab-f_ba)(Dp_ba-Dp_ab).
// goal = trace(A).  mode: 0 step (local search, P^L), 1 eval, 2 init.
namespace {
constexpr int kTile = 64, kKc = 32;

template <bool MUL24>
__device__ __forceinline__ int imul(int a, int b) { return MUL24 ? __mul24(a, b) : a * b; }

template <bool MUL24>
__device__ void gemm_to_scratch(int n, const int* __restrict__ Fm, const int* __restrict__ Dm, const uint8_t* pl,
                                int* __restrict__ out, int (*Fs)[kKc + 1], int (*Ds)[kKc + 1])
{
    // out[x][y] = sum_k Fm[x][k] * Dm[p_y][p_k]
    const int tid = threadIdx.x, ti = tid / 16, tj = tid % 16;
    const int nt = (n + kTile - 1) / kTile;
    for (int ty = 0; ty < nt; ++ty)
        for (int tx = 0; tx < nt; ++tx) {
            int acc[4][4] = {};
            for (int k0 = 0; k0 < n; k0 += kKc) {
                for (int e = tid; e < kTile * kKc; e += 256) {
                    const int i = e / kKc, kk = e % kKc;
                    const int x = ty * kTile + i, y = tx * kTile + i, kx = k0 + kk;
                    Fs[i][kk] = (x < n && kx < n) ? Fm[(size_t)x * n + kx] : 0;
                    Ds[i][kk] = (y < n && kx < n) ? Dm[(size_t)pl[y] * n + pl[kx]] : 0;
                }
                __syncthreads();
                // the chunk's columns past n are zero: stop at n
                const int kend = min(kKc, n - k0);
#pragma unroll 4
                for (int kk = 0; kk < kend; ++kk) {
                    int fa[4], db[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) { fa[u] = Fs[ti * 4 + u][kk]; db[u] = Ds[tj * 4 + u][kk]; }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[u][v] += imul<MUL24>(fa[u], db[v]);
                }
                __syncthreads();
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int x = ty * kTile + ti * 4 + u, y = tx * kTile + tj * 4 + v;
                    if (x < n && y < n) out[(size_t)x * n + y] = acc[u][v];
                }
        }
}
}  // namespace

template <bool GEN, bool MUL24>
__global__ __launch_bounds__(256) void k_goal_delta_i32(InstDesc d, const uint8_t* __restrict__ perms, int count,
                                                        int mode, long long* __restrict__ goals_out,
                                                        long long* __restrict__ deltas_out)
{
    __shared__ int Fs[kTile][kKc + 1];
    __shared__ int Ds[kTile][kKc + 1];
    __shared__ uint8_t pl[kMaxN];
    __shared__ long long diag[kMaxN];
    __shared__ int fdiag[kMaxN], ddiag[kMaxN];  // f_aa and Dp_aa = D[p_a][p_a]
    __shared__ long long red_d[4];
    __shared__ int red_a[4], red_b[4];
    __shared__ long long red_goal[4];
    const int n = d.n, tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const size_t nn = (size_t)n * n;
    int* A = d.scratch + (size_t)blockIdx.x * nn * (GEN ? 2 : 1);
    int* B = GEN ? A + nn : A;
    const int tprev = *d.iter;
    const int cur = tprev & 1;
    for (int e = blockIdx.x; e < count; e += gridDim.x) {
        const uint8_t* pe = perms + (size_t)e * n;
        // clamp: a malformed permutation on the device can give wrong numbers, never a stray address
        for (int j = tid; j < n; j += 256) pl[j] = pe[j] < n ? pe[j] : (uint8_t)(n - 1);
        __syncthreads();
        // step mode: up to d.ls exchanges; one found while more are allowed is
        // made in pl and everything recomputed, the last allowed one is applied
        // when X(t+1) is written
        int swaps = 0;
        long long goal, bd;
        int ba, bb;
        for (;;) {
        gemm_to_scratch<MUL24>(n, d.F32, d.D32, pl, A, Fs, Ds);
        if (GEN) {
            // B[x][y] = sum_k F[k][x] D[p_k][p_y]: the same product on (F^T, D^T)
            // F^T read through a transposed index: stage via the generic routine on transposed views
            __syncthreads();
            const int nt = (n + kTile - 1) / kTile;
            const int ti = tid / 16, tj = tid % 16;
            for (int ty = 0; ty < nt; ++ty)
                for (int tx = 0; tx < nt; ++tx) {
                    int acc[4][4] = {};
                    for (int k0 = 0; k0 < n; k0 += kKc) {
                        for (int q = tid; q < kTile * kKc; q += 256) {
                            const int i = q / kKc, kk = q % kKc;
                            const int x = ty * kTile + i, y = tx * kTile + i, kx = k0 + kk;
                            Fs[i][kk] = (x < n && kx < n) ? d.F32[(size_t)kx * n + x] : 0;
                            Ds[i][kk] = (y < n && kx < n) ? d.D32[(size_t)pl[kx] * n + pl[y]] : 0;
                        }
                        __syncthreads();
                        const int kend = min(kKc, n - k0);
#pragma unroll 4
                        for (int kk = 0; kk < kend; ++kk) {
                            int fa[4], db[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) { fa[u] = Fs[ti * 4 + u][kk]; db[u] = Ds[tj * 4 + u][kk]; }
#pragma unroll
                            for (int u = 0; u < 4; ++u)
#pragma unroll
                                for (int v = 0; v < 4; ++v) acc[u][v] += imul<MUL24>(fa[u], db[v]);
                        }
                        __syncthreads();
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int x = ty * kTile + ti * 4 + u, y = tx * kTile + tj * 4 + v;
                            if (x < n && y < n) B[(size_t)x * n + y] = acc[u][v];
                        }
                }
        }
        __syncthreads();
        // diagonal and goal
        long long gpart = 0;
        for (int a = tid; a < n; a += 256) {
            const long long da = (long long)A[(size_t)a * n + a];
            diag[a] = GEN ? da + (long long)B[(size_t)a * n + a] : 2 * da;
            gpart += da;
            fdiag[a] = d.F32[(size_t)a * n + a];
            ddiag[a] = d.D32[(size_t)pl[a] * n + pl[a]];
        }
        gpart = wave_sum_i64(gpart);
        if (l == 0) red_goal[w] = gpart;
        __syncthreads();
        goal = red_goal[0] + red_goal[1] + red_goal[2] + red_goal[3];
        // pair deltas
        bd = LLONG_MAX;
        ba = 0x7fffffff;
        bb = 0x7fffffff;
        if (mode != 2) {
            // wave w takes the rows a = w, w + 4, ..., its lanes the b > a
            for (int a = w; a < n - 1; a += 4)
            for (int b = a + 1 + l; b < n; b += 64) {
                const int pa = pl[a], pb = pl[b];
                const long long faa = fdiag[a], fbb = fdiag[b];
                const long long fab = d.F32[(size_t)a * n + b], fba = d.F32[(size_t)b * n + a];
                const long long Daa = ddiag[a], Dbb = ddiag[b];
                const long long Dab = d.D32[(size_t)pa * n + pb], Dba = d.D32[(size_t)pb * n + pa];
                long long s = (long long)A[(size_t)a * n + b] + (long long)A[(size_t)b * n + a];
                if (GEN) s += (long long)B[(size_t)a * n + b] + (long long)B[(size_t)b * n + a];
                else s *= 2;
                const long long kap = (faa - fba) * (Dba - Daa) + (fab - fbb) * (Dbb - Dab) +
                                      (faa - fab) * (Dab - Daa) + (fba - fbb) * (Dbb - Dba);
                const long long lam = (faa - fbb) * (Dbb - Daa) + (fab - fba) * (Dba - Dab);
                const long long del = s - diag[a] - diag[b] - kap + lam;
                if (mode == 1 && deltas_out) {
                    long long* out = deltas_out + (size_t)e * nn;
                    out[(size_t)a * n + b] = del;
                    out[(size_t)b * n + a] = del;
                }
                if (del < bd || (del == bd && (a < ba || (a == ba && b < bb)))) { bd = del; ba = a; bb = b; }
            }
            if (mode == 1 && deltas_out)
                for (int a = tid; a < n; a += 256) deltas_out[(size_t)e * nn + (size_t)a * n + a] = 0;
            wave_argmin_pair(bd, ba, bb);
            if (l == 0) { red_d[w] = bd; red_a[w] = ba; red_b[w] = bb; }
            __syncthreads();
            bd = red_d[0]; ba = red_a[0]; bb = red_b[0];
            for (int u = 1; u < 4; ++u)
                if (red_d[u] < bd || (red_d[u] == bd && (red_a[u] < ba || (red_a[u] == ba && red_b[u] < bb)))) {
                    bd = red_d[u]; ba = red_a[u]; bb = red_b[u];
                }
        }
        if (mode != 0 || d.ls <= swaps + 1 || ba >= n || bd >= 0) break;
        __syncthreads();  // every thread has read the reductions
        if (tid == 0) {
            const uint8_t t = pl[ba];
            pl[ba] = pl[bb];
            pl[bb] = t;
        }
        __syncthreads();
        ++swaps;
        }
        if (mode == 1) {
            if (tid == 0 && goals_out) goals_out[e] = goal;
        } else {
            const bool swap = (mode == 0) && d.ls > swaps && ba < n && bd < 0;
            if (swap) goal += bd;
            uint8_t* xo = (mode == 0) ? d.X[cur ^ 1] + (size_t)e * n : nullptr;
            const bool improve = (mode == 2) || goal < d.goalPL[e];
            for (int j = tid; j < n; j += 256) {
                uint8_t v = pl[j];
                if (swap && j == ba) v = pl[bb];
                if (swap && j == bb) v = pl[ba];
                if (xo) xo[j] = v;
                if (improve) d.PL[(size_t)e * n + j] = v;
            }
            if (tid == 0) {
                d.goal[e] = goal;
                if (improve) d.goalPL[e] = goal;
            }
        }
        __syncthreads();
    }
}

template __global__ void k_goal_delta_i32<false, false>(InstDesc, const uint8_t*, int, int, long long*, long long*);
template __global__ void k_goal_delta_i32<false, true>(InstDesc, const uint8_t*, int, int, long long*, long long*);
template __global__ void k_goal_delta_i32<true, false>(InstDesc, const uint8_t*, int, int, long long*, long long*);
template __global__ void k_goal_delta_i32<true, true>(InstDesc, const uint8_t*, int, int, long long*, long long*);

// ------------------------------------------------------------------ swarm best
// One workgroup per swarm of any instance of the handle (smap: workgroup ->
// (instance, swarm)): the best member of this iteration (lowest index on
// ties); P^G <- its current solution on strict improvement (Sec. 3.2 P^G[k]).
// init != 0: iteration 0 (solutions in buffer 0).
__global__ __launch_bounds__(256) void k_swarm_best(const InstDesc* __restrict__ descs, const int2* __restrict__ smap,
                                                    int init)
{
    __shared__ long long sg[4];
    __shared__ int sm[4];
    const int2 ig = smap[blockIdx.x];
    const InstDesc& d = descs[ig.x];
    const int g = ig.y, tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int n = d.n, S = d.S;
    const int nxt = init ? 0 : ((*d.iter & 1) ^ 1);
    long long bg = LLONG_MAX;
    int bm = 0x7fffffff;
    for (int s = tid; s < S; s += 256) {
        const long long v = d.goal[(size_t)g * S + s];
        if (v < bg) { bg = v; bm = s; }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const long long v2 = __shfl_xor(bg, off, kWave);
        const int m2 = __shfl_xor(bm, off, kWave);
        if (v2 < bg || (v2 == bg && m2 < bm)) { bg = v2; bm = m2; }
    }
    if (l == 0) { sg[w] = bg; sm[w] = bm; }
    __syncthreads();
    bg = sg[0]; bm = sm[0];
    for (int u = 1; u < 4; ++u)
        if (sg[u] < bg || (sg[u] == bg && sm[u] < bm)) { bg = sg[u]; bm = sm[u]; }
    const bool upd = bg < d.goalPG[g];
    const uint8_t* src = d.X[nxt] + ((size_t)g * S + bm) * n;
    if (upd)
        for (int j = tid; j < n; j += 256) d.PG[(size_t)g * n + j] = src[j];
    __syncthreads();
    if (tid == 0) {
        if (upd) d.goalPG[g] = bg;
        d.smin[g].goal = bg;
        d.smin[g].member = bm;
    }
}

// ------------------------------------------------------------------ migration
// Alg. 2 after iteration tau, one workgroup, X(tau) in buffer xb: swarms are
// ranked by (goal of P^G, index); for q < d a uniformly drawn member of the
// q-th best swarm gives its current solution and goal to the q-th worst swarm.
__device__ void migrate_swarms(const InstDesc& d, int tau, int xb)
{
    int* __restrict__ order = d.order;
    const int tid = threadIdx.x, n = d.n, m = d.m, S = d.S;
    for (int g = tid; g < m; g += blockDim.x) {
        const long long vg = d.goalPG[g];
        int rank = 0;
        for (int h = 0; h < m; ++h) {
            const long long vh = d.goalPG[h];
            rank += (vh < vg) || (vh == vg && h < g);
        }
        order[rank] = g;
    }
    __syncthreads();
    for (int q = 0; q < d.migr_d; ++q) {
        const int donor = order[q], recip = order[m - 1 - q];
        const uint32_t j = bounded_u32(stream_word(d.seed, (uint32_t)q, (uint32_t)tau, 0xFFFFFFFFu, 0u), (uint32_t)S);
        const size_t pi = (size_t)donor * S + j;
        for (int c = tid; c < n; c += blockDim.x) d.PG[(size_t)recip * n + c] = d.X[xb][pi * n + c];
        if (tid == 0) d.goalPG[recip] = d.goal[pi];
    }
}

// Alg. 2 for instances stepped in several stream groups (whose own finish
// steps do not migrate), once every group has finished iteration tau (the
// counter the instance's descriptor points at): one workgroup per instance,
// which acts only when tau is a multiple of its period.
__global__ __launch_bounds__(256) void k_migrate(const InstDesc* __restrict__ descs)
{
    const InstDesc& d = descs[blockIdx.x];
    const int tau = *d.iter;
    if (d.migr_d <= 0 || tau % d.period != 0) return;
    migrate_swarms(d, tau, tau & 1);
}

// ------------------------------------------------------------------ finish
// One workgroup per instance (descs[blockIdx.x]): best-ever record, migration
// (Alg. 2) when due, and the iteration counter.  Swarms are ranked by (goal of
// P^G, index); for k < d a uniformly drawn member of the k-th best swarm gives
// its current solution and goal to the k-th worst swarm.
__global__ __launch_bounds__(256) void k_finish(const InstDesc* __restrict__ descs, int init)
{
    const InstDesc& d = descs[blockIdx.x];
    __shared__ long long sg[4];
    __shared__ int ss[4];
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int n = d.n, m = d.m, S = d.S;
    const int tprev = init ? -1 : *d.iter;
    const int tau = tprev + 1;
    const int nxt = init ? 0 : ((tprev & 1) ^ 1);
    // best over swarm minima, lowest swarm on ties
    long long bg = LLONG_MAX;
    int bs = 0x7fffffff;
    for (int g = tid; g < m; g += 256) {
        const long long v = d.smin[g].goal;
        if (v < bg) { bg = v; bs = g; }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const long long v2 = __shfl_xor(bg, off, kWave);
        const int s2 = __shfl_xor(bs, off, kWave);
        if (v2 < bg || (v2 == bg && s2 < bs)) { bg = v2; bs = s2; }
    }
    if (l == 0) { sg[w] = bg; ss[w] = bs; }
    __syncthreads();
    bg = sg[0]; bs = ss[0];
    for (int u = 1; u < 4; ++u)
        if (sg[u] < bg || (sg[u] == bg && ss[u] < bs)) { bg = sg[u]; bs = ss[u]; }
    const bool upd = bg < d.best->goal;
    __syncthreads();
    if (upd) {
        const int mem = d.smin[bs].member;
        const uint8_t* src = d.X[nxt] + ((size_t)bs * S + mem) * n;
        for (int j = tid; j < n; j += 256) d.best->perm[j] = src[j];
        if (tid == 0) {
            d.best->goal = bg;
            d.best->iter = tau;
            d.best->swarm = bs + d.swarm_base;
            d.best->member = mem;
        }
    }
    if (!init && d.migrate && d.migr_d > 0 && (tau % d.period) == 0) migrate_swarms(d, tau, nxt);
    __syncthreads();
    if (tid == 0 && !init) *d.iter = tau;
}

// ------------------------------------------------------------------ launchers
static inline unsigned blocks_for(long long items, int per_block)
{
    return (unsigned)((items + per_block - 1) / per_block);
}

hipError_t launch_goal_delta_i32(const InstDesc& d, int mul24, int grid_gd, const uint8_t* perms, int count,
                                 int mode, long long* goals, long long* deltas, hipStream_t st)
{
    const int grid = count < grid_gd ? count : grid_gd;
    if (grid <= 0) return hipSuccess;
    const bool gen = !d.sym;
    if (gen && mul24)
        hipLaunchKernelGGL((k_goal_delta_i32<true, true>), dim3(grid), dim3(256), 0, st, d, perms, count, mode, goals, deltas);
    else if (gen)
        hipLaunchKernelGGL((k_goal_delta_i32<true, false>), dim3(grid), dim3(256), 0, st, d, perms, count, mode, goals, deltas);
    else if (mul24)
        hipLaunchKernelGGL((k_goal_delta_i32<false, true>), dim3(grid), dim3(256), 0, st, d, perms, count, mode, goals, deltas);
    else
        hipLaunchKernelGGL((k_goal_delta_i32<false, false>), dim3(grid), dim3(256), 0, st, d, perms, count, mode, goals, deltas);
    return hipGetLastError();
}

hipError_t launch_bests(const InstDesc* descs, const int2* smap, int total_swarms, int count, int init,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_swarm_best, dim3((unsigned)total_swarms), dim3(256), 0, st, descs, smap, init);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finish, dim3((unsigned)count), dim3(256), 0, st, descs, init);
    return hipGetLastError();
}

hipError_t launch_migrate(const InstDesc* descs, int count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_migrate, dim3((unsigned)count), dim3(256), 0, st, descs);
    return hipGetLastError();
}

hipError_t launch_init(const InstDesc& d, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_perm, dim3(blocks_for(d.P, 64)), dim3(64), 0, st, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_init_vel, dim3(blocks_for((long long)d.P * d.n, 256)), dim3(256), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_sx_probe(const InstDesc& d, int k, int tprev, uint8_t* out, hipStream_t st)
{
    const int cpl = d.n <= 64 ? 1 : d.n <= 128 ? 2 : 4;
    switch (cpl) {
    case 1: hipLaunchKernelGGL(k_sx_probe<1>, dim3(1), dim3(kWave), 0, st, d, k, tprev, out); break;
    case 2: hipLaunchKernelGGL(k_sx_probe<2>, dim3(1), dim3(kWave), 0, st, d, k, tprev, out); break;
    default: hipLaunchKernelGGL(k_sx_probe<4>, dim3(1), dim3(kWave), 0, st, d, k, tprev, out); break;
    }
    return hipGetLastError();
}

hipError_t launch_plain_step(const InstDesc& d, int mul24, int grid_gd, hipStream_t st, hipEvent_t* ev)
{
    const int cpl = d.n <= 64 ? 1 : d.n <= 128 ? 2 : 4;
    const dim3 gst(blocks_for(d.P, 4)), bst(256);
    hipError_t e;
#define REC(i) do { if (ev) { e = hipEventRecord(ev[i], st); if (e != hipSuccess) return e; } } while (0)
    REC(0);
    if (d.sx == 1) {
        switch (cpl) {
        case 1: hipLaunchKernelGGL(k_pick_column<1>, gst, bst, 0, st, d); break;
        case 2: hipLaunchKernelGGL(k_pick_column<2>, gst, bst, 0, st, d); break;
        default: hipLaunchKernelGGL(k_pick_column<4>, gst, bst, 0, st, d); break;
        }
    } else {
        switch (cpl) {
        case 1: hipLaunchKernelGGL(k_second_target<1>, gst, bst, 0, st, d); break;
        case 2: hipLaunchKernelGGL(k_second_target<2>, gst, bst, 0, st, d); break;
        default: hipLaunchKernelGGL(k_second_target<4>, gst, bst, 0, st, d); break;
        }
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    REC(1);
    REC(2);
    hipLaunchKernelGGL(k_velocity, dim3(blocks_for((long long)d.P * d.n, 256)), dim3(256), 0, st, d);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    REC(3);
    REC(4);
    e = launch_goal_delta_i32(d, mul24, grid_gd, d.Xnew, d.P, 0, nullptr, nullptr, st);
    if (e != hipSuccess) return e;
    REC(5);
#undef REC
    return hipSuccess;
}

}  // namespace qap
