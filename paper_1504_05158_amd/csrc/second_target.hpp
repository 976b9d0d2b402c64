// S_x = SecondTarget (Alg. 1 of the paper) for one particle on one wave64.
//
// Input: the particle's V(t) (global, [n][n] unnormalised U with the
// per-column scale Vs, V = fl(U * Vs); row = location, column = facility) and
// its solution z = X(t).  Keys are W = X + V in binary32: a cell
// of Z has key 1 + v, every other cell v.  Selection i = 0 .. n-1 takes the
// maximum key over the remaining rows and columns, leaving out the cells of
// Z while i < depth; exact ties are broken by the k-th tied cell in
// column-major order, k = bounded(stream word 4 + i, number of tied cells).
//
// Work layout: lane l owns columns l, l + 64, ... (CPL of them).  Per column
// it keeps the Z cell's key and a cache of the best non-Z key over the alive
// rows (value, first row, count).  The cache is an upper bound once one of
// its rows may have gone ("stale"); it is recomputed by the whole wave
// (one read of the column) only when the column's bound reaches the current
// maximum.  After the first `depth` selections, the Z cells above every non-Z
// key are taken together; the exact selection (one wave max plus a ballot) is
// needed only between such groups, a few times per particle-iteration, instead
// of the n scans of the remaining matrix of the plain procedure (O(n^3)).
#pragma once
#include "common.hpp"
#include "philox.hpp"
#include <climits>

namespace qap {

template <int CPL>
struct StState {
    float zk[CPL];   // key of the Z cell (1 + v)
    int zr[CPL];     // row of the Z cell
    bool zal[CPL];   // Z row still alive
    float nzv[CPL];  // best non-Z key over alive rows (upper bound if stale)
    int nzr[CPL];    // first row holding nzv (valid if !stale)
    int nzc[CPL];    // number of alive non-Z rows holding nzv (valid if !stale)
    bool stale[CPL];
    bool cal[CPL];   // column not yet assigned
    unsigned rowbits;  // bit j: row lane + 64 j alive
};

// Exact best non-Z key of column c over the alive rows (whole wave).
template <int CPL, class PV>
__device__ __forceinline__ void st_rescan(int n, PV __restrict__ V, PV __restrict__ Vs, int c,
                                          int zr, unsigned rowbits, float& mv, int& mr, int& mc)
{
    const int l = lane_id();
    const float sc = Vs[c];
    float v[CPL];
    bool ok[CPL];
    float best = -INFINITY;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const int r = l + kWave * j;
        ok[j] = (r < n) && ((rowbits >> j) & 1u) && (r != zr);
        v[j] = ok[j] ? __fmul_rn(V[(size_t)r * n + c], sc) : -INFINITY;
        best = fmaxf(best, v[j]);
    }
    const float m = wave_max(best);
    int cnt = 0, first = -1;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const uint64_t b = ballot64(ok[j] && v[j] == m);
        cnt += __popcll(b);
        if (first < 0 && b) first = kWave * j + __ffsll((long long)b) - 1;
    }
    mv = m;
    mr = first;
    mc = cnt;
}

// Row of the k-th tied cell (ascending row) of column c with key m.
template <int CPL, class PV>
__device__ __forceinline__ int st_kth_tied_row(int n, PV __restrict__ V, PV __restrict__ Vs,
                                               int c, int zr, bool withZ, unsigned rowbits, float m, int k)
{
    const int l = lane_id();
    const float sc = Vs[c];
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const int r = l + kWave * j;
        bool ok = (r < n) && ((rowbits >> j) & 1u) && (withZ || r != zr);
        float key = -INFINITY;
        if (ok) {
            const float v = __fmul_rn(V[(size_t)r * n + c], sc);
            key = (r == zr) ? 1.0f + v : v;
        }
        const uint64_t b = ballot64(ok && key == m);
        const int pc = __popcll(b);
        if (k < pc) {
            const uint64_t below = b & ((l == 0) ? 0ull : (~0ull >> (64 - l)));
            const bool mine = ((b >> l) & 1ull) && (__popcll(below) == k);
            const uint64_t w = ballot64(mine);
            return kWave * j + __ffsll((long long)w) - 1;
        }
        k -= pc;
    }
    return -1;  // unreachable when the counts are consistent
}

// Initial per-column cache by a full scan of V (exact, not stale).
template <int CPL, class PV>
__device__ __forceinline__ void st_init_scan(int n, PV __restrict__ V, PV __restrict__ Vs,
                                             const uint8_t* __restrict__ z, StState<CPL>& s)
{
    const int l = lane_id();
    s.rowbits = 0;
#pragma unroll
    for (int j = 0; j < CPL; ++j)
        if (l + kWave * j < n) s.rowbits |= 1u << j;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const int c = l + kWave * k;
        s.cal[k] = c < n;
        s.zr[k] = c < n ? (int)z[c] : -1;
        s.zal[k] = c < n;
        s.zk[k] = -INFINITY;
        s.nzv[k] = -INFINITY;
        s.nzr[k] = -1;
        s.nzc[k] = 0;
        s.stale[k] = false;
    }
    float sc[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) sc[k] = (l + kWave * k < n) ? Vs[l + kWave * k] : 1.0f;
    for (int r = 0; r < n; ++r) {
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const int c = l + kWave * k;
            if (c < n) {
                const float v = __fmul_rn(V[(size_t)r * n + c], sc[k]);
                if (r == s.zr[k]) {
                    s.zk[k] = 1.0f + v;
                } else if (v > s.nzv[k]) {
                    s.nzv[k] = v; s.nzr[k] = r; s.nzc[k] = 1;
                } else if (v == s.nzv[k]) {
                    s.nzc[k] += 1;
                }
            }
        }
    }
}

// Per-wave LDS scratch of the selection: dead-row / dead-column flags and
// the row claims of a tie group.
template <int S>
struct StLds {
    uint8_t deadrow[kMaxN];
    uint8_t deadcol[kMaxN];
    uint8_t claim[kMaxN];
};

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A run of selections among the cells holding the current maximum m when
// every column holds at most one tied Z cell (tz) and at most one tied non-Z
// cell of known row (tn).  Keys never change and no removal raises one, so
// the tied set only shrinks, by the chosen column and row, and stays the set
// of maximal cells until it is empty: each selection i draws the k-th of the
// T cells left (column-major order, k = bounded(stream word 4 + i, T)), and
// the run continues without rescans.  Selections are recorded in out and the
// dead flags (cal cleared for chosen columns; the rest of the per-lane state
// is brought up to date by st_sync).  Returns the number of selections made.
template <int CPL, class L>
__device__ int st_tie_run(int n, int i, StState<CPL>& s, bool (&tz)[CPL], bool (&tn)[CPL], uint8_t* out, L* lds,
                          uint64_t seed, uint32_t iter, uint32_t member, uint32_t swarm)
{
    const int l = lane_id();
    // stream words of 64 blocks ahead, block b0 + l on lane l
    uint32_t b0 = (4u + (uint32_t)i) >> 2;
    Philox4 pw = philox4x32_10(b0 + (uint32_t)l, iter, member, swarm, (uint32_t)seed, (uint32_t)(seed >> 32));
    int taken = 0;
    for (;;) {
        int cnt[CPL], incl[CPL], tot[CPL], T = 0;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            cnt[k] = (int)tz[k] + (int)tn[k];
            incl[k] = wave_incl_scan_i32(cnt[k]);
            tot[k] = readlane_i32(incl[k], kWave - 1);
            T += tot[k];
        }
        if (T == 0) break;
        int kk = 0;
        if (T > 1) {
            const uint32_t e = 4u + (uint32_t)(i + taken);
            if ((e >> 2) - b0 >= (uint32_t)kWave) {
                b0 = e >> 2;
                pw = philox4x32_10(b0 + (uint32_t)l, iter, member, swarm, (uint32_t)seed, (uint32_t)(seed >> 32));
            }
            const int src = (int)((e >> 2) - b0), el = (int)(e & 3u);
            const uint32_t w = (uint32_t)readlane_i32((int)(el == 0 ? pw.w[0] : el == 1 ? pw.w[1] : el == 2 ? pw.w[2] : pw.w[3]), src);
            kk = (int)bounded_u32(w, (uint32_t)T);
        }
        int c = -1, r = -1;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            if (c >= 0) break;
            if (kk < tot[k]) {
                const uint64_t hit = ballot64(cnt[k] > 0 && incl[k] > kk && incl[k] - cnt[k] <= kk);
                const int owner = __ffsll((long long)hit) - 1;
                const int within = kk - readlane_i32(incl[k] - cnt[k], owner);
                const int za = tz[k] ? s.zr[k] : INT_MAX, nb = tn[k] ? s.nzr[k] : INT_MAX;
                const int lo = min(za, nb), hi = max(za, nb);
                c = owner + kWave * k;
                r = readlane_i32(within == 0 ? lo : hi, owner);
            } else {
                kk -= tot[k];
            }
        }
        if (c < 0 || c >= n || r < 0 || r >= n) break;  // unreachable when the flags are consistent
        if (l == 0) {
            out[c] = (uint8_t)r;
            lds->deadcol[c] = 1;
            lds->deadrow[r] = 1;
        }
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            if (l + kWave * k == c) { s.cal[k] = false; tz[k] = false; tn[k] = false; }
            if (tz[k] && s.zr[k] == r) tz[k] = false;
            if (tn[k] && s.nzr[k] == r) tn[k] = false;
        }
        ++taken;
        if (i + taken >= n) break;
    }
    return taken;
}

// One selection by the exact procedure: returns the column (uniform) and
// sets selr.  A column's candidate is exact unless its cache is stale; a
// stale cache only bounds the true value from above, so the maximum over all
// candidates is the true maximum as soon as every column that reaches it is
// exact.  Only those columns are rescanned (lazy argmax).
//
// Tie groups (lds != NULL, Z cells included): when the cells holding the
// maximum lie in pairwise distinct rows and columns, taking one of them
// removes none of the others and lowers no key, so the next selections take
// all of them, whatever the random order; they are taken at once (written to
// out and the dead flags, cal cleared), *group = their number, and the
// return value is -1.  The per-lane state other than cal is then stale until
// st_sync.
template <int CPL, class L, class PV>
__device__ int st_generic_pick(int n, int i, bool skipZ, PV __restrict__ V, PV __restrict__ Vs,
                               StState<CPL>& s, uint64_t seed, uint32_t iter, uint32_t member, uint32_t swarm,
                               int& selr, L* lds = nullptr, uint8_t* out = nullptr, int* group = nullptr)
{
    const int l = lane_id();
    float cv[CPL], m;
    int cc[CPL], cr[CPL];
    uint64_t bal[CPL];
    for (;;) {
        bool inexact[CPL];
        float lbest = -INFINITY;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            float v = s.nzv[k];
            int cnt = s.nzc[k], row = s.nzr[k];
            bool inx = s.stale[k];
            if (!skipZ && s.zal[k]) {
                if (s.zk[k] > s.nzv[k]) { v = s.zk[k]; cnt = 1; row = s.zr[k]; inx = false; }
                else if (s.zk[k] == s.nzv[k]) { cnt += 1; row = min(row, s.zr[k]); }
            }
            if (!s.cal[k] || (!inx && cnt == 0)) { v = -INFINITY; inx = false; }
            cv[k] = v; cc[k] = cnt; cr[k] = row; inexact[k] = inx;
            lbest = fmaxf(lbest, v);
        }
        m = wave_max(lbest);
        bool again = false;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            uint64_t b = ballot64(inexact[k] && cv[k] == m);
            again |= b != 0;
            while (b) {
                const int owner = __ffsll((long long)b) - 1;
                b &= b - 1;
                const int c = owner + kWave * k;
                const int zr = readlane_i32(s.zr[k], owner);
                float mv; int mr, mc;
                st_rescan<CPL>(n, V, Vs, c, zr, s.rowbits, mv, mr, mc);
                if (l == owner) { s.nzv[k] = mv; s.nzr[k] = mr; s.nzc[k] = mc; s.stale[k] = false; }
            }
        }
        if (!again) break;
    }
    int ncols = 0;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        bal[k] = ballot64(cv[k] == m && cv[k] != -INFINITY);
        ncols += __popcll(bal[k]);
    }
    int selc = -1;
    selr = -1;
    if (ncols == 1) {
#pragma unroll
        for (int k = 0; k < CPL; ++k)
            if (bal[k]) {
                const int owner = __ffsll((long long)bal[k]) - 1;
                if (readlane_i32(cc[k], owner) == 1) {
                    selc = owner + kWave * k;
                    selr = readlane_i32(cr[k], owner);
                }
            }
    }
    if (selc < 0 && lds) {
        // a group of single-cell tied columns in distinct rows is taken at once
        bool multi = false;
#pragma unroll
        for (int k = 0; k < CPL; ++k) multi |= ballot64(((bal[k] >> l) & 1ull) && cc[k] > 1) != 0;
        if (!multi) {
#pragma unroll
            for (int k = 0; k < CPL; ++k)
                if ((bal[k] >> l) & 1ull) lds->claim[cr[k]] = (uint8_t)(l + kWave * k);
            wave_lds_sync();
            bool clash = false;
#pragma unroll
            for (int k = 0; k < CPL; ++k)
                clash |= ballot64(((bal[k] >> l) & 1ull) && lds->claim[cr[k]] != (uint8_t)(l + kWave * k)) != 0;
            if (!clash) {
#pragma unroll
                for (int k = 0; k < CPL; ++k)
                    if ((bal[k] >> l) & 1ull) {
                        const int c = l + kWave * k;
                        out[c] = (uint8_t)cr[k];
                        lds->deadcol[c] = 1;
                        lds->deadrow[cr[k]] = 1;
                        s.cal[k] = false;
                    }
                *group = ncols;
                return -1;
            }
        }
        // otherwise a run of selections while the tied set stays of the simple kind
        bool tz[CPL], tn[CPL], bad = false;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const bool in = (bal[k] >> l) & 1ull;
            const bool nzt = in && s.nzv[k] == m;
            tz[k] = in && s.zal[k] && s.zk[k] == m;
            tn[k] = nzt && s.nzc[k] == 1;
            bad |= nzt && s.nzc[k] != 1;
        }
        if (ballot64(bad) == 0) {
            *group = st_tie_run<CPL>(n, i, s, tz, tn, out, lds, seed, iter, member, swarm);
            return -1;
        }
    }
    if (selc < 0) {
        // |M| tied cells: take the k-th in column-major order
        int mycnt = 0;
#pragma unroll
        for (int k = 0; k < CPL; ++k) mycnt += ((bal[k] >> l) & 1ull) ? cc[k] : 0;
        const int total = wave_sum_i32(mycnt);
        const uint32_t w = stream_word(seed, 4u + (uint32_t)i, iter, member, swarm);
        int kk = (int)bounded_u32(w, (uint32_t)total);
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            if (selc >= 0) break;
            const int x = ((bal[k] >> l) & 1ull) ? cc[k] : 0;
            const int incl = wave_incl_scan_i32(x);
            const int tot = readlane_i32(incl, 63);
            if (kk < tot) {
                const uint64_t hit = ballot64(incl > kk && x > 0 && incl - x <= kk);
                const int owner = __ffsll((long long)hit) - 1;
                const int before = readlane_i32(incl - x, owner);
                const int c = owner + kWave * k;
                const int zr = readlane_i32(s.zr[k], owner);
                const bool withZ = !skipZ && readlane_i32((int)s.zal[k], owner);
                selc = c;
                // a column holding one tied cell has its row in the (exact) cache
                selr = readlane_i32(cc[k], owner) == 1
                           ? readlane_i32(cr[k], owner)
                           : st_kth_tied_row<CPL>(n, V, Vs, c, zr, withZ, s.rowbits, m, kk - before);
            } else {
                kk -= tot;
            }
        }
    }
    return selc;
}

// Per-lane bookkeeping of a selection (row selr, column selc).
template <int CPL>
__device__ __forceinline__ void st_apply(StState<CPL>& s, int selc, int selr)
{
    const int l = lane_id();
    if (l == (selr & 63)) s.rowbits &= ~(1u << (selr >> 6));
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        if (selc == l + kWave * k) s.cal[k] = false;
        if (s.cal[k]) {
            if (s.zr[k] == selr) s.zal[k] = false;
            // the cached row left, or the cached value was tied: bound only
            if (!s.stale[k] && (s.nzr[k] == selr || s.nzc[k] > 1)) s.stale[k] = true;
        }
    }
}

// Bring the per-lane state up to date after selections recorded only in the
// dead-row / dead-column flags.
template <int CPL, class L>
__device__ __forceinline__ void st_sync(int n, StState<CPL>& s, const L* lds)
{
    const int l = lane_id();
    unsigned rb = 0;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const int r = l + kWave * j;
        if (r < n && !lds->deadrow[r]) rb |= 1u << j;
    }
    s.rowbits = rb;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const int c = l + kWave * k;
        if (s.cal[k] && lds->deadcol[c]) s.cal[k] = false;
        if (s.cal[k]) {
            if (s.zal[k] && lds->deadrow[s.zr[k]]) s.zal[k] = false;
            if (!s.stale[k] && ((s.nzr[k] >= 0 && lds->deadrow[s.nzr[k]]) || s.nzc[k] > 1)) s.stale[k] = true;
        }
    }
}

// Largest non-Z bound over the alive columns (an upper bound of every non-Z
// key; -inf when no alive column has a non-Z cell left).
template <int CPL>
__device__ __forceinline__ float st_nonz_bound(const StState<CPL>& s)
{
    float b = -INFINITY;
#pragma unroll
    for (int k = 0; k < CPL; ++k)
        if (s.cal[k]) b = fmaxf(b, s.nzv[k]);
    return wave_max(b);
}

// Run the n selections.  Writes out[c] = chosen row for every column c < n.
// The first `depth` selections (Z cells excluded) use the exact procedure.
// Afterwards: taking a Z cell never removes another Z cell (they share no row
// or column), and every non-Z key is bounded by the largest cached non-Z
// bound, which only falls.  So all alive Z cells whose key exceeds that bound
// are exactly the next selections, in some order -- ties among them only
// reorder picks that are all taken -- and they are taken at once.  The
// selection after them (a non-Z cell or a Z cell not above the bound) uses
// the exact procedure, then the bound is recomputed and the next group taken.
// lds: the wave's scratch.
template <int CPL, class PV>
__device__ void st_select(int n, int depth, PV __restrict__ V, PV __restrict__ Vs,
                          StState<CPL>& s, uint8_t* out, StLds<CPL>* lds, uint64_t seed, uint32_t iter,
                          uint32_t member, uint32_t swarm)
{
    static_assert(CPL == 1 || CPL == 2 || CPL == 4, "column slots per lane must be 1, 2 or 4");
    const int l = lane_id();
    for (int r = l; r < kMaxN; r += kWave) { lds->deadrow[r] = 0; lds->deadcol[r] = 0; }
    wave_lds_sync();
    int i = 0;
    for (; i < depth && i < n; ++i) {
        int selr;
        const int selc = st_generic_pick<CPL, StLds<CPL>>(n, i, true, V, Vs, s, seed, iter, member, swarm, selr);
        if (selc < 0 || selc >= n || selr < 0 || selr >= n) continue;
        if (l == 0) { out[selc] = (uint8_t)selr; lds->deadcol[selc] = 1; lds->deadrow[selr] = 1; }
        st_apply<CPL>(s, selc, selr);
    }
    wave_lds_sync();
    while (i < n) {
        // ---- every alive Z cell above the non-Z bound, at once
        const float bound = st_nonz_bound<CPL>(s);
        int taken = 0;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const bool take = s.cal[k] && s.zal[k] && s.zk[k] > bound;
            taken += __popcll(ballot64(take));
            if (take) {
                const int c = l + kWave * k, zr = s.zr[k];
                out[c] = (uint8_t)zr;
                lds->deadcol[c] = 1;
                lds->deadrow[zr] = 1;
                s.cal[k] = false;
            }
        }
        i += taken;
        if (i >= n) break;
        wave_lds_sync();
        if (taken) st_sync<CPL>(n, s, lds);
        // ---- one exact selection, or a row/column-disjoint tie group at once
        int selr, group = 0;
        const int selc = st_generic_pick<CPL>(n, i, false, V, Vs, s, seed, iter, member, swarm, selr, lds, out, &group);
        if (group > 0) {
            i += group;
            wave_lds_sync();
            st_sync<CPL>(n, s, lds);
            continue;
        }
        ++i;
        if (selc < 0 || selc >= n || selr < 0 || selr >= n) continue;
        if (l == 0) { out[selc] = (uint8_t)selr; lds->deadcol[selc] = 1; lds->deadrow[selr] = 1; }
        st_apply<CPL>(s, selc, selr);
        wave_lds_sync();
    }
}

}  // namespace qap
