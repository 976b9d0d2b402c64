/*
 * CPU oracle for the multi-swarm discrete PSO for the Quadratic Assignment
 * Problem (Szwed & Chmiel, "Multi-swarm PSO algorithm for the Quadratic
 * Assignment Problem: a massive parallel implementation on the OpenCL
 * platform", arXiv:1504.05158).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant generator with the GPU library.
 *
 * Precision: velocities in double; costs and swap deltas in int64.  The one
 * place where floating point decides an integer -- the SecondTarget argmax --
 * is taken in binary32 (the paper's implied 4-byte element type, and the
 * GPU kernel's type): the key of a cell is fl32(x + fl32(v)).
 *
 * Notation (Sec. 2.1 and Sec. 3.1 of the paper): facilities i, j index the
 * COLUMNS of the particle matrices X and V, locations k, l, r index the ROWS.
 * A permutation is stored as p[j] = location of facility j, so that
 * X[p[j]][j] = 1.  The goal is C(p) = sum_ij F[i][j] * D[p[i]][p[j]]
 * (eq. qap with x_ki = [k = p(i)]).
 *
 * Everything the paper leaves open (tie-breaking, random-number streams, the
 * local-improvement step, migration indexing, the init distribution) is fixed
 * by the readings written next to each function below.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox counter-based generator, written from Salmon, Moraes, Dror & Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3" (SC'11), Sec. 4: the
 * 4-word, 10-round variant.  One round maps (c0,c1,c2,c3) with key (k0,k1) to
 * (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)); the key is
 * bumped by the Weyl constants between rounds.                              */

static void philox_round32(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
        philox_round32(c, k);
    }
    memcpy(out, c, sizeof c);
}

/* The 64-bit-word variant of the same construction.  It is not used by the
 * method; it exists so that the round structure above can be pinned against
 * an independent published implementation of Philox4x64-10.               */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    const unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint64_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += 0x9E3779B97F4A7C15ull; k[1] += 0xBB67AE8584CAA73Bull; }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(0xD2E7470EE14C6C93ull, c[0], &hi0, &lo0);
        mulhilo64(0xCA5A826395121157ull, c[2], &hi1, &lo1);
        const uint64_t n0 = hi1 ^ c[1] ^ k[0];
        const uint64_t n2 = hi0 ^ c[3] ^ k[1];
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
    memcpy(out, c, sizeof c);
}

/* Random-number streams of the method (the paper only says "random").
 * Key = (seed low word, seed high word).  Counter = (block, t, particle index
 * within its swarm, swarm index).  Element e of a stream is word (e & 3) of
 * block (e >> 2).  The blocks used are:
 *   t >= 1 (the step that produces iteration t):
 *     block 0, words 0/1  : r2, r3 of eq. (velocity)
 *     block 1 + (i >> 2)  : tie-break word of SecondTarget selection i
 *   t = 0 (initialisation):
 *     elements 0 .. n-2   : Fisher-Yates draws
 *     elements 256 + r*n + c : V(0) cell (r, c)
 *   migration after step t: particle = 0xFFFFFFFF, swarm = 0, element k is the
 *     donor draw of the k-th migration.                                     */
uint32_t orc_word(uint64_t seed, uint32_t element, uint32_t t, uint32_t particle, uint32_t swarm)
{
    const uint32_t ctr[4] = {element >> 2, t, particle, swarm};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[element & 3u];
}

/* Uniform in [0,1): the top 24 bits of a word, scaled by 2^-24 (exact in both
 * binary32 and binary64).                                                   */
double orc_u01(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

/* Integer in [0, m): the high word of the 64-bit product w*m (multiply-shift
 * mapping of a 32-bit word onto a range, without rejection).              */
uint32_t orc_bounded(uint32_t w, uint32_t m) { return (uint32_t)(((uint64_t)w * m) >> 32); }

/* ------------------------------------------------------------------------ */
/* Goal function, eq. (qap): sum over facility pairs (i, j) of the flow f_ij
 * times the distance between their locations.  Diagonal terms are kept: they
 * are the linear installation cost the paper mentions (Sec. 2.1).          */
int64_t orc_cost(int n, const int32_t* F, const int32_t* D, const int32_t* p)
{
    int64_t s = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            s += (int64_t)F[i * n + j] * (int64_t)D[p[i] * n + p[j]];
    return s;
}

/* Pair-exchange move of the local-improvement step.  The paper names local
 * neighbourhood search (Sec. 4.2) and cites pairwise-exchange tabu search but
 * defines no formula; the cost change of exchanging the locations of
 * facilities a and b is the standard pair-exchange delta (Taillard's robust
 * tabu search for the QAP), i.e. C(p o (a b)) - C(p) written out term by term:
 *   (f_aa - f_bb)(d_{p_b p_b} - d_{p_a p_a}) + (f_ab - f_ba)(d_{p_b p_a} - d_{p_a p_b})
 *   + sum_{k != a,b} (f_ak - f_bk)(d_{p_b p_k} - d_{p_a p_k})
 *                  + (f_ka - f_kb)(d_{p_k p_b} - d_{p_k p_a}).
 * out is n*n, out[a*n + b] = out[b*n + a] = delta(a,b), diagonal 0.         */
int64_t orc_delta(int n, const int32_t* F, const int32_t* D, const int32_t* p, int a, int b)
{
#define FF(i, j) ((int64_t)F[(i) * n + (j)])
#define DD(k, l) ((int64_t)D[(k) * n + (l)])
    const int pa = p[a], pb = p[b];
    int64_t d = (FF(a, a) - FF(b, b)) * (DD(pb, pb) - DD(pa, pa))
              + (FF(a, b) - FF(b, a)) * (DD(pb, pa) - DD(pa, pb));
    for (int k = 0; k < n; ++k) {
        if (k == a || k == b) continue;
        const int pk = p[k];
        d += (FF(a, k) - FF(b, k)) * (DD(pb, pk) - DD(pa, pk))
           + (FF(k, a) - FF(k, b)) * (DD(pk, pb) - DD(pk, pa));
    }
    return d;
#undef FF
#undef DD
}

void orc_deltas(int n, const int32_t* F, const int32_t* D, const int32_t* p, int64_t* out)
{
    for (int a = 0; a < n; ++a) {
        out[a * n + a] = 0;
        for (int b = a + 1; b < n; ++b) {
            const int64_t d = orc_delta(n, F, D, p, a, b);
            out[a * n + b] = d;
            out[b * n + a] = d;
        }
    }
}

/* One best-improvement pair exchange: the minimum delta over a < b, ties to
 * the smallest a, then the smallest b; applied only if it is negative.
 * Returns 1 if a swap was made; *best receives the minimum delta.          */
int orc_local_search(int n, const int32_t* F, const int32_t* D, int32_t* p, int64_t* goal,
                     int32_t* best_a, int32_t* best_b, int64_t* best)
{
    int ba = -1, bb = -1;
    int64_t bd = INT64_MAX;
    for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b) {
            const int64_t d = orc_delta(n, F, D, p, a, b);
            if (d < bd) { bd = d; ba = a; bb = b; }
        }
    if (best_a) *best_a = ba;
    if (best_b) *best_b = bb;
    if (best) *best = bd;
    if (ba >= 0 && bd < 0) {
        const int32_t t = p[ba]; p[ba] = p[bb]; p[bb] = t;
        *goal += bd;
        return 1;
    }
    return 0;
}

/* S_x = PickColumn (the second of the three S_x procedures of Sec. 3.1): the
 * columns are visited in a random order and each visited column takes its
 * largest key over the rows not yet taken.  Reading: the order is a
 * Fisher-Yates shuffle of 0 .. n-1 drawn from the particle's stream (for
 * i = n-1 .. 1, swap positions i and bounded(element 4 + n + (n-1-i), i+1)),
 * and equal largest keys in a column go to the k-th such row (ascending),
 * k = bounded(element 4 + v, count) for the v-th visit, as in SecondTarget.
 * There is no depth: cells of X(t) take part like any other.               */
void orc_pick_column(int n, const float* W, uint64_t seed, uint32_t t, uint32_t particle, uint32_t swarm,
                     int32_t* out)
{
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    unsigned char* rowAlive = (unsigned char*)malloc((size_t)n);
    memset(rowAlive, 1, (size_t)n);
    for (int c = 0; c < n; ++c) order[c] = c;
    for (int i = n - 1; i >= 1; --i) {
        const uint32_t j = orc_bounded(orc_word(seed, 4u + (uint32_t)n + (uint32_t)(n - 1 - i), t, particle, swarm),
                                       (uint32_t)(i + 1));
        const int32_t tmp = order[i];
        order[i] = order[j];
        order[j] = tmp;
    }
    for (int v = 0; v < n; ++v) {
        const int c = order[v];
        float best = -INFINITY;
        int found = 0;
        uint32_t count = 0;
        for (int r = 0; r < n; ++r) {
            if (!rowAlive[r]) continue;
            const float key = W[r * n + c];
            if (!found || key > best) { best = key; found = 1; count = 0; }
            if (key == best) ++count;
        }
        uint32_t k = 0;
        if (count > 1) k = orc_bounded(orc_word(seed, 4u + (uint32_t)v, t, particle, swarm), count);
        int sel = -1;
        uint32_t seen = 0;
        for (int r = 0; r < n && sel < 0; ++r) {
            if (!rowAlive[r] || W[r * n + c] != best) continue;
            if (seen == k) sel = r;
            ++seen;
        }
        out[c] = sel;
        rowAlive[sel] = 0;
    }
    free(order);
    free(rowAlive);
}

/* ------------------------------------------------------------------------ */
/* Velocity update, eq. (velocity), with the aggregation S_v of Sec. 3.1:
 *   V' = S_v(c1 V + c2 r2 (P^L - X) + c3 r3 (P^G - X)).
 * P^L, P^G and X are permutation matrices, so (P^L - X) and (P^G - X) are
 * entries in {-1, 0, 1}.  The arithmetic order is
 *   t = c1*v;  t = t + (c2*r2)*a;  t = t + (c3*r3)*b.
 * S_v "raw" clamps every entry to [-vmax, vmax]; "norm" clamps and then
 * divides every column by its L1 norm n_j = sum_i |v_ij| (a column whose
 * norm is 0 stays 0).                                                       */
void orc_velocity(int n, const double* V, const int32_t* p, const int32_t* pl, const int32_t* pg,
                  double c1, double c2, double c3, double r2, double r3, double vmax, int norm,
                  double* Vout)
{
    const double s2 = c2 * r2, s3 = c3 * r3;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            const int x = (p[c] == r), l = (pl[c] == r), g = (pg[c] == r);
            double t = c1 * V[r * n + c];
            t = t + s2 * (double)(l - x);
            t = t + s3 * (double)(g - x);
            if (t > vmax) t = vmax;
            if (t < -vmax) t = -vmax;
            Vout[r * n + c] = t;
        }
    if (!norm) return;
    for (int c = 0; c < n; ++c) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) s += fabs(Vout[r * n + c]);
        if (s > 0.0)
            for (int r = 0; r < n; ++r) Vout[r * n + c] /= s;
    }
}

/* Key matrix of the position update, eq. (position): W = X + V, taken in
 * binary32, W[r][c] = fl32(x_rc + fl32(v_rc)).                               */
void orc_keys(int n, const double* V, const int32_t* p, float* W)
{
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            const float v = (float)V[r * n + c];
            W[r * n + c] = (p[c] == r) ? (1.0f + v) : v;
        }
}

/* S_x = SecondTarget (Alg. 1 of the paper) on the key matrix W with Z the
 * previous solution z (a permutation) and the given depth.
 * Reading of Alg. 1, taken literally: selection i = 0 .. n-1 (0-based) looks
 * at the cells of the remaining rows R and columns C; while i < depth the
 * cells with z_rc = 1 are left out.  M is the set of cells whose key equals
 * the maximum key exactly.  A cell of M is taken uniformly at random: if
 * |M| > 1, the k-th cell of M in column-major order (column ascending, then
 * row ascending) with k = bounded(word, |M|), the word being element 4 + i of
 * the particle's stream for this step.  The chosen row and column leave R
 * and C and the facility of that column is put at that row.
 * Requires 0 <= depth <= n - 1 (the paper's d < n), so M is never empty.
 * ties_out (optional, n entries) receives |M| of every selection.          */
void orc_second_target(int n, const float* W, const int32_t* z, int depth,
                       uint64_t seed, uint32_t t, uint32_t particle, uint32_t swarm,
                       int32_t* out, int32_t* ties_out)
{
    unsigned char* rowAlive = (unsigned char*)malloc((size_t)n);
    unsigned char* colAlive = (unsigned char*)malloc((size_t)n);
    memset(rowAlive, 1, (size_t)n);
    memset(colAlive, 1, (size_t)n);
    for (int i = 0; i < n; ++i) {
        const int skipZ = (i < depth);
        float best = -INFINITY;
        int found = 0;
        for (int c = 0; c < n; ++c) {
            if (!colAlive[c]) continue;
            for (int r = 0; r < n; ++r) {
                if (!rowAlive[r] || (skipZ && z[c] == r)) continue;
                const float key = W[r * n + c];
                if (!found || key > best) { best = key; found = 1; }
            }
        }
        uint32_t count = 0;
        for (int c = 0; c < n; ++c) {
            if (!colAlive[c]) continue;
            for (int r = 0; r < n; ++r) {
                if (!rowAlive[r] || (skipZ && z[c] == r)) continue;
                if (W[r * n + c] == best) ++count;
            }
        }
        uint32_t k = 0;
        if (count > 1) k = orc_bounded(orc_word(seed, 4u + (uint32_t)i, t, particle, swarm), count);
        if (ties_out) ties_out[i] = (int32_t)count;
        int selr = -1, selc = -1;
        uint32_t seen = 0;
        for (int c = 0; c < n && selc < 0; ++c) {
            if (!colAlive[c]) continue;
            for (int r = 0; r < n; ++r) {
                if (!rowAlive[r] || (skipZ && z[c] == r)) continue;
                if (W[r * n + c] == best) {
                    if (seen == k) { selr = r; selc = c; break; }
                    ++seen;
                }
            }
        }
        out[selc] = selr;
        rowAlive[selr] = 0;
        colAlive[selc] = 0;
    }
    free(rowAlive);
    free(colAlive);
}

/* ------------------------------------------------------------------------ */
/* Swarm state.  Particles are numbered g*S + s (swarm g, member s).  V is
 * [P][n][n] row-major (row = location, column = facility); X, PL are [P][n];
 * PG is [m][n]; best_info = {iteration found, swarm, member}.                */

/* Initialisation (iteration 0).  The paper generates random particles on
 * the host (Sec. 3.3) and counts iteration 0 (Table 2, Iter = 0).
 * Reading: X(0) is a Fisher-Yates shuffle of the identity (for i = n-1 .. 1
 * swap p[i] with p[bounded(word_{n-1-i}, i+1)]); V(0)_rc = vmax (2u - 1) with
 * u from element 256 + r*n + c, followed by S_v; P^L = X(0); P^G of a swarm is
 * its best member (lowest index on ties); the best-ever record is the best
 * P^G (lowest swarm on ties) at iteration 0.  No local search at init.      */
static void swarm_reduce(int n, int m, int S, const int32_t* X, const int64_t* goal,
                         int32_t* PG, int64_t* goalPG, int64_t* best_goal, int32_t* best_perm,
                         int32_t* best_info, int32_t t)
{
    for (int g = 0; g < m; ++g) {
        int bj = 0;
        for (int s = 1; s < S; ++s)
            if (goal[(size_t)g * S + s] < goal[(size_t)g * S + bj]) bj = s;
        const size_t pi = (size_t)g * S + bj;
        if (goal[pi] < goalPG[g]) {
            goalPG[g] = goal[pi];
            memcpy(PG + (size_t)g * n, X + pi * n, sizeof(int32_t) * (size_t)n);
        }
        if (goal[pi] < *best_goal) {
            *best_goal = goal[pi];
            memcpy(best_perm, X + pi * n, sizeof(int32_t) * (size_t)n);
            best_info[0] = t; best_info[1] = g; best_info[2] = bj;
        }
    }
}

void orc_init(int n, const int32_t* F, const int32_t* D, int m, int S, double vmax, int norm,
              uint64_t seed, double* V, int32_t* X, int32_t* PL, int64_t* goal, int64_t* goalPL,
              int32_t* PG, int64_t* goalPG, int64_t* best_goal, int32_t* best_perm, int32_t* best_info)
{
    const long P = (long)m * S;
#pragma omp parallel for schedule(dynamic, 4)
    for (long pi = 0; pi < P; ++pi) {
        const uint32_t g = (uint32_t)(pi / S), s = (uint32_t)(pi % S);
        int32_t* x = X + pi * n;
        for (int j = 0; j < n; ++j) x[j] = j;
        for (int e = 0; e <= n - 2; ++e) {
            const int i = n - 1 - e;
            const int j = (int)orc_bounded(orc_word(seed, (uint32_t)e, 0, s, g), (uint32_t)(i + 1));
            const int32_t tmp = x[i]; x[i] = x[j]; x[j] = tmp;
        }
        double* v = V + (size_t)pi * n * n;
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) {
                const double u = orc_u01(orc_word(seed, 256u + (uint32_t)(r * n + c), 0, s, g));
                double t = vmax * (2.0 * u - 1.0);
                if (t > vmax) t = vmax;
                if (t < -vmax) t = -vmax;
                v[r * n + c] = t;
            }
        if (norm)
            for (int c = 0; c < n; ++c) {
                double sum = 0.0;
                for (int r = 0; r < n; ++r) sum += fabs(v[r * n + c]);
                if (sum > 0.0)
                    for (int r = 0; r < n; ++r) v[r * n + c] /= sum;
            }
        goal[pi] = orc_cost(n, F, D, x);
        goalPL[pi] = goal[pi];
        memcpy(PL + pi * n, x, sizeof(int32_t) * (size_t)n);
    }
    for (int g = 0; g < m; ++g) goalPG[g] = INT64_MAX;
    *best_goal = INT64_MAX;
    swarm_reduce(n, m, S, X, goal, PG, goalPG, best_goal, best_perm, best_info, 0);
}

/* Migration, Alg. 2 of the paper, 0-based.  Swarms are sorted by their P^G
 * goal ascending (lower index first on ties) into s_0 .. s_{m-1}; for
 * k = 0 .. d-1 a current solution of a uniformly drawn member of swarm s_k
 * (member bounded(word_k, S) of the migration stream) replaces P^G of swarm
 * s_{m-1-k}, together with its goal, even when it is worse (Sec. 3.2).
 * d < m/2 keeps donors and recipients disjoint.                             */
void orc_migrate(int n, int m, int S, int d, uint64_t seed, uint32_t t,
                 const int32_t* X, const int64_t* goal, int32_t* PG, int64_t* goalPG)
{
    int* order = (int*)malloc(sizeof(int) * (size_t)m);
    for (int g = 0; g < m; ++g) order[g] = g;
    /* insertion sort: stable, so equal goals keep the lower swarm first */
    for (int a = 1; a < m; ++a) {
        const int key = order[a];
        int b = a - 1;
        while (b >= 0 && goalPG[order[b]] > goalPG[key]) { order[b + 1] = order[b]; --b; }
        order[b + 1] = key;
    }
    for (int k = 0; k < d; ++k) {
        const int donor = order[k], recip = order[m - 1 - k];
        const uint32_t j = orc_bounded(orc_word(seed, (uint32_t)k, t, 0xFFFFFFFFu, 0u), (uint32_t)S);
        const size_t pi = (size_t)donor * S + j;
        memcpy(PG + (size_t)recip * n, X + pi * n, sizeof(int32_t) * (size_t)n);
        goalPG[recip] = goal[pi];
    }
    free(order);
}

/* One iteration t-1 -> t of every particle (the step that produces
 * iteration t >= 1), in the order of Sec. 3.1:
 *   1. r2, r3 drawn per particle;
 *   2. X' = SecondTarget(X(t-1) + V(t-1), Z = X(t-1), depth)  (eq. position),
 *      or PickColumn(X(t-1) + V(t-1)) when sx = 1;
 *   3. V(t) = S_v(c1 V + c2 r2 (P^L - X) + c3 r3 (P^G - X)), all at t-1 (eq. velocity);
 *   4. goal of X'; then up to local_search best-improvement pair exchanges,
 *      one after another, stopping at the first one that does not improve;
 *   5. P^L <- X(t) on strict improvement (best position so far);
 * then per swarm: P^G <- the current solution of the best member (lowest
 * index on ties) on strict improvement; the best-ever record likewise; and
 * in migration mode, when t is a multiple of the period, Alg. 2.
 * deltas_out (optional, [P][n][n]) receives the pair-exchange deltas of X'
 * before the exchange.                                                      */
void orc_step(int n, const int32_t* F, const int32_t* D, int m, int S,
              double c1, double c2, double c3, double vmax, int norm, int depth, int sx, int local_search,
              int migrate, int migr_d, int period, uint64_t seed, int32_t t,
              double* V, int32_t* X, int32_t* PL, int64_t* goal, int64_t* goalPL,
              int32_t* PG, int64_t* goalPG, int64_t* best_goal, int32_t* best_perm, int32_t* best_info,
              int64_t* deltas_out)
{
    const long P = (long)m * S;
    const size_t nn = (size_t)n * n;
#pragma omp parallel
    {
        float* W = (float*)malloc(sizeof(float) * nn);
        double* Vn = (double*)malloc(sizeof(double) * nn);
        int32_t* xn = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
#pragma omp for schedule(dynamic, 1)
        for (long pi = 0; pi < P; ++pi) {
            const uint32_t g = (uint32_t)(pi / S), s = (uint32_t)(pi % S);
            const double r2 = orc_u01(orc_word(seed, 0, (uint32_t)t, s, g));
            const double r3 = orc_u01(orc_word(seed, 1, (uint32_t)t, s, g));
            int32_t* x = X + pi * n;
            double* v = V + (size_t)pi * nn;
            orc_keys(n, v, x, W);
            if (sx == 1)
                orc_pick_column(n, W, seed, (uint32_t)t, s, g, xn);
            else
                orc_second_target(n, W, x, depth, seed, (uint32_t)t, s, g, xn, NULL);
            orc_velocity(n, v, x, PL + pi * n, PG + (size_t)g * n, c1, c2, c3, r2, r3, vmax, norm, Vn);
            memcpy(v, Vn, sizeof(double) * nn);
            int64_t gl = orc_cost(n, F, D, xn);
            if (deltas_out) orc_deltas(n, F, D, xn, deltas_out + (size_t)pi * nn);
            for (int q = 0; q < local_search; ++q)
                if (!orc_local_search(n, F, D, xn, &gl, NULL, NULL, NULL)) break;
            memcpy(x, xn, sizeof(int32_t) * (size_t)n);
            goal[pi] = gl;
            if (gl < goalPL[pi]) {
                goalPL[pi] = gl;
                memcpy(PL + pi * n, xn, sizeof(int32_t) * (size_t)n);
            }
        }
        free(W); free(Vn); free(xn);
    }
    swarm_reduce(n, m, S, X, goal, PG, goalPG, best_goal, best_perm, best_info, t);
    if (migrate && migr_d > 0 && period > 0 && (t % period) == 0)
        orc_migrate(n, m, S, migr_d, seed, (uint32_t)t, X, goal, PG, goalPG);
}

void orc_set_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
