// Launch interface between the host runtime and the kernels.
#pragma once
#include "common.hpp"
#include "philox.hpp"

namespace qap {

// Initialisation (iteration 0) of one instance.
hipError_t launch_init(const InstDesc& d, hipStream_t st);

// Per-stage engine: the stage kernels of one iteration of one instance (S_x,
// velocity, goal + deltas + local search); the bests follow, batched over the
// handle (launch_bests).  If ev is not NULL, events are recorded around the
// stages: ev[2s], ev[2s+1] for stage s (0 S_x, 1 velocity, 2 goal/deltas).
hipError_t launch_plain_step(const InstDesc& d, int mul24, int grid_gd, hipStream_t st, hipEvent_t* ev);

// S_x output of particle k at state tprev into out [n] (device): one wave
// recomputes the selection the step from tprev to tprev + 1 made, from the
// buffers of state tprev.
hipError_t launch_sx_probe(const InstDesc& d, int k, int tprev, uint8_t* out, hipStream_t st);

// Goal (+ deltas) of `count` permutations [count][n] (device) on the int32 path.
// mode 1: eval into goals/deltas; mode 2: initial goals of the particles.
hipError_t launch_goal_delta_i32(const InstDesc& d, int mul24, int grid_gd, const uint8_t* perms, int count,
                                 int mode, long long* goals, long long* deltas, hipStream_t st);

// Swarm bests + finish (best-ever, migration, iteration counter) of every
// instance of a handle: descs [count] device descriptors, smap [total_swarms]
// device map workgroup -> (instance, swarm).
hipError_t launch_bests(const InstDesc* descs, const int2* smap, int total_swarms, int count, int init,
                        hipStream_t st);

// Alg. 2 for the instances descs [count] (device; whole-instance descriptors)
// that are stepped in several stream groups: run after every group finished
// the iteration; each instance migrates if the iteration is a multiple of its
// period.
hipError_t launch_migrate(const InstDesc* descs, int count, hipStream_t st);

// Fused engine: one iteration of every instance of one kernel class (npad,
// byte-split contraction, symmetric, zero diagonals) in one launch.  A class of one instance passes its
// host descriptor `one` (a kernel argument); otherwise one = NULL and descs
// [instances of the class] and blkmap [blocks] (workgroup -> (class-local
// instance, first particle)) are device tables.  Bests follow separately.
// wide: 0 int8, else the byte-split pattern (1 F split, 2 D split, 3 both).
hipError_t launch_fused_class(int npad, int wide, bool sym, bool zd, const InstDesc* one, const InstDesc* descs,
                              const int2* blkmap, int blocks, hipStream_t st);

// Particles (waves) per workgroup of a fused-kernel class.  The waves of a
// workgroup share one LDS copy of F and D.  Larger workgroups where LDS, not
// registers, limited the kernel: the npad-160 int8 symmetric kernels (F, D and
// the per-wave data take 59 KB per 4-wave workgroup: 2 per CU, while the
// registers allow 3 waves per SIMD) take 12 waves; the byte-split kernels with
// one matrix split take 8 at npad 128 with zero diagonals (three planes and 8
// waves' data: 64 KB, 2 workgroups per CU, 4 waves per SIMD as the registers
// allow) and at npad 160 (one workgroup per CU).  4 elsewhere.
constexpr int fused_wpb(int npad, int wide, bool sym, bool zd)
{
    return (wide == 0 && sym && npad == 160)                                                     ? 12
           : ((wide == 1 || wide == 2) && npad == 128 && zd) || ((wide == 1 || wide == 2) && npad == 160) ? 8
                                                                                                            : 4;
}
int fused_particles_per_block(int npad, int wide, bool sym, bool zd);

// Whether the fused kernel covers an instance (int8 path, or the byte-split
// path with F and D symmetric; n <= 160; SecondTarget).
bool fused_supported(const InstDesc& d);

// Whether the byte-split kernels cover a padded size and split pattern (bit 0
// F split, bit 1 D split).
bool split_supported(int npad, int split);

// Goal (+ deltas) of `count` permutations on the int8 or byte-split MFMA path
// (eval only).
hipError_t launch_eval_mfma(const InstDesc& d, const uint8_t* perms, int count, long long* goals,
                            long long* deltas, hipStream_t st);

// Population statistics.  launch_select: for every segment s (values
// [seg_off[s], seg_off[s+1])) and rank j, out[s*nr + j] = the value at
// 1-based position ranks[s*nr + j] in ascending order.  launch_hist:
// out[s*bins + i] = number of values g of segment s with lo <= g < hi and
// ((g - lo) * bins) / (hi - lo) == i.  All pointers are device memory.
hipError_t launch_select(const long long* values, const int* seg_off, int nseg, const long long* ranks, int nr,
                         long long* out, hipStream_t st);
hipError_t launch_hist(const long long* values, const int* seg_off, int nseg, int bins, long long lo, long long hi,
                       unsigned long long* out, hipStream_t st);

// One record of the per-iteration statistics of an instance into slot
// (*iter - 1) % capacity of its ring (see k_history).  All pointers are device
// memory.
hipError_t launch_history(const long long* goals, const int* iter, int m, int S, int nq, const long long* ranks,
                          int bins, long long lo, long long hi, int capacity, int* ring_t, long long* ring_q,
                          unsigned long long* ring_h, hipStream_t st);

// The ranks of a statistics request in parts per million (passed by value).
constexpr int kStatsMaxRanks = 64;
struct StatsRanks {
    int ppm[kStatsMaxRanks];
};

// seg_off [m + 3] and ranks [(m + 1) nq] of a request (see k_stats_setup).
hipError_t launch_stats_setup(int* seg_off, long long* ranks, int m, int S, int P, int nq, const StatsRanks& q,
                              hipStream_t st);

}  // namespace qap
