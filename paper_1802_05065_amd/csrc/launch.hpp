// launch.hpp -- host entry points of the kernels in kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace fpt {

// `kind`: integrator kind (kUnderExplicit, kOver, kUnderSemiImplicit).
// a.st_mt non-null selects the MT19937 kernels (R = 1, single set only).
hipError_t launch_slice(bool fp64, int kind, int R, bool multi,
                        const SliceArgs& a, uint32_t n_groups, hipStream_t st);
// Workgroups of the slice kernel instance that fit on one CU at once (one
// 256-thread workgroup is one wave per SIMD), 0 if unknown.
int slice_resident_groups(bool fp64, int kind, int R, bool multi, bool mt);
hipError_t launch_init(bool fp64, const SliceArgs& a, uint64_t n_slots,
                       uint64_t n_assign, hipStream_t st);
// Tail compaction (no MT19937 state): count the active slots of `a` into
// a.ctr->compact, then move them to positions [0, count) of `dst` (whose
// first n_dst_slots slots are first marked inactive); the counter must be
// zero before each pass.
hipError_t launch_compact_count(const SliceArgs& a, uint64_t n_slots, hipStream_t st);
hipError_t launch_compact_move(const SliceArgs& src, const SliceArgs& dst, uint64_t n_slots,
                               uint64_t n_dst_slots, hipStream_t st);
// Grouping by set (multi-set plans and the server).  launch_group_count:
// first[0, n_sets) gets the first position of each set's active slots in set
// order, each set starting a wavefront, and ctr->compact the end of the last
// set's wavefronts; counts[0, n_sets) must be zero and is left zero.  The
// move then writes the slots there in dst (n_dst_slots slots, all others
// marked free); n_dst_slots must be at least ctr->compact.
hipError_t launch_group_count(const SliceArgs& a, uint64_t n_slots, unsigned long long* counts,
                              unsigned long long* first, uint64_t n_sets, hipStream_t st);
hipError_t launch_group_move(const SliceArgs& src, const SliceArgs& dst, uint64_t n_slots,
                             uint64_t n_dst_slots, unsigned long long* first, hipStream_t st);
// Refill of the free slots past ctr->compact with the next undrawn replicas,
// after a move in set order; the copy of the state back then also moves the
// cursor past them (advance_cursor).
hipError_t launch_group_refill(bool fp64, const SliceArgs& a, uint64_t n_slots,
                               hipStream_t st);
hipError_t launch_copy_state(const SliceArgs& src, const SliceArgs& dst, uint64_t n_slots,
                             bool advance_cursor, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, uint64_t n,
                           unsigned long long value, hipStream_t st);
hipError_t launch_rng_words(uint64_t seed, uint64_t replica0, uint64_t n_rep,
                            uint64_t block0, uint64_t n_blk, uint32_t* out,
                            hipStream_t st);
hipError_t launch_normals(bool fp64, uint64_t seed, uint64_t replica0,
                          uint64_t n_rep, uint64_t block0, uint64_t n_blk,
                          void* out, hipStream_t st);
// `mt`: 2496 bytes of MT19937 state (FPT_RNG_MT19937), else null.
hipError_t launch_trajectory(bool fp64, int kind, const SetDev& sd,
                             uint64_t replica, int64_t n_steps, double* out_phi,
                             double* out_v, uint4* mt, hipStream_t st);
// `state`: n_rep * 2496 bytes.
hipError_t launch_mt_words(uint64_t seed, uint64_t replica0, uint64_t n_rep,
                           uint64_t block0, uint64_t n_blk, uint4* state,
                           uint32_t* out, hipStream_t st);

}  // namespace fpt
