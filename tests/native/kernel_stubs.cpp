// Stand-ins for the kernel launchers of pss_kernels.hip (and the scratch
// address lookup of pss_noalloc.hip), so that the host code of pss_api.hip
// can be linked into a host-only test program without the device code.  Each
// reports hipErrorNotSupported; the host checks never reach them.
#include "../../paper_2305_05245_amd/csrc/pss_internal.hpp"

namespace pss {
namespace {
hipError_t none() { return hipErrorNotSupported; }
}  // namespace

hipError_t scratch_setup(int) { return none(); }
hipError_t read_device_error(uint32_t *, bool) { return none(); }
hipError_t read_device_error_async(uint32_t *, hipStream_t) { return none(); }
hipError_t launch_tile_sort(int, bool, const void *, const uint32_t *, void *, uint32_t *, uint64_t,
                            uint64_t, uint32_t, int, void *, hipStream_t) { return none(); }
hipError_t launch_seg_plan(const uint64_t *, uint32_t, uint64_t, const SegPlanPtrs &, uint32_t,
                           uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, hipStream_t) {
  return none();
}
hipError_t launch_seg_tile_sorts(int, bool, const void *, const uint32_t *, void *, void *,
                                 uint32_t *, uint32_t *, void *, const uint64_t *,
                                 const SegPlanPtrs &, uint32_t, uint64_t, uint32_t, hipStream_t) {
  return none();
}
hipError_t launch_corank(int, const void *, const RunGeom &, uint32_t *, void *, uint64_t *,
                         hipStream_t, const void *) { return none(); }
hipError_t launch_corank_sampled(int, const void *, const RunGeom &, uint32_t *, const uint32_t *,
                                 const uint32_t *, hipStream_t, const void *, const RunGeom *) {
  return none();
}
hipError_t launch_merge(int, int, const void *, const uint32_t *, void *, uint32_t *,
                        const RunGeom &, const uint32_t *, const uint64_t *, int, void *,
                        uint32_t *, hipStream_t, const MergeAlt *) { return none(); }
hipError_t launch_partition_offsets(const RunGeom &, const uint32_t *, uint64_t *, uint64_t *,
                                    hipStream_t) { return none(); }
hipError_t launch_split_table(const RunGeom &, const uint32_t *, uint64_t *, hipStream_t) {
  return none();
}
hipError_t launch_unmap_copy(int, const void *, void *, uint64_t, hipStream_t) { return none(); }
hipError_t launch_sort_merge(int, bool, const void *, const uint32_t *, void *, uint32_t *,
                             const RunGeom &, const uint32_t *, const uint64_t *, int,
                             hipStream_t) { return none(); }
hipError_t launch_record_keys(int, const void *, uint64_t, uint32_t, uint32_t, void *, uint32_t *,
                              hipStream_t) { return none(); }
hipError_t launch_record_gather(const void *, void *, const uint32_t *, uint64_t, uint32_t,
                                hipStream_t) { return none(); }
hipError_t launch_psrs_samples(int, const void *, const RunGeom &, void *, hipStream_t) {
  return none();
}
hipError_t launch_psrs_partition(int, const void *, const RunGeom &, const void *, uint64_t,
                                 uint64_t *, void *, uint64_t *, hipStream_t) { return none(); }
hipError_t launch_psrs_chunks(const RunGeom &, const uint64_t *, uint64_t *, uint64_t *,
                              uint64_t *, hipStream_t) { return none(); }
}  // namespace pss
