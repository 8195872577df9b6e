// Helpers shared by the library's translation units (defined in api.hip);
// hidden from the public interface.
#pragma once

#include <stdint.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "device.h"
#include "hjg.h"

#define HJG_HIDDEN __attribute__((visibility("hidden")))

extern "C" HJG_HIDDEN int hjg_internal_fail(int code, const char* msg);

namespace hjg {
namespace detail {

// Argument checks of a problem record (the same as every sweep entry point).
HJG_HIDDEN int check_problem(const hjg_problem* p);
// Only the state dimension and the datum fields (for records that describe a
// level function, such as an avoid set).
HJG_HIDDEN int check_datum(const hjg_problem* p);
HJG_HIDDEN DatumP datum_params(const hjg_problem* p);
HJG_HIDDEN HamP ham_params(const hjg_problem* p);
// Philox counter tag of (problem, time step, iteration).
HJG_HIDDEN uint32_t make_tag(uint32_t pid, uint32_t step, uint32_t iter);

// A roctx range around one interface call: profilers that record markers
// (rocprofv3 --marker-trace) attribute the call's kernels to it.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace detail
}  // namespace hjg
