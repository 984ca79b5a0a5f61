// perm_mod3_batch_packed_noalloc: the packed batch call with its work set in a
// static device array, for callers that cannot allocate device memory.
//
// The array below is one work set (the layout perm_mod3_batch_packed carves
// from its growable buffer) sized for PERM_NOALLOC_MAX_COUNT matrices of the
// largest order.  In host code its name is only a stand-in: the device address
// is looked up with hipGetSymbolAddress once per device, when that device's
// context is made, and only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <cstring>

#include "perm3.h"
#include "perm3_internal.h"
#include "perm3_runtime.h"

namespace perm3 {
namespace {

constexpr int64_t NOALLOC_MAX_ROWS = (int64_t)PERM_NOALLOC_MAX_COUNT * PERM_MAX_N;
constexpr size_t NOALLOC_BYTES = workset_layout(PERM_NOALLOC_MAX_COUNT, NOALLOC_MAX_ROWS, true).off[9];
static_assert(NOALLOC_BYTES == PERM_NOALLOC_SCRATCH_BYTES, "perm3.h states the array's size");

}  // namespace
}  // namespace perm3

// One per device, held until the process ends.
static __device__ __align__(256) uint8_t scratch[perm3::NOALLOC_BYTES];

namespace perm3 {

int32_t noalloc_init(Context &c)
{
    // the context's device is current here (get_context runs on it)
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return set_error(PERM_EDEVICE, "no device address for the static work set");
    c.noalloc_scratch = ptr;
    return PERM_OK;
}

}  // namespace perm3

using namespace perm3;

extern "C" int32_t perm_mod3_batch_packed_noalloc(const uint64_t *planes_dev, const int64_t *row_off_dev,
                                                  const int32_t *ns_dev, int32_t count, uint8_t *out_dev,
                                                  uint64_t *hist_dev, void *stream)
{
    set_error_index(-1);
    if (count < 0 || count > PERM_NOALLOC_MAX_COUNT)
        return set_error(PERM_EINVAL, "count = %d is outside [0, %d], the allocation-free call's limit", count,
                         PERM_NOALLOC_MAX_COUNT);
    if (count == 0) return PERM_OK;
    if (!planes_dev || !row_off_dev || !ns_dev || !out_dev) return set_error(PERM_EINVAL, "null pointer argument");
    const hipStream_t st = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (st) {
        const hipError_t e = hipStreamIsCapturing(st, &cs);
        if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    }
    if (cs == hipStreamCaptureStatusInvalidated)
        return set_error(PERM_EDEVICE, "the stream's capture has been invalidated");
    Context *c = nullptr;
    int32_t rc;
    if (cs == hipStreamCaptureStatusActive) {
        // making the context on a first call is no stream operation
        hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
        hipError_t e = hipThreadExchangeStreamCaptureMode(&mode);
        if (e != hipSuccess) return hip_fail(e, "hipThreadExchangeStreamCaptureMode");
        rc = get_context(&c);
        (void)hipThreadExchangeStreamCaptureMode(&mode);
    } else {
        rc = get_context(&c);
    }
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    const WorkSet w = workset_carve(c->noalloc_scratch, PERM_NOALLOC_MAX_COUNT, NOALLOC_MAX_ROWS, true);
    Launch L;
    memset(&L, 0, sizeof L);
    L.pack_kind = 1;
    L.planes_dev = planes_dev;
    L.row_off_dev = row_off_dev;
    L.ns_dev = ns_dev;
    L.count = count;
    L.out_dev = out_dev;
    L.hist_dev = hist_dev;
    L.cls = count == 1 ? PERM_TUNE_LARGE : PERM_TUNE_BATCH;
    L.defer = count > 1 ? 1 : 0;
    // the one-launch path's accumulator words must start at zero: a fill kernel clears them
    // (the plan kernel of a larger call clears its own tallies, counts and queue)
    L.zero_acc = count <= SMALL_PLAN_MAX ? 1 : 0;
    return c->enqueue(L, w, c->tn(L.cls), st, false);
}
