#include "twod.hpp"

namespace riros {

int run_twod(const DevDesign&, TwoDWorkspace&, const uint64_t*, uint32_t, const riros_fault*, const float*,
             uint32_t, int, const TwoDParams&, uint32_t*, uint64_t*, hipEvent_t, hipEvent_t, hipStream_t,
             std::string& err)
{
    err = "two-dimensional mode is not available in this build";
    return RIROS_EINVAL;
}

void twod_free(TwoDWorkspace& ws)
{
    if (ws.mem) (void)hipFree(ws.mem);
    ws.mem = nullptr;
    ws.bytes = 0;
}

}  // namespace riros
