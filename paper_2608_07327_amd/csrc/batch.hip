// Batched solve of many independent systems (placeholder until the
// persistent batched kernel lands).
#include <string>

#include "runtime.hpp"

namespace mb {

mbpcg_status batch_entry(int32_t, const mbpcg_system*, const mbpcg_params&, mbpcg_info*, mbpcg_mem,
                         hipStream_t, std::string& err) {
    err = "batched solve not built";
    return MBPCG_ERR_UNSUPPORTED;
}

}  // namespace mb
