// persistent.h -- host-side sizing of persistent launches: as many
// workgroups as the whole device holds at once, for the kernels whose
// workgroups take their work from per-XCD counters until it runs out.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

namespace fspb {

// Resident workgroups of `kernel` (threads per workgroup, dynamic LDS bytes)
// on n_cu compute units, rounded up to a multiple of 8 so that every XCD
// (workgroup q runs on XCD q mod 8) gets the same number.  The occupancy
// query is made once per (kernel, threads, LDS) and kept.
inline int persistent_grid_of(const void* kernel, int threads, size_t lds, int n_cu) {
    static std::mutex mu;
    static std::map<std::tuple<const void*, int, size_t>, int> per_cu_of;
    const auto key = std::make_tuple(kernel, threads, lds);
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = per_cu_of.find(key);
        if (it != per_cu_of.end()) {
            per_cu = it->second;
        } else {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) !=
                    hipSuccess || per_cu < 1) {
                (void)hipGetLastError();
                per_cu = 1;
            }
            per_cu_of[key] = per_cu;
        }
    }
    return 8 * ((per_cu * std::max(n_cu, 8) + 7) / 8);
}

template <class K>
int persistent_grid(K kernel, int threads, size_t lds, int n_cu) {
    return persistent_grid_of(reinterpret_cast<const void*>(kernel), threads, lds, n_cu);
}

}  // namespace fspb
