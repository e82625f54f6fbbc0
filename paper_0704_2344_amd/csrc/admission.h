// The server's admission pass, kept free of device code so the scheduling
// policy can be driven by a host-only simulation.
#pragma once

#include <cstdint>
#include <vector>

namespace femh {

// One pass over the waiting requests in arrival order (queued_bytes: each
// one's estimated device footprint).  At most `window` of them are looked
// at, from the front; each is admitted while fewer than max_slots requests
// run, if its estimate fits the budget beside the resident bytes (a request
// that does not fit is passed over, so a later, smaller one can start).
// Returns the admitted positions in order and adds their bytes to resident.
inline std::vector<int> plan_admissions(const std::vector<int64_t>& queued_bytes, int64_t& resident, int64_t budget,
                                        int running, int max_slots, int window = 16) {
  std::vector<int> out;
  const int n = (int)queued_bytes.size();
  for (int i = 0; i < n && i < window; ++i) {
    if (running + (int)out.size() >= max_slots) break;
    if (resident + queued_bytes[i] <= budget) {
      resident += queued_bytes[i];
      out.push_back(i);
    }
  }
  return out;
}

}  // namespace femh
