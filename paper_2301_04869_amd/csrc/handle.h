// Definition of the opaque handle, shared by the C ABI (api.cpp) and the
// interior-point driver (ipm.cpp).
#pragma once

#include <string>
#include <vector>

#include "device.h"
#include "ipm.h"
#include "rkkt.h"
#include "symbolic.h"

struct rkkt_problem {
  rkkt::Sym sym;
  rkkt::DP d{};
  int device = 0;
  std::vector<void*> allocs;
  long long bytes = 0;
  long long idx_bytes = 0;  // of which shared index arrays
  std::string err;
  // stage timing (rkkt_profile_begin / rkkt_profile_end)
  bool prof = false;
  std::vector<hipEvent_t> events;  // 2 per record
  std::vector<int> rec_stage;
  size_t rec_used = 0;
  // interior-point driver workspace (allocated by the first rkkt_solve)
  bool ipm_ready = false;
  rkkt::IpmDev ipm{};
  std::vector<void*> ipm_allocs;
  // captured hot-path pass
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // second stream of rkkt_iterate and its two fork / join event pairs
  hipStream_t side_stream = nullptr;
  hipEvent_t fork_ev[2] = {nullptr, nullptr}, join_ev[2] = {nullptr, nullptr};
};
