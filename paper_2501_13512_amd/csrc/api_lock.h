// Serialisation of HIP graph capture against the HIP calls that the runtime
// refuses while any thread of the process is capturing (allocation, free,
// stream and event creation or destruction, device-wide synchronisation).
#pragma once
#include <shared_mutex>

namespace vie {

std::shared_mutex& api_mutex();

// Held around one such call (never nested on a thread).
struct ApiShared {
  std::shared_lock<std::shared_mutex> lock;
  ApiShared() : lock(api_mutex()) {}
};

}  // namespace vie
