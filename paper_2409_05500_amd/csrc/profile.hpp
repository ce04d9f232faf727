// Opt-in stage timing (declarations).  Usage at a launch site:
//   { ProfileScope ps("pairwise_moments", stream); kernel<<<..., stream>>>(...); }
#pragma once
#include "common.hpp"

namespace vl {

class ProfileScope {
 public:
  ProfileScope(const char* name, hipStream_t stream);
  ~ProfileScope();
  ProfileScope(const ProfileScope&) = delete;
  ProfileScope& operator=(const ProfileScope&) = delete;

 private:
  const char* name_;
  hipStream_t stream_;
  void* start_ = nullptr;
};

}  // namespace vl
