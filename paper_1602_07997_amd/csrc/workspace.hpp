// Device arrays carved out of one caller-owned buffer (the library never
// allocates device memory: the caller sizes the buffer with the matching
// *_workspace_bytes query and keeps it alive as long as the handle).
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>

namespace dgw {

constexpr size_t kWorkspaceAlign = 256;

inline size_t align_up(size_t n) { return (n + kWorkspaceAlign - 1) / kWorkspaceAlign * kWorkspaceAlign; }

// Lays out arrays back to back, each on a 256-byte boundary.  With a null
// base it only measures: running the same sequence of take() calls on a null
// arena gives the number of bytes the buffer needs, so the query and the
// carving cannot disagree.  Pointers taken from a buffer that turns out too
// small (fits() false) must not be used.
class Arena {
 public:
  Arena(void* base, size_t bytes) : base_(static_cast<char*>(base)), cap_(bytes) {}

  template <class T>
  T* take(size_t count) {
    off_ = align_up(off_);
    T* p = base_ ? reinterpret_cast<T*>(base_ + off_) : nullptr;
    off_ += std::max<size_t>(count, 1) * sizeof(T);
    return p;
  }
  size_t used() const { return align_up(off_); }
  bool fits() const { return used() <= cap_; }
  size_t capacity() const { return cap_; }

 private:
  char* base_;
  size_t cap_;
  size_t off_ = 0;
};

// A workspace must start on the arena's alignment.
inline bool workspace_aligned(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) % kWorkspaceAlign) == 0;
}

}  // namespace dgw
