// Internal definitions shared by the host builder and the HIP decoder.
#pragma once

#include <cstdint>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "met_bp.h"

namespace met {

// Records a message for met_last_error() and returns `code`.
int fail(int code, const char *fmt, ...);
void clear_error();

// Runs the body of a C-ABI entry point: a C++ exception (above all a failed
// allocation of a host container) becomes an error code and a message for
// met_last_error() instead of crossing the C boundary.
template <class F>
int guarded(const char *name, F &&body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc &) {
    return fail(MET_ENOMEM, "%s: out of host memory", name);
  } catch (const std::exception &e) {
    return fail(MET_ESTATE, "%s: %s", name, e.what());
  } catch (...) {
    return fail(MET_ESTATE, "%s: unexpected exception", name);
  }
}

// Check shapes with a compiled kernel path: (message edges, leaf edges) per
// check.  "Message" edges go to variable nodes of degree >= 2; "leaf" edges go
// to degree-1 variable nodes, whose variable-to-check message is always the
// channel LLR and which therefore never enter the iterations.  (4, 0) is the
// 4-check of the MET profiles when degree-1 nodes are iterated like the others.
constexpr int kNumFixedShapes = 7;
constexpr int kShapeMsg[kNumFixedShapes] = {3, 2, 12, 11, 6, 5, 4};
constexpr int kShapeLeaf[kNumFixedShapes] = {1, 1, 0, 0, 0, 0, 0};
constexpr int kShapeGeneric = kNumFixedShapes;  // per-check row pointers

constexpr int kMaxClasses = 16;
constexpr int kMaxDevices = 16;

// A run of consecutive checks decoded by one kernel shape.
struct CheckClass {
  int32_t shape;
  int32_t n_msg, n_leaf;   // per check (fixed shapes); 0 for generic
  int64_t first_check, n_checks;
  int64_t first_msg, first_leaf;  // first message / leaf edge of the run
};

// Device copy of the adjacency (one allocation, typed views).
struct DeviceCode {
  bool ready = false;
  void *base = nullptr;
  size_t bytes = 0;
  const int32_t *edge_msgvn = nullptr;   // [E12] message VN index of each message edge (check order)
  const int8_t *edge_type = nullptr;     // [E12]
  const int32_t *vn_ptr = nullptr;       // [N2+1]
  const int32_t *vn_edges = nullptr;     // [E12] message edge positions, grouped by VN
  const int32_t *leaf_vn = nullptr;      // [EL] user index of each leaf edge's VN (check order)
  const int8_t *leaf_type = nullptr;     // [EL]
  const int32_t *msg_vn_user = nullptr;  // [N2]
  const int32_t *vn_slot = nullptr;      // [N] >= 0: message VN index; < 0: -(leaf edge) - 1
  const int32_t *chk_msg_ptr = nullptr;  // [M+1]
  const int32_t *chk_leaf_ptr = nullptr; // [M+1]
  const int32_t *all_vn = nullptr;       // [E] user VN of every edge (check order)
  const int32_t *all_ptr = nullptr;      // [M+1]
  const int32_t *chk_pos = nullptr;      // [M] check index of the code -> decoder check order
};

}  // namespace met

struct met_code {
  uint64_t uid = 0;  // unique per handle in this process (caches key on it, not on the address)
  int64_t N = 0, M = 0, E = 0;
  int32_t ntypes = 1;
  // Edge list in (check, type, VN) order.
  std::vector<int32_t> vn, cn;
  std::vector<int8_t> et;
  std::vector<int32_t> chk_ptr;  // [M+1]
  // Derived decoder structures.
  int64_t N2 = 0, E12 = 0, EL = 0;
  std::vector<int32_t> msg_vn_user, edge_msgvn, vn_ptr, vn_edges, leaf_vn_user, vn_slot;
  std::vector<int32_t> chk_msg_ptr, chk_leaf_ptr;  // [M+1] in decoder check order
  std::vector<int32_t> chk_orig;                   // [M] decoder check -> check of the code
  std::vector<int32_t> chk_pos;                    // [M] check of the code -> decoder check
  std::vector<int8_t> edge_type_msg, leaf_type;
  std::vector<met::CheckClass> classes;
  int32_t max_check_deg = 0, max_vn_deg = 0;
  int64_t n_deg1 = 0;
  std::mutex mu;
  met::DeviceCode dev[met::kMaxDevices];
  // The same graph with every variable node iterated, degree-1 nodes included
  // (no leaf edges); built on first use by decodes with MET_NO_DEG1_SKIP.
  met_code *all_vns = nullptr;
};

namespace met {
// Builds the derived structures from (vn, cn, et); returns MET_OK or an error.
// With skip_deg1 false, degree-1 variable nodes are message nodes like the
// others (no leaf edges).
int finalize_code(met_code *c, bool skip_deg1 = true);
// The code's view with every variable node iterated (c->all_vns), built on
// first use.
int all_vns_view(const met_code *c, const met_code **out);
// Uploads the adjacency to the current device if needed (decoder side).
int device_code(const met_code *c, const DeviceCode **out);
}  // namespace met
