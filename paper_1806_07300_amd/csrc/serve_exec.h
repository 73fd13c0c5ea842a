// The device side of the serving loop, behind an interface: the scheduler
// (serve.cpp) owns admission, coalescing, tickets and retries; an executor
// owns the staging rings' memory and runs launches.  The HIP executor
// (serve_hip.cpp) is the product path; the CPU fake executor (serve.cpp)
// stands in for the device in tests of the scheduler.
#pragma once

#include <stdint.h>
#include <stddef.h>

#include <memory>
#include <vector>

#include "forestpack.h"

struct fp_packed;

namespace fp {

// One request of a launch: its forest, its rows at x_start of the row ring
// (n_rows x F fp32, packed), its votes at v_start of the vote ring
// (n_rows x C int32).
struct ServeItem {
    const fp_packed* packed;
    int64_t n_rows;
    int32_t F, C;
    size_t x_start, x_size, v_start, v_size;
};

class ServeExecutor {
   public:
    virtual ~ServeExecutor() = default;
    // Allocates the rings (xcap + vcap bytes on the device and mirrored on
    // the host) and n_slots launch slots.
    virtual int init(const fp_server_opts& o, size_t xcap, size_t vcap, int n_slots) = 0;
    virtual uint8_t* host_rows() = 0;   // the host mirror of the row ring
    virtual uint8_t* host_votes() = 0;  // the host mirror of the vote ring
    virtual int device() const = 0;     // device id, -1 for none
    // Validates a forest for this executor (called by fp_server_add_forest).
    virtual int check_forest(const fp_packed* p) = 0;
    // Called once from the scheduler thread before any launch.
    virtual void bind_thread() {}
    // Starts slot `slot`'s launch for `batch` (rows to the device, the
    // launch, votes back) without waiting.  An error means nothing is in
    // flight on the slot afterwards.
    virtual int issue(int slot, const std::vector<ServeItem>& batch) = 0;
    // FP_OK: the slot's launch is done and its votes are in the host vote
    // ring; FP_ENOTREADY: still running; anything else: it failed.
    virtual int query(int slot) = 0;
    // Waits until nothing runs on the slot (after a failure, before its
    // ring space is reused).
    virtual void drain(int slot) = 0;
};

// HIP executor on the current device (serve_hip.cpp).
std::unique_ptr<ServeExecutor> make_hip_executor();
// CPU fake executor (serve.cpp).
std::unique_ptr<ServeExecutor> make_fake_executor();

}  // namespace fp
