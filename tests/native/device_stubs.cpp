// Host-only stand-ins for the library's device operations, so that the
// packer and the serving scheduler can be built and run under sanitizers on
// a machine without a GPU: every device operation reports FP_ENODEV.
#include <memory>

#include "fp_internal.h"
#include "serve_exec.h"

namespace fp {

int device_upload(void*, const void*, size_t, void*, int*) { return fp_set_error(FP_ENODEV, "no device in this build"); }

int device_leaf_counts(const uint8_t*, size_t, const Header&, int32_t, const float*, int64_t, int64_t, int32_t*,
                       void*) {
    return fp_set_error(FP_ENODEV, "no device in this build");
}

namespace {
class NoDevice final : public ServeExecutor {
   public:
    int init(const fp_server_opts&, size_t, size_t, int) override {
        return fp_set_error(FP_ENODEV, "no device in this build");
    }
    uint8_t* host_rows() override { return nullptr; }
    uint8_t* host_votes() override { return nullptr; }
    int device() const override { return -1; }
    int check_forest(const fp_packed*) override { return FP_ENODEV; }
    int issue(int, const std::vector<ServeItem>&) override { return FP_ENODEV; }
    int query(int) override { return FP_ENODEV; }
    void drain(int) override {}
};
}  // namespace

std::unique_ptr<ServeExecutor> make_hip_executor() { return std::unique_ptr<ServeExecutor>(new NoDevice()); }

}  // namespace fp
