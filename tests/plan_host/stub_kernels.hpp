// stub_kernels.hpp -- kernel table of the CPU stand-in of the HIP runtime:
// the batched plan code gets its kernel entry points from
// sweep::batched_kernels / sweep::backward_kernels, which the stand-in
// replaces by addresses of table entries that list each kernel's parameters
// (size and whether it is a device pointer that may be null).
#pragma once

#include <cstddef>
#include <string>
#include <vector>

namespace stub {

enum ArgKind { kValue, kDevicePtr, kNullablePtr };

struct ArgSig {
    size_t size;
    ArgKind kind;
};

struct KernelSig {
    const char* name;
    std::vector<ArgSig> args;
};

// The table entry of a kernel entry point handed out by the stand-in, or null.
const KernelSig* lookup(const void* fn);
// Every table entry (for comparing parameter counts with the kernel sources).
std::vector<const KernelSig*> all_kernels();
// For the arc-length kernels, which take a work list by path degree of
// (sweep, first span index or u-sample) per block: whether the `grid`
// entries a launch reads name sweeps of that degree and start inside the
// sweep; "" if so (or for other kernels), else what is wrong.  Reads the
// stand-in's device memory (host memory).
std::string check_work_list(const void* fn, unsigned grid, const std::vector<std::vector<unsigned char>>& args);
// Violations counted so far (printed when print is set); reset.
int report(bool print);
void reset_violations();

}  // namespace stub
