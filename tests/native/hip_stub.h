// Hooks of the CPU stand-in for the HIP runtime (hip_stub.cpp), used by the
// stand-ins of the kernel launchers and by the host-code test driver.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <functional>

// Run op on stream s in order with its other work (or record it into the
// stream's capture).
hipError_t stub_enqueue(hipStream_t s, std::function<void()> op);
// Inconsistencies the stand-ins found (bad frees, launch plans that do not
// fit their grids, reads of a model's buffers that are not resident).
long stub_errors();
void stub_report(const char* msg);
// Device allocations still live, in bytes, and all live allocations.
size_t stub_live_device_bytes();
size_t stub_live_allocations();
