// Kernel launch that reports the status of that launch itself.
#pragma once
#include <hip/hip_runtime.h>

#include <tuple>

namespace mifft {

// Launches __global__ function k with the given arguments (converted to its
// parameter types) and returns hipLaunchKernel's own status: an error left
// pending by earlier, unrelated work is neither reported as this launch's
// failure nor cleared, as a hipGetLastError() after the launch would do.
template <typename... P, typename... A>
inline hipError_t launch_kernel(void (*k)(P...), dim3 grid, dim3 block, size_t shmem, hipStream_t stream,
                                A&&... a)
{
    static_assert(sizeof...(P) == sizeof...(A), "argument count differs from the kernel's parameters");
    std::tuple<P...> args{static_cast<P>(a)...};
    void* ptrs[sizeof...(P) > 0 ? sizeof...(P) : 1] = {nullptr};
    std::apply(
        [&ptrs](auto&... x) {
            int i = 0;
            ((ptrs[i++] = static_cast<void*>(&x)), ...);
        },
        args);
    return hipLaunchKernel(reinterpret_cast<const void*>(k), grid, block, ptrs, shmem, stream);
}

}  // namespace mifft
