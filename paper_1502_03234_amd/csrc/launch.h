// launch.h -- one launch path for every kernel of the library: direct, or recorded for a batch.
//
// Each kernel is a struct K with
//   K::Args                      its arguments (trivially copyable),
//   K::kThreads                  threads per workgroup,
//   K::kWaves                    waves per SIMD to compile for (0: the compiler's choice),
//   static __device__ void run(const Args &a, uint32_t blk, uint32_t nblk)
// where blk / nblk stand for blockIdx.x / gridDim.x. emit<K>(args, blocks, stream) launches
// k_direct<K> at once, or, while a Recorder is installed on the calling thread, appends the
// launch to it without running anything. The serving loop records one detection period of
// every resident system, and where the recorded sequences of several systems name the same
// kernels in the same order it launches each position once for all of them: k_batched<K>
// covers the systems' workgroups back to back, and each workgroup finds its system in a
// table of first workgroups and reads that system's arguments from a device array.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

namespace dcm {

template <class K>
__global__ void __launch_bounds__(K::kThreads) k_direct(typename K::Args a)
{
    K::run(a, blockIdx.x, gridDim.x);
}

template <class K>
__global__ void __launch_bounds__(K::kThreads) __attribute__((amdgpu_waves_per_eu(K::kWaves, K::kWaves)))
k_direct_w(typename K::Args a)
{
    K::run(a, blockIdx.x, gridDim.x);
}

// Workgroup blockIdx.x belongs to system s with first[s] <= blockIdx.x < first[s + 1]
// (first[0] = 0, first[nsys] = the launch's workgroup count; systems without workgroups have
// equal neighbours and are never selected).
__device__ __forceinline__ int batch_system(const uint32_t *first, int nsys, uint32_t blk)
{
    int lo = 0, hi = nsys;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= blk) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The argument table is read-only for the whole launch. Each workgroup copies its system's
// entry once (uniform loads); the copy lives in registers like kernel arguments would.
template <class K>
__global__ void __launch_bounds__(K::kThreads) k_batched(const typename K::Args *__restrict__ tab,
                                                         const uint32_t *__restrict__ first, int nsys)
{
    const int s = batch_system(first, nsys, blockIdx.x);
    const typename K::Args a = tab[s];
    K::run(a, blockIdx.x - first[s], first[s + 1] - first[s]);
}

template <class K>
__global__ void __launch_bounds__(K::kThreads) __attribute__((amdgpu_waves_per_eu(K::kWaves, K::kWaves)))
k_batched_w(const typename K::Args *__restrict__ tab, const uint32_t *__restrict__ first, int nsys)
{
    const int s = batch_system(first, nsys, blockIdx.x);
    const typename K::Args a = tab[s];
    K::run(a, blockIdx.x - first[s], first[s + 1] - first[s]);
}

// One recorded launch: the batched entry of its kernel, its arguments and workgroup count.
struct Launch {
    const void *batched;
    uint32_t threads;
    uint32_t blocks;
    std::vector<uint8_t> args;
};

struct Recorder {
    std::vector<Launch> ops;
};

// The recorder of the calling thread (nullptr: launch directly).
Recorder *&current_recorder();

template <class K>
void emit(const typename K::Args &a, uint32_t blocks, hipStream_t st)
{
    static_assert(std::is_trivially_copyable<typename K::Args>::value, "kernel arguments must be plain data");
    if (Recorder *r = current_recorder()) {
        Launch l;
        if constexpr (K::kWaves > 0) l.batched = reinterpret_cast<const void *>(&k_batched_w<K>);
        else l.batched = reinterpret_cast<const void *>(&k_batched<K>);
        l.threads = (uint32_t)K::kThreads;
        l.blocks = blocks;
        l.args.resize(sizeof(a));
        std::memcpy(l.args.data(), &a, sizeof(a));
        r->ops.push_back(std::move(l));
        return;
    }
    if (blocks == 0) return;
    if constexpr (K::kWaves > 0)
        hipLaunchKernelGGL(k_direct_w<K>, dim3(blocks), dim3(K::kThreads), 0, st, a);
    else
        hipLaunchKernelGGL(k_direct<K>, dim3(blocks), dim3(K::kThreads), 0, st, a);
}

}  // namespace dcm
