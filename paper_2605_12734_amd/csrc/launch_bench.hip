// Launch-cost microbenchmark for overdecomposed execution (Section III-A,
// "Managing Overdecomposition"): how much of a fine-grained kernel's cost is
// device-side launch processing.
//
//  - overlap: a fixed amount of work (total_threads threads, `work` dependent
//    integer multiply-adds each) split into nkernels kernels on a pool of
//    non-blocking streams.  Every stream first runs a one-wave gate kernel
//    that polls a flag in pinned host memory; once everything is enqueued,
//    the host sets the flag and all streams proceed at once.  The device
//    makespan (earliest work-workgroup start to latest work-workgroup end,
//    constant-rate wall clock) therefore excludes host submission cost.
//    The gate is released by the host, not by a stream operation: HIP
//    multiplexes streams onto a few hardware queues, so a release enqueued
//    on another stream can sit in the same queue behind a gate and never
//    run.  Every gate gives up after a bounded wait and reports it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "od_runtime.hpp"

namespace {

constexpr int kWorkBlock = 256;
constexpr size_t kStampBytes = 256;   // stamp area ahead of the outputs

__global__ void __launch_bounds__(kWorkBlock)
k_work(uint32_t* __restrict__ out, unsigned long long* __restrict__ stamps, int64_t first, int64_t count,
       int32_t work) {
    if (threadIdx.x == 0) atomicMin(&stamps[0], (unsigned long long)wall_clock64());
    const int64_t i = (int64_t)blockIdx.x * kWorkBlock + threadIdx.x;
    if (i < count) {
        uint32_t x = (uint32_t)(first + i) ^ 0x9E3779B9u;
        for (int32_t k = 0; k < work; ++k) x = x * 1664525u + 1013904223u;
        out[first + i] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(&stamps[1], (unsigned long long)wall_clock64());
}

__global__ void k_stamp_init(unsigned long long* stamps) {
    if (threadIdx.x == 0) {
        stamps[0] = ~0ull;
        stamps[1] = 0ull;
        stamps[2] = 0ull;
    }
}

// Waits until the host sets *flag (system-scope polls), at most wait_ticks
// of the constant-rate clock; a timeout is recorded in stamps[2].
__global__ void k_gate(const uint32_t* flag, unsigned long long* stamps, int64_t wait_ticks) {
    if (threadIdx.x != 0) return;
    const int64_t t0 = wall_clock64();
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) == 0u) {
        __builtin_amdgcn_s_sleep(8);
        if (wall_clock64() - t0 > wait_ticks) {
            atomicOr(&stamps[2], 1ull);
            break;
        }
    }
}

double now_us() {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// One pinned, device-visible host flag per device, kept until the process ends.
uint32_t* host_flag(int dev, std::string& err) {
    static std::vector<uint32_t*> flags(64, nullptr);
    if (dev < 0 || dev >= (int)flags.size()) {
        err = "device index out of range";
        return nullptr;
    }
    if (!flags[dev]) {
        void* p = nullptr;
        hipError_t e = hipHostMalloc(&p, 64, hipHostMallocMapped | hipHostMallocCoherent);
        if (e != hipSuccess) {
            err = std::string("hipHostMalloc(flag): ") + hipGetErrorString(e);
            return nullptr;
        }
        flags[dev] = static_cast<uint32_t*>(p);
    }
    return flags[dev];
}

struct Streams {
    std::vector<hipStream_t> s;
    std::vector<hipEvent_t> e;
    ~Streams() {
        for (auto ev : e) hipEventDestroy(ev);
        for (auto st : s) hipStreamDestroy(st);
    }
    hipError_t create(int n) {
        for (int i = 0; i < n; ++i) {
            hipStream_t st = nullptr;
            hipError_t r = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (r != hipSuccess) return r;
            s.push_back(st);
            hipEvent_t ev = nullptr;
            r = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (r != hipSuccess) return r;
            e.push_back(ev);
        }
        return hipSuccess;
    }
};

// Waits for every event with a wall-clock bound.
bool wait_events(const std::vector<hipEvent_t>& evs, double seconds) {
    const double t_end = now_us() + seconds * 1e6;
    for (auto ev : evs) {
        for (;;) {
            const hipError_t q = hipEventQuery(ev);
            if (q == hipSuccess) break;
            if (q != hipErrorNotReady) return false;
            if (now_us() > t_end) return false;
            std::this_thread::yield();
        }
    }
    return true;
}

}  // namespace

#define OD_HIP_OR_FAIL(call)                                                        \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) return od::fail(OD_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

extern "C" {

size_t od_launch_overlap_bytes(int64_t total_threads) {
    if (total_threads <= 0) return 0;
    return kStampBytes + (size_t)total_threads * sizeof(uint32_t);
}

od_status od_launch_overlap(void* dev_ws, size_t ws_bytes, int64_t total_threads, int32_t nkernels,
                            int32_t nstreams, int32_t work, od_overlap_result* out) {
    try {
        if (!out) return od::fail(OD_EINVAL, "out is NULL");
        std::memset(out, 0, sizeof(*out));
        if (!dev_ws) return od::fail(OD_EINVAL, "dev_ws is NULL");
        if (total_threads <= 0 || total_threads > (int64_t(1) << 31))
            return od::fail(OD_EINVAL, "total_threads must be in [1, 2^31]");
        if (nkernels <= 0 || nkernels > 65536 || nkernels > total_threads)
            return od::fail(OD_EINVAL, "nkernels must be in [1, min(65536, total_threads)]");
        if (nstreams <= 0 || nstreams > 256) return od::fail(OD_EINVAL, "nstreams must be in [1, 256]");
        if (work < 0 || work > (1 << 24)) return od::fail(OD_EINVAL, "work must be in [0, 2^24]");
        if (ws_bytes < od_launch_overlap_bytes(total_threads))
            return od::fail(OD_EINVAL, "workspace smaller than od_launch_overlap_bytes(total_threads)");
        if ((reinterpret_cast<uintptr_t>(dev_ws) & 255) != 0) return od::fail(OD_EINVAL, "dev_ws not 256-byte aligned");
        int dev = 0, khz = 0;
        OD_HIP_OR_FAIL(hipGetDevice(&dev));
        OD_HIP_OR_FAIL(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        if (khz <= 0) return od::fail(OD_EHIP, "device reports no wall-clock rate");
        std::string err;
        uint32_t* flag = host_flag(dev, err);
        if (!flag) return od::fail(OD_EHIP, err);
        uint32_t* dflag = nullptr;
        OD_HIP_OR_FAIL(hipHostGetDevicePointer(reinterpret_cast<void**>(&dflag), flag, 0));
        const int64_t gate_ticks = (int64_t)(10.0 * 1e3 * (double)khz);   // 10 s

        const int ns = std::min(nstreams, nkernels);
        Streams S;
        OD_HIP_OR_FAIL(S.create(ns));
        auto* stamps = static_cast<unsigned long long*>(dev_ws);
        auto* outv = reinterpret_cast<uint32_t*>(static_cast<char*>(dev_ws) + kStampBytes);
        // arm: flag down, stamps reset (completed before any gate is enqueued)
        __atomic_store_n(flag, 0u, __ATOMIC_SEQ_CST);
        hipLaunchKernelGGL(k_stamp_init, dim3(1), dim3(64), 0, S.s[0], stamps);
        OD_HIP_OR_FAIL(hipGetLastError());
        OD_HIP_OR_FAIL(hipStreamSynchronize(S.s[0]));

        // enqueue: a gate per stream, then the kernels round-robin over the streams
        const double t0 = now_us();
        hipError_t enq = hipSuccess;
        for (int s = 0; s < ns && enq == hipSuccess; ++s) {
            hipLaunchKernelGGL(k_gate, dim3(1), dim3(64), 0, S.s[s], dflag, stamps, gate_ticks);
            enq = hipGetLastError();
        }
        const int64_t per = total_threads / nkernels, rem = total_threads % nkernels;
        int64_t first = 0;
        for (int32_t k = 0; k < nkernels && enq == hipSuccess; ++k) {
            const int64_t cnt = per + (k < rem ? 1 : 0);
            const unsigned int blocks = (unsigned int)((cnt + kWorkBlock - 1) / kWorkBlock);
            hipLaunchKernelGGL(k_work, dim3(blocks), dim3(kWorkBlock), 0, S.s[k % ns], outv, stamps, first, cnt,
                               work);
            enq = hipGetLastError();
            first += cnt;
        }
        for (int s = 0; s < ns && enq == hipSuccess; ++s) enq = hipEventRecord(S.e[s], S.s[s]);
        const double t1 = now_us();
        // release from the host (always, also after a failed enqueue)
        __atomic_store_n(flag, 1u, __ATOMIC_SEQ_CST);
        const double t2 = now_us();
        const bool done = wait_events(S.e, 60.0);
        const double t3 = now_us();
        if (enq != hipSuccess) {
            hipDeviceSynchronize();
            return od::fail(OD_EHIP, std::string("enqueue: ") + hipGetErrorString(enq));
        }
        if (!done) return od::fail(OD_ETIMEDOUT, "released kernels did not complete within 60 s");
        unsigned long long st[3] = {0, 0, 0};
        OD_HIP_OR_FAIL(hipMemcpy(st, stamps, sizeof(st), hipMemcpyDeviceToHost));
        if (st[2] != 0) return od::fail(OD_ETIMEDOUT, "a stream gate was not released within its bound");
        out->total_threads = total_threads;
        out->nkernels = nkernels;
        out->nstreams = ns;
        out->work = work;
        out->enqueue_us = t1 - t0;
        out->host_us = t3 - t2;
        out->makespan_us = st[1] >= st[0] ? (double)(st[1] - st[0]) * 1e3 / (double)khz : 0.0;
        return OD_OK;
    } catch (const std::exception& ex) {
        return od::fail(OD_EINVAL, std::string("internal error: ") + ex.what());
    } catch (...) {
        return od::fail(OD_EINVAL, "internal error");
    }
}

}  // extern "C"
