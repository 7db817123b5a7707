// Host-resident 3DES-ECB, two ways.
//
// Direct: the buffers are pinned host memory, mapped into the device's
// address space, and the bitsliced kernel reads and writes them there over
// PCIe; both directions of the link carry data at once and nothing is
// staged.
//
// Staged (any host memory): the buffer is processed in chunks staged
// through device slots.  Each slot has its own stream, on which its chunks
// are copied in, encrypted in place and copied out, in that order.  The
// slots' streams run side by side, so the copy to the device of one chunk,
// the kernel of another and the copy back of a third overlap.
#include <deque>
#include <mutex>

#include "internal.h"

namespace tdes {

namespace {

struct DeviceStreams {
    int device;
    hipStream_t s[TDES_HOST_MAX_SLOTS];
};

std::mutex g_host_mutex;             // one pipeline at a time per process
std::deque<DeviceStreams> g_streams;  // one entry per device used; kept until exit

// The current device's slot streams, created at its first use (default
// priority, not synchronising with the null stream).
hipError_t device_streams(hipStream_t (&out)[TDES_HOST_MAX_SLOTS]) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    for (const DeviceStreams &d : g_streams)
        if (d.device == dev) {
            for (int i = 0; i < TDES_HOST_MAX_SLOTS; i++) out[i] = d.s[i];
            return hipSuccess;
        }
    DeviceStreams d{dev, {}};
    for (int i = 0; i < TDES_HOST_MAX_SLOTS; i++) {
        e = hipStreamCreateWithFlags(&d.s[i], hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (int j = 0; j < i; j++) (void)hipStreamDestroy(d.s[j]);
            return e;
        }
    }
    g_streams.push_back(d);
    for (int i = 0; i < TDES_HOST_MAX_SLOTS; i++) out[i] = d.s[i];
    return hipSuccess;
}

}  // namespace

hipError_t run_host_pipeline(const BitsliceKeys &k, const uint8_t *h_in, uint8_t *h_out,
                             size_t nbytes, uint8_t *d_work, size_t n_slots, size_t chunk) {
    std::lock_guard<std::mutex> lock(g_host_mutex);
    hipStream_t s[TDES_HOST_MAX_SLOTS];
    hipError_t first = device_streams(s);
    if (first != hipSuccess) return first;
    const size_t chunks = (nbytes + chunk - 1) / chunk;
    const size_t used = chunks < n_slots ? chunks : n_slots;
    // A slot is reused only on its own stream, after its previous chunk's
    // copy back; in place, a chunk's output range is its own input range,
    // copied in earlier on the same stream.
    for (size_t i = 0; i < chunks && first == hipSuccess; i++) {
        const size_t slot = i % n_slots, off = i * chunk;
        const size_t len = nbytes - off < chunk ? nbytes - off : chunk;
        uint8_t *d = d_work + slot * chunk;
        hipError_t e = hipMemcpyAsync(d, h_in + off, len, hipMemcpyHostToDevice, s[slot]);
        if (e == hipSuccess) e = launch_bitslice(k, d, d, len, s[slot]);
        if (e == hipSuccess) e = hipMemcpyAsync(h_out + off, d, len, hipMemcpyDeviceToHost, s[slot]);
        first = e;
    }
    // wait for every stream that received work, also after a failure
    for (size_t j = 0; j < used; j++) {
        const hipError_t e = hipStreamSynchronize(s[j]);
        if (first == hipSuccess) first = e;
    }
    return first;
}

// Device address of the host range [h, h + n): h must be pinned host memory
// mapped into the device's address space, and the whole range must lie in
// the allocation that holds h (a kernel must never touch an unmapped page).
// A refused range is an argument error, not a device failure: the HIP
// runtime's last-error state is cleared, or the caller's next HIP call (a
// torch launch, say) would report it as its own.
hipError_t mapped_range(const void *h, size_t n, uint8_t **d) {
    void *a = nullptr;
    hipError_t e = hipHostGetDevicePointer(&a, const_cast<void *>(h), 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, a);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    const uintptr_t lo = (uintptr_t)base, p = (uintptr_t)a;
    if (p < lo || p - lo > size || n > size - (p - lo)) return hipErrorInvalidValue;
    *d = static_cast<uint8_t *>(a);
    return hipSuccess;
}

hipError_t run_host_direct(const BitsliceKeys &k, const uint8_t *d_in, uint8_t *d_out,
                           size_t nbytes) {
    std::lock_guard<std::mutex> lock(g_host_mutex);
    hipStream_t s[TDES_HOST_MAX_SLOTS];
    hipError_t e = device_streams(s);
    if (e != hipSuccess) return e;
    e = launch_bitslice(k, d_in, d_out, nbytes, s[0]);
    const hipError_t w = hipStreamSynchronize(s[0]);
    return e != hipSuccess ? e : w;
}

}  // namespace tdes
