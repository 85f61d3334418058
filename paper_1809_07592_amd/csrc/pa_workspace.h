// One stream's library workspace: a device buffer that grows on demand and
// is leased to one call at a time.
//
// A call takes the lease before it reads the buffer's address and keeps it
// until every launch that uses the buffer is enqueued.  Growing the buffer
// first waits for the stream (the work already enqueued on the old buffer),
// then frees and reallocates it.  Because the lease covers the span from
// reading the address to enqueueing the work, another host thread on the
// same stream cannot free the buffer between the two: its own growth waits
// for the lease, and by then the first call's work is on the stream, so the
// wait covers it.
//
// Dev supplies the device operations, each returning true on success:
//   bool sync();                     wait for all work enqueued on the stream
//   bool release(void *p);           free a buffer
//   bool allocate(void **p, size_t); allocate a buffer
// and `const char *what` naming the operation that failed.  The library
// binds it to HIP; the host tests bind it to a simulated stream.
#pragma once

#include <cstddef>
#include <mutex>

namespace pa {

template <class Dev>
struct StreamWorkspace {
    static constexpr size_t kMinBytes = (size_t)1 << 20;

    std::mutex use;  // the lease
    void *ptr = nullptr;
    size_t bytes = 0;

    // At least `need` bytes at *out, with the lease moved into *hold;
    // *grew (optional) tells whether the buffer was (re)allocated.  On
    // failure returns false with dev.what set and holds nothing.
    bool acquire(Dev &dev, size_t need, void **out, std::unique_lock<std::mutex> *hold, bool *grew = nullptr) {
        std::unique_lock<std::mutex> lk(use);
        if (grew) *grew = bytes < need;
        if (bytes < need) {
            if (ptr) {
                if (!dev.sync()) return false;
                if (!dev.release(ptr)) return false;
                ptr = nullptr;
                bytes = 0;
            }
            const size_t alloc = need > kMinBytes ? need : kMinBytes;
            if (!dev.allocate(&ptr, alloc)) return false;
            bytes = alloc;
        }
        *out = ptr;
        *hold = std::move(lk);
        return true;
    }
};

}  // namespace pa
