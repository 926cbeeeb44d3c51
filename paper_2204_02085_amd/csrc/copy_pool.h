// Host-side helper of the host-memory pipeline: a pool of threads that
// copies one host buffer into another (pageable caller memory into
// page-locked staging slots and back).  Plain C++ with no device calls, so
// it also builds into host-only checks.
#pragma once

#include <algorithm>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

namespace wfa {

// A pool of host threads that copy one buffer into another in equal parts
// (the caller copies one part itself); used to move pageable caller memory
// through page-locked staging slots at several times one thread's rate.
class CopyPool {
  public:
    explicit CopyPool(unsigned workers) {
        try {
            for (unsigned i = 0; i < workers; i++) th_.emplace_back([this, i] { run(i + 1); });
        } catch (...) {
            // fewer workers: the caller covers the missing parts
        }
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    void copy(void* dst, const void* src, size_t bytes) {
        const unsigned parts = (unsigned)th_.size() + 1;
        if (parts == 1 || bytes < ((size_t)1 << 20)) {
            std::memcpy(dst, src, bytes);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            dst_ = (unsigned char*)dst;
            src_ = (const unsigned char*)src;
            bytes_ = bytes;
            parts_ = parts;
            left_ = parts - 1;
            gen_++;
        }
        cv_.notify_all();
        part(0);
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [&] { return left_ == 0; });
    }

  private:
    // part i of `parts_` equal parts, each a multiple of 64 bytes except the
    // last; the parts cover all bytes_ bytes (rounding the share up first)
    void part(unsigned i) {
        const size_t per = ((bytes_ + parts_ - 1) / parts_ + 63) & ~(size_t)63;
        const size_t a = std::min(bytes_, per * i), b = std::min(bytes_, per * (i + 1));
        if (b > a) std::memcpy(dst_ + a, src_ + a, b - a);
    }
    void run(unsigned i) {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
            }
            part(i);
            {
                std::lock_guard<std::mutex> lk(mu_);
                left_--;
            }
            done_.notify_one();
        }
    }
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_;
    uint64_t gen_ = 0;
    unsigned parts_ = 1, left_ = 0;
    bool stop_ = false;
    unsigned char* dst_ = nullptr;
    const unsigned char* src_ = nullptr;
    size_t bytes_ = 0;
};

}  // namespace wfa
