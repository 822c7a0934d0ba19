// Host-side copy helper shared by the serving loop and the streamed path.
#pragma once

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

namespace ecc {

// Host copies split over a few persistent threads (a single thread's memcpy
// is what limits how fast large requests can be staged).
class Copier {
  public:
    Copier() {
        for (int i = 0; i < kThreads; ++i) th_.emplace_back([this] { loop(); });
    }
    ~Copier() {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    // copy n bytes; returns when every byte is copied
    void copy(char *dst, const char *src, size_t n) {
        const size_t parts = std::min<size_t>(kThreads + 1, std::max<size_t>(1, n / kChunk));
        if (parts <= 1) {
            std::memcpy(dst, src, n);
            return;
        }
        Call call;
        call.left = (int)parts - 1;
        const size_t step = (n / parts + 4095) & ~size_t(4095);
        {
            std::lock_guard<std::mutex> lk(m_);
            for (size_t k = 1; k < parts; ++k) {
                const size_t a = std::min(n, k * step), b = std::min(n, (k + 1) * step);
                if (k + 1 == parts) q_.push_back({dst + a, src + a, n - a, &call});
                else q_.push_back({dst + a, src + a, b - a, &call});
            }
        }
        cv_.notify_all();
        std::memcpy(dst, src, std::min(n, step));  // this thread takes the first part
        std::unique_lock<std::mutex> lk(call.m);
        call.cv.wait(lk, [&call] { return call.left == 0; });
    }

  private:
    static constexpr int kThreads = 7;
    static constexpr size_t kChunk = size_t(1) << 20;
    struct Call {
        std::mutex m;
        std::condition_variable cv;
        int left = 0;
    };
    struct Job {
        char *dst;
        const char *src;
        size_t n;
        Call *call;
    };
    void loop() {
        for (;;) {
            Job j;
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [this] { return stop_ || !q_.empty(); });
                if (q_.empty()) return;
                j = q_.front();
                q_.pop_front();
            }
            std::memcpy(j.dst, j.src, j.n);
            std::lock_guard<std::mutex> lk(j.call->m);
            if (--j.call->left == 0) j.call->cv.notify_all();
        }
    }
    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_;
    std::deque<Job> q_;
    bool stop_ = false;
};

}  // namespace ecc
