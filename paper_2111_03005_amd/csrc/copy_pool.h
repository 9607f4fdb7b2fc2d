// Host-side parallel copy of a list of memory segments (plain C++, no HIP):
// used by the serving loop for the edges of admitted requests and the
// results of finished ones.
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace gesmc {

// Host copies of the serving loop (edges into the pinned staging, results out
// of it) spread over a few persistent threads: one thread moves ~8 GB/s, and
// the worker waits for these copies with the device idle.  Every call gets
// its own job object, so a thread still finishing an earlier call never
// touches a later one.
class CopyPool {
  public:
    struct Seg {
        void *dst;
        const void *src;
        size_t bytes;
    };
    explicit CopyPool(unsigned nthreads) {
        for (unsigned i = 0; i < nthreads; ++i) th_.emplace_back([this] { loop(); });
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (std::thread &t : th_) t.join();
    }
    // Copies every segment; returns when all bytes are in place.
    void copy(const std::vector<Seg> &segs) {
        auto job = std::make_shared<Job>();
        for (const Seg &g : segs)
            for (size_t o = 0; o < g.bytes; o += kChunk)
                job->chunks.push_back(Seg{(char *)g.dst + o, (const char *)g.src + o, std::min(kChunk, g.bytes - o)});
        if (job->chunks.empty()) return;
        if (th_.empty() || job->chunks.size() == 1) {
            for (const Seg &c : job->chunks) memcpy(c.dst, c.src, c.bytes);
            return;
        }
        job->left = job->chunks.size();
        {
            std::lock_guard<std::mutex> lk(mu_);
            cur_ = job;
            ++gen_;
        }
        cv_.notify_all();
        run(*job);
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [&] { return job->left.load() == 0; });
        cur_.reset();
    }

  private:
    static constexpr size_t kChunk = 2u << 20;
    struct Job {
        std::vector<Seg> chunks;
        std::atomic<size_t> next{0}, left{0};
    };
    void run(Job &j) {
        size_t k;
        while ((k = j.next.fetch_add(1)) < j.chunks.size()) {
            memcpy(j.chunks[k].dst, j.chunks[k].src, j.chunks[k].bytes);
            if (j.left.fetch_sub(1) == 1) {
                std::lock_guard<std::mutex> lk(mu_);
                done_.notify_all();
            }
        }
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            std::shared_ptr<Job> job;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                job = cur_;
            }
            if (job) run(*job);
        }
    }
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_;
    std::shared_ptr<Job> cur_;
    uint64_t gen_ = 0;
    bool stop_ = false;
};


}  // namespace gesmc
