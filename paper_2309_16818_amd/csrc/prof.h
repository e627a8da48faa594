// prof.h - per-kernel HIP event timing shared by the map and the network
// handles (host side only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "mem.h"
#include "mem_internal.h"

namespace memk {

// While `on`, every launcher passed to timed() is bracketed by two events on
// its stream; drain() folds finished pairs into per-name totals.
struct Profiler {
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    bool on = false;
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<int64_t, double>> totals;

    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }

    void drain()
    {
        if (pending.empty()) return;
        for (auto& r : pending) (void)hipEventSynchronize(r.b);  // pairs may be on several streams
        for (auto& r : pending) {
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, r.a, r.b);
            auto& t = totals[r.name];
            t.first += 1;
            t.second += ms;
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }

    template <class F>
    void timed(hipStream_t s, const char* name, F&& f)
    {
        if (!on) {
            f();
            return;
        }
        hipEvent_t a = get(), b = get();
        (void)hipEventRecord(a, s);
        f();
        (void)hipEventRecord(b, s);
        pending.push_back({name, a, b});
        if (pending.size() >= 8192) drain();
    }

    // As timed(), for launchers that take the events themselves (LaunchEv:
    // recorded by the kernels' own dispatch, so without the dispatch gap).
    template <class F>
    void timed_ext(hipStream_t s, const char* name, F&& f)
    {
        (void)s;
        if (!on) {
            f(LaunchEv{});
            return;
        }
        hipEvent_t a = get(), b = get();
        f(LaunchEv{a, b});
        pending.push_back({name, a, b});
        if (pending.size() >= 8192) drain();
    }

    void enable(bool v)
    {
        if (!v) drain();
        on = v;
    }

    // Copies up to max totals out, returns how many there are, and clears them.
    int read(mem_kernel_time* out, int max)
    {
        drain();
        int k = 0;
        for (auto& kv : totals) {
            if (k < max) {
                memset(out[k].name, 0, sizeof out[k].name);
                strncpy(out[k].name, kv.first.c_str(), sizeof out[k].name - 1);
                out[k].launches = kv.second.first;
                out[k].total_ms = kv.second.second;
            }
            k++;
        }
        totals.clear();
        return k;
    }

    void release()
    {
        for (auto& r : pending) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        pending.clear();
        for (auto e : pool) (void)hipEventDestroy(e);
        pool.clear();
    }
};

}  // namespace memk
