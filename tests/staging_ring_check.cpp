// Host check of the staging ring's position logic (csrc/staging.h) against a
// simulated in-order stream.  Every staged region is written on the host at
// put time, copied to the "device" ring by a queued copy, and read by queued
// "kernels"; the check fails if a copy finds its host bytes already
// overwritten or a kernel finds its device bytes changed.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <set>
#include <stdexcept>
#include <vector>

#include "../paper_2509_03024_amd/csrc/staging.h"

struct Sim {
    struct Op { int kind; size_t off, len; uint32_t tag; int marker; };   // 0 copy, 1 read, 2 marker
    std::deque<Op> q;
    std::vector<uint32_t> host, dev;       // tag per 256-byte unit
    std::set<int> done;
    int next_marker = 0;
    long errors = 0;
    explicit Sim(size_t cap) : host(cap / 256, 0), dev(cap / 256, 0) {}
    void step() {
        if (q.empty()) return;
        Op op = q.front();
        q.pop_front();
        for (size_t u = op.off / 256; u < (op.off + op.len) / 256; ++u) {
            if (op.kind == 0) {
                if (host[u] != op.tag) ++errors;      // host bytes overwritten before the copy ran
                dev[u] = host[u];
            } else if (op.kind == 1) {
                if (dev[u] != op.tag) ++errors;       // device bytes overwritten before the kernel ran
            }
        }
        if (op.kind == 2) done.insert(op.marker);
    }
};

struct Ops {
    Sim* s;
    int record() { int m = s->next_marker++; s->q.push_back({2, 0, 0, 0, m}); return m; }
    void wait(int m) { while (!s->done.count(m)) { if (s->q.empty()) throw std::logic_error("wait on a marker never queued"); s->step(); } }
    void release(int) {}
};

int main(int argc, char** argv) {
    const size_t cap = 1 << 20;
    const int iters = argc > 1 ? atoi(argv[1]) : 200000;
    std::mt19937_64 rng(12345);
    Sim sim(cap);
    Ops ops{&sim};
    csrmf::RingPositions<Ops, int> ring(cap);
    uint32_t tag = 1;
    long puts = 0;
    for (int it = 0; it < iters; ++it) {
        const int n_put = 1 + (int)(rng() % 5);
        std::vector<std::pair<size_t, size_t>> regs;
        std::vector<uint32_t> tags;
        for (int p = 0; p < n_put; ++p) {
            size_t bytes = 1 + rng() % (rng() % 8 == 0 ? cap / 6 : 4096);
            size_t off = ring.reserve(bytes, ops);
            size_t len = (bytes + 255) / 256 * 256;
            if (off % 256 || off + len > cap) { printf("bad offset\n"); return 1; }
            ++tag;
            for (size_t u = off / 256; u < (off + len) / 256; ++u) sim.host[u] = tag;
            sim.q.push_back({0, off, len, tag, 0});
            regs.push_back({off, len});
            tags.push_back(tag);
            ++puts;
        }
        for (size_t r = 0; r < regs.size(); ++r)          // kernels of this call read every region
            sim.q.push_back({1, regs[r].first, regs[r].second, tags[r], 0});
        ring.fence(ops);
        const int steps = (int)(rng() % 12);               // the device makes some progress
        for (int s = 0; s < steps; ++s) sim.step();
    }
    while (!sim.q.empty()) sim.step();
    // one call that needs more than the ring must be refused, not corrupt data
    bool refused = false;
    try {
        ring.reserve(cap / 2 + 256, ops);
        ring.reserve(cap / 2 + 256, ops);
    } catch (const std::length_error&) {
        refused = true;
    }
    printf("puts %ld errors %ld refused %d\n", puts, sim.errors, (int)refused);
    return (sim.errors == 0 && refused) ? 0 : 1;
}
