// Staging ring for the small per-launch arguments of the evaluation calls
// (device pointer tables, task lists, per-limb constants).
//
// Bytes are written into a ring of pinned host memory and copied
// asynchronously, on the context's stream, into a device ring of the same
// size, so no call has to wait for the device before returning.  A region is
// handed out again only after every kernel that may read it has finished:
// callers enqueue their launches and then call fence(), which records a
// completion marker (an event) covering everything staged so far; put() waits
// for the oldest markers only when the ring has wrapped onto regions they
// cover.
//
// The position logic is a template over the marker type so that it can be
// exercised on the host with a simulated stream (tests/test_staging_ring.py).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <stdexcept>

namespace csrmf {

// Ops must provide:
//   Marker record();          enqueue a marker behind all work enqueued so far
//   void wait(Marker);        block until the marker's work has completed
//   void release(Marker);     the marker is no longer needed
template <class Ops, class Marker>
class RingPositions {
public:
    explicit RingPositions(size_t capacity) : cap_(capacity) {}

    // Reserve `bytes` (a multiple of kAlign, at most the capacity); returns the
    // byte offset into the ring.  Waits for markers as needed.
    size_t reserve(size_t bytes, Ops& ops) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        if (bytes == 0) bytes = kAlign;
        if (bytes > cap_) throw std::length_error("staging request larger than the ring");
        uint64_t start = head_;
        const uint64_t off = start % cap_;
        if (off + bytes > cap_) start += cap_ - off;          // do not straddle the end
        const uint64_t need_free_to = start + bytes;         // logical positions up to here get overwritten
        // logical position p reuses the physical bytes of p - cap_; those must be consumed
        while (consumed_ + cap_ < need_free_to) {
            if (marks_.empty()) {
                // everything still unconsumed was staged after the last fence: the
                // current call alone needs more than the ring holds
                throw std::length_error("staging ring overrun within one call");
            }
            Mark m = marks_.front();
            marks_.pop_front();
            ops.wait(m.marker);
            ops.release(m.marker);
            consumed_ = m.pos;
        }
        head_ = need_free_to;
        return (size_t)(start % cap_);
    }

    // Everything reserved so far is consumed once the work enqueued up to now completes.
    void fence(Ops& ops) {
        if (head_ == fenced_) return;
        marks_.push_back(Mark{head_, ops.record()});
        fenced_ = head_;
    }

    // Forget all markers after the caller has synchronised the stream.
    void drained(Ops& ops) {
        for (auto& m : marks_) ops.release(m.marker);
        marks_.clear();
        consumed_ = fenced_ = head_;
    }

    uint64_t head() const { return head_; }
    uint64_t consumed() const { return consumed_; }
    size_t pending_marks() const { return marks_.size(); }

    static constexpr size_t kAlign = 256;

private:
    struct Mark {
        uint64_t pos;
        Marker marker;
    };
    size_t cap_;
    uint64_t head_ = 0;      // next free logical position
    uint64_t fenced_ = 0;    // head at the last fence
    uint64_t consumed_ = 0;  // logical positions below this are free
    std::deque<Mark> marks_;
};

}  // namespace csrmf
