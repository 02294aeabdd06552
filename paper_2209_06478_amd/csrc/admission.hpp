// Admission queue of the serving loop: pure host logic (no HIP), so it can
// be exercised on the CPU with scripted arrivals.
//
// Requests queue in arrival order.  A unit of work is admitted only when the
// request at the head fits: a free slot, and its footprint within the HBM
// budget left (0 = no budget).  A large head is admitted alone.  A small head
// is admitted together with every other queued small request that also fits
// once the ones before it are admitted, up to batch_max, in arrival order;
// large requests stay queued in place.  A head that does not fit blocks the
// queue (first come, first served: no small request overtakes a large head
// that waits for budget).  release() returns a finished request's slot and
// bytes.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <vector>

namespace dsm {

class Admission {
  public:
    struct Item {
        uint64_t id;
        size_t footprint;
        bool small;
    };

    Admission(int slots, size_t budget, int batch_max) : slots_(slots), budget_(budget), batch_max_(batch_max) {}

    void push(uint64_t id, size_t footprint, bool small) { q_.push_back({id, footprint, small}); }

    // The next unit of work, or an empty vector when the head cannot be
    // admitted now (or nothing is queued).  *small tells which path it takes.
    std::vector<Item> take(bool *small) {
        std::vector<Item> out;
        if (q_.empty() || !fits(q_.front())) return out;
        const bool s = q_.front().small;
        if (small) *small = s;
        admit(q_.begin(), out);
        if (s)
            for (auto it = q_.begin(); it != q_.end() && (int)out.size() < batch_max_;) {
                if (it->small && fits(*it)) it = admit(it, out);
                else ++it;
            }
        return out;
    }

    void release(size_t footprint) {
        in_flight_--;
        bytes_ -= footprint;
    }

    bool fits(const Item &r) const { return in_flight_ < slots_ && (budget_ == 0 || bytes_ + r.footprint <= budget_); }
    bool empty() const { return q_.empty(); }
    size_t queued() const { return q_.size(); }
    int in_flight() const { return in_flight_; }
    size_t bytes_in_flight() const { return bytes_; }
    size_t budget() const { return budget_; }

  private:
    std::deque<Item>::iterator admit(std::deque<Item>::iterator it, std::vector<Item> &out) {
        in_flight_++;
        bytes_ += it->footprint;
        out.push_back(*it);
        return q_.erase(it);
    }

    std::deque<Item> q_;
    int slots_;
    size_t budget_;
    int batch_max_;
    int in_flight_ = 0;
    size_t bytes_ = 0;
};

}  // namespace dsm
