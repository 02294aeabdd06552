// Admission queue of the serving loop: pure host logic (no HIP), so it can
// be exercised on the CPU with scripted arrivals.
//
// Requests queue in arrival order.  A unit of work is admitted only when the
// request at the head fits: a free slot, and its bytes within the HBM budget
// left (0 = no budget).  A large head is admitted alone.  A small head is
// admitted together with every other queued small request that also fits
// once the ones before it are admitted, up to batch_max, in arrival order;
// large requests stay queued in place.  A head that does not fit blocks the
// queue (first come, first served: no small request overtakes a large head
// that waits for budget).
//
// What the budget counts: the matrices of the requests in flight (unless
// the budget is the context's, whose bytes in use already hold every
// resident matrix: then `external` bytes, what the context holds besides
// the workers' workspaces, are counted instead), plus the device workspaces
// the workers hold.  Workers keep their workspaces between
// requests (growing one means freeing and allocating, and a free waits for
// the whole device), so a worker's workspaces stay charged while it is idle;
// admitting a request charges only the growth the worker taking it needs.
// Each worker tells the queue what it really holds after every unit of work
// (settle).  An idle worker whose workspaces keep the head from fitting
// gives them back (should_shrink); a unit whose workspace allocation failed
// on the device goes back to the head of the queue (requeue) and the queue
// admits nothing until a unit in flight finishes.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <vector>

namespace dsm {

// Kinds of workspace a worker keeps: the batched solver's arena, the
// device-wide CG vectors, the SpMV scratch some formats need inside CG.
enum { WS_BATCH = 0, WS_CG = 1, WS_SPMV = 2, WS_KINDS = 3 };

// Size a workspace is allocated at when it grows: the next power of two of
// the request, at least 64 KiB, so a worker's workspaces settle after a few
// growths on a mixed stream.
inline size_t ws_round(size_t bytes) {
    size_t r = (size_t)1 << 16;
    while (r < bytes) r <<= 1;
    return r;
}

class Admission {
  public:
    struct Item {
        uint64_t id;
        size_t matrix;         // bytes of the request's matrix
        size_t ws[WS_KINDS];   // workspace it needs of each kind (small: its share of the arena)
        bool small;
    };

    // batch_fixed: arena bytes a batch needs beyond its members' shares.
    // count_matrices: charge in-flight matrices (false: the budget is the
    // context's and set_external gives the bytes it holds besides the
    // workers' workspaces).
    Admission(int slots, size_t budget, int batch_max, int workers, size_t batch_fixed = 0,
              bool count_matrices = true)
        : slots_(slots), budget_(budget), batch_max_(batch_max), batch_fixed_(batch_fixed),
          count_matrices_(count_matrices), held_(workers > 0 ? workers : 1) {}

    void set_external(size_t bytes) { external_ = bytes; }

    void push(const Item &r) { q_.push_back(r); }

    // Bytes an idle server needs to run r alone on a worker holding nothing
    // (besides the external bytes).
    size_t alone_bytes(const Item &r) const {
        size_t b = count_matrices_ ? r.matrix : 0;
        if (r.small) return b + ws_round(batch_fixed_ + r.ws[WS_BATCH]);
        for (int k = WS_CG; k < WS_KINDS; k++)
            if (r.ws[k]) b += ws_round(r.ws[k]);
        return b;
    }

    // Whether r could run on an idle server whose workers hold nothing.
    bool could_fit_alone(const Item &r) const {
        return budget_ == 0 || (count_matrices_ ? 0 : external_) + alone_bytes(r) <= budget_;
    }

    // The next unit of work for `worker`, or an empty vector when the head
    // cannot be admitted now (or nothing is queued).  *small tells which
    // path it takes.
    std::vector<Item> take(int worker, bool *small) {
        std::vector<Item> out;
        if (stalled_ || q_.empty()) return out;
        Held &h = held_[worker];
        const Item &head = q_.front();
        if (!head.small) {
            size_t cap[WS_KINDS];
            const size_t grow = growth_large(h, head, cap);
            if (!fits(1, head.matrix, grow)) return out;
            if (small) *small = false;
            charge(h, cap, grow);
            admit(q_.begin(), out);
            note_peak();
            return out;
        }
        size_t share = 0, matrix = 0;
        int count = 0;
        // members in arrival order, each kept if the batch still fits with it
        std::vector<char> pick(q_.size(), 0);
        size_t pos = 0;
        for (auto it = q_.begin(); it != q_.end() && count < batch_max_; ++it, ++pos) {
            if (!it->small) continue;
            const size_t s2 = share + it->ws[WS_BATCH], m2 = matrix + it->matrix;
            if (fits(count + 1, m2, growth_batch(h, s2))) {
                share = s2;
                matrix = m2;
                count++;
                pick[pos] = 1;
            } else if (pos == 0) {
                return out;  // the head itself does not fit
            }
        }
        if (small) *small = true;
        const size_t need = ws_round(batch_fixed_ + share);
        size_t cap[WS_KINDS] = {h.cap[WS_BATCH] >= need ? h.cap[WS_BATCH] : need, h.cap[WS_CG], h.cap[WS_SPMV]};
        charge(h, cap, growth_batch(h, share));
        size_t w = 0;
        for (size_t r = 0; r < q_.size(); r++) {
            if (r < pick.size() && pick[r]) {
                out.push_back(q_[r]);
            } else {
                if (w != r) q_[w] = q_[r];
                w++;
            }
        }
        q_.resize(w);
        in_flight_ += count;
        matrix_ += matrix;
        note_peak();
        return out;
    }

    // A finished request returns its slot and its matrix bytes.
    void release(const Item &r) {
        in_flight_--;
        matrix_ -= r.matrix;
        stalled_ = false;
    }

    // What `worker` holds now, kind by kind (after every unit of work, and
    // after it gave its workspaces back).
    void settle(int worker, const size_t cap[WS_KINDS]) {
        Held &h = held_[worker];
        for (int k = 0; k < WS_KINDS; k++) {
            held_total_ -= h.cap[k];
            h.cap[k] = cap[k];
            held_total_ += cap[k];
        }
        note_peak();
    }

    // A unit whose workspace allocation failed goes back to the head of the
    // queue, in its order, while other work is in flight (whose end may free
    // memory); then nothing is admitted until a unit in flight finishes.
    // Returns false, and keeps the unit admitted, when nothing else is in
    // flight: the caller fails it.
    bool requeue(const std::vector<Item> &items) {
        if (in_flight_ - (int)items.size() <= 0) return false;
        for (auto it = items.rbegin(); it != items.rend(); ++it) {
            in_flight_--;
            matrix_ -= it->matrix;
            q_.push_front(*it);
        }
        stalled_ = true;
        return true;
    }

    // True when the head does not fit on `worker` for lack of budget (a slot
    // is free, and no failed allocation holds the queue).
    bool head_blocked_by_budget(int worker) const {
        if (stalled_ || q_.empty() || budget_ == 0 || in_flight_ >= slots_) return false;
        const Held &h = held_[worker];
        const Item &head = q_.front();
        size_t cap[WS_KINDS];
        const size_t grow = head.small ? growth_batch(h, head.ws[WS_BATCH]) : growth_large(h, head, cap);
        return !fits(1, head.matrix, grow);
    }

    // True when `worker` holds workspace and the head does not fit on it
    // for lack of budget: giving the workspace back can only help the head in.
    bool should_shrink(int worker) const { return held_bytes(worker) > 0 && head_blocked_by_budget(worker); }

    uint64_t head_id() const { return q_.empty() ? 0 : q_.front().id; }

    // True when the head can never get in as things stand: it does not fit
    // for lack of budget, nothing is in flight (no end of a unit will free
    // anything) and no worker holds workspace to give back.  Only possible
    // when the bytes counted from outside grew after the head was submitted.
    bool head_stuck(int worker) const {
        return in_flight_ == 0 && held_total_ == 0 && head_blocked_by_budget(worker);
    }

    // Removes the head without admitting it (to fail it).
    Item pop_head() {
        Item it = q_.front();
        q_.pop_front();
        return it;
    }
    size_t peak_charged() const { return peak_; }
    bool empty() const { return q_.empty(); }
    size_t queued() const { return q_.size(); }
    int in_flight() const { return in_flight_; }
    size_t matrix_bytes_in_flight() const { return matrix_; }
    size_t held_bytes() const { return held_total_; }
    size_t held_bytes(int worker) const {
        const Held &h = held_[worker];
        return h.cap[0] + h.cap[1] + h.cap[2];
    }
    size_t charged() const { return used(); }
    size_t budget() const { return budget_; }
    bool stalled() const { return stalled_; }

  private:
    struct Held {
        size_t cap[WS_KINDS] = {0, 0, 0};
    };

    bool fits(int count, size_t matrix, size_t grow) const {
        return in_flight_ + count <= slots_ && (budget_ == 0 || used() + (count_matrices_ ? matrix : 0) + grow <= budget_);
    }

    size_t used() const { return (count_matrices_ ? matrix_ : external_) + held_total_; }

    // bytes the worker's arena grows by for a batch whose shares sum to share
    size_t growth_batch(const Held &h, size_t share) const {
        const size_t need = ws_round(batch_fixed_ + share);
        return need > h.cap[WS_BATCH] ? need - h.cap[WS_BATCH] : 0;
    }

    // bytes the worker's CG/SpMV workspaces grow by for r; cap receives the
    // capacities the worker will hold
    size_t growth_large(const Held &h, const Item &r, size_t cap[WS_KINDS]) const {
        size_t grow = 0;
        cap[WS_BATCH] = h.cap[WS_BATCH];
        for (int k = WS_CG; k < WS_KINDS; k++) {
            const size_t need = r.ws[k] ? ws_round(r.ws[k]) : 0;
            cap[k] = h.cap[k];
            if (need > h.cap[k]) {
                grow += need - h.cap[k];
                cap[k] = need;
            }
        }
        return grow;
    }

    void charge(Held &h, const size_t cap[WS_KINDS], size_t grow) {
        for (int k = 0; k < WS_KINDS; k++) h.cap[k] = cap[k];
        held_total_ += grow;
    }

    void note_peak() {
        if (used() > peak_) peak_ = used();
    }

    void admit(std::deque<Item>::iterator it, std::vector<Item> &out) {
        in_flight_++;
        matrix_ += it->matrix;
        out.push_back(*it);
        q_.erase(it);
    }

    std::deque<Item> q_;
    int slots_;
    size_t budget_;
    int batch_max_;
    size_t batch_fixed_;
    bool count_matrices_;
    size_t external_ = 0;
    std::vector<Held> held_;
    size_t held_total_ = 0;
    int in_flight_ = 0;
    size_t matrix_ = 0;
    bool stalled_ = false;
    size_t peak_ = 0;
};

}  // namespace dsm
