// Host-side batch schedule: greedy first-fit colouring of scan positions
// into batches of pairwise disjoint windows, and the per-sweep shuffle.
#pragma once

#include <stdint.h>

#include <string>
#include <unordered_map>
#include <vector>

namespace ptyc {

// Two n x n windows with top-left corners a and b share a pixel.
inline bool overlap(int32_t ay, int32_t ax, int32_t by, int32_t bx, int32_t n) {
    const int32_t dy = ay > by ? ay - by : by - ay;
    const int32_t dx = ax > bx ? ax - bx : bx - ax;
    return dy < n && dx < n;
}

// Incremental colouring in index order: adding positions never changes the
// colour of an earlier one.  A spatial hash with n x n cells limits the
// overlap search to the 3 x 3 neighbouring cells.
class Colouring {
public:
    Colouring(int32_t n, int32_t max_batch) : n_(n), cap_(max_batch) {}
    // pos_yx holds all positions so far (2 int32 each); colours first..first+count-1
    void extend(const int32_t* pos_yx, int64_t first, int64_t count);
    const std::vector<int32_t>& colour() const { return colour_; }
    const std::vector<std::vector<int64_t>>& members() const { return members_; }
    int64_t size() const { return (int64_t)colour_.size(); }

private:
    int32_t n_, cap_;
    std::vector<int32_t> colour_;
    std::vector<std::vector<int64_t>> members_;
    std::unordered_map<int64_t, std::vector<int64_t>> cells_;
    std::vector<uint32_t> mark_;   // mark_[c] == stamp: colour c is blocked
    uint32_t stamp_ = 0;
};

// SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) and unbiased bounded integers by Lemire's
// multiply-and-reject method ("Fast random integer generation in an
// interval", ACM TOMACS 2019).
class SplitMix64 {
public:
    explicit SplitMix64(uint64_t seed) : s_(seed) {}
    uint64_t next() {
        uint64_t z = (s_ += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    uint64_t below(uint64_t m);  // uniform on [0, m), m >= 1
private:
    uint64_t s_;
};

// Fisher-Yates permutation of 0..n-1 from (seed, sweep).
std::vector<int64_t> shuffled(int64_t n, uint64_t seed, uint64_t sweep);

// Validate an explicit batch schedule; on failure returns false and a message.
bool check_batches(int64_t count, const int32_t* pos_yx, int32_t n, const int64_t* order,
                   int64_t order_len, const int64_t* off, int64_t n_batches, std::string* why);

}  // namespace ptyc
