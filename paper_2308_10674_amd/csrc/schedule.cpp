#include "schedule.h"

#include <algorithm>

namespace ptyc {

static inline int64_t cell_key(int64_t cy, int64_t cx) { return (cy << 32) ^ (cx & 0xffffffffll); }

void Colouring::extend(const int32_t* pos_yx, int64_t first, int64_t count) {
    colour_.resize((size_t)(first + count), -1);
    for (int64_t j = first; j < first + count; ++j) {
        const int32_t y = pos_yx[2 * j], x = pos_yx[2 * j + 1];
        const int64_t cy = y / n_, cx = x / n_;
        ++stamp_;
        if (stamp_ == 0) {  // wrapped: clear the marks
            std::fill(mark_.begin(), mark_.end(), 0u);
            stamp_ = 1;
        }
        for (int64_t dy = -1; dy <= 1; ++dy)
            for (int64_t dx = -1; dx <= 1; ++dx) {
                auto it = cells_.find(cell_key(cy + dy, cx + dx));
                if (it == cells_.end()) continue;
                for (int64_t i : it->second)
                    if (overlap(y, x, pos_yx[2 * i], pos_yx[2 * i + 1], n_))
                        mark_[(size_t)colour_[(size_t)i]] = stamp_;
            }
        int32_t c = 0;
        const int32_t nc = (int32_t)members_.size();
        while (c < nc && (mark_[(size_t)c] == stamp_ || (int32_t)members_[(size_t)c].size() >= cap_)) ++c;
        if (c == nc) {
            members_.emplace_back();
            mark_.push_back(0u);
        }
        colour_[(size_t)j] = c;
        members_[(size_t)c].push_back(j);
        cells_[cell_key(cy, cx)].push_back(j);
    }
}

uint64_t SplitMix64::below(uint64_t m) {
    unsigned __int128 p = (unsigned __int128)next() * m;
    uint64_t lo = (uint64_t)p;
    if (lo < m) {
        const uint64_t thresh = (0 - m) % m;
        while (lo < thresh) {
            p = (unsigned __int128)next() * m;
            lo = (uint64_t)p;
        }
    }
    return (uint64_t)(p >> 64);
}

std::vector<int64_t> shuffled(int64_t n, uint64_t seed, uint64_t sweep) {
    std::vector<int64_t> v((size_t)n);
    for (int64_t i = 0; i < n; ++i) v[(size_t)i] = i;
    SplitMix64 g(seed ^ (0xD1B54A32D192ED03ull * (sweep + 1)));
    for (int64_t i = n - 1; i > 0; --i) {
        const int64_t k = (int64_t)g.below((uint64_t)i + 1);
        std::swap(v[(size_t)i], v[(size_t)k]);
    }
    return v;
}

bool check_batches(int64_t count, const int32_t* pos_yx, int32_t n, const int64_t* order,
                   int64_t order_len, const int64_t* off, int64_t n_batches, std::string* why) {
    if (n_batches < 0 || off[0] != 0 || off[n_batches] != order_len) {
        *why = "batch offsets must start at 0 and end at order_len";
        return false;
    }
    for (int64_t b = 0; b < n_batches; ++b)
        if (off[b + 1] < off[b]) {
            *why = "batch offsets must be non-decreasing";
            return false;
        }
    for (int64_t i = 0; i < order_len; ++i)
        if (order[i] < 0 || order[i] >= count) {
            *why = "order index " + std::to_string(order[i]) + " is not a loaded position";
            return false;
        }
    for (int64_t b = 0; b < n_batches; ++b)
        for (int64_t u = off[b]; u < off[b + 1]; ++u)
            for (int64_t v = u + 1; v < off[b + 1]; ++v) {
                const int64_t p = order[u], q = order[v];
                if (overlap(pos_yx[2 * p], pos_yx[2 * p + 1], pos_yx[2 * q], pos_yx[2 * q + 1], n)) {
                    *why = "batch " + std::to_string(b) + ": windows of positions " + std::to_string(p) +
                           " and " + std::to_string(q) + " overlap";
                    return false;
                }
            }
    return true;
}

}  // namespace ptyc
