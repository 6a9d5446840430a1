// keymap.hpp -- hash map from packed block keys (sim, level, ix, iy, iz in 62
// bits) to int values for the host tree code: one flat table with linear
// probing (the keys hashed with the 64-bit finaliser of MurmurHash3), at most
// half full, no single-key deletion (a map is cleared whole), and the keys
// kept in insertion order for iteration.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace mapk {

class KeyMap {
  public:
    explicit KeyMap(size_t expected = 0) { reserve(expected); }

    void reserve(size_t n)
    {
        size_t cap = 16;
        while (cap < 2 * n)
            cap <<= 1;
        if (cap > tab_.size())
            rehash(cap);
    }

    // k -> v unless k is present; whether it was inserted
    bool insert(uint64_t k, int v)
    {
        if (2 * (keys_.size() + 1) > tab_.size())
            rehash(tab_.empty() ? 16 : 2 * tab_.size());
        Ent &e = tab_[probe(k)];
        if (e.key == k)
            return false;
        e = Ent{k, v};
        keys_.push_back(k);
        return true;
    }

    // k -> v, replacing a present value
    void set(uint64_t k, int v)
    {
        if (!insert(k, v))
            tab_[probe(k)].val = v;
    }

    // the value of k, or -1 when absent
    int find(uint64_t k) const
    {
        if (tab_.empty())
            return -1;
        const Ent &e = tab_[probe(k)];
        return e.key == k ? e.val : -1;
    }

    bool contains(uint64_t k) const { return !tab_.empty() && tab_[probe(k)].key == k; }

    void clear()
    {
        std::fill(tab_.begin(), tab_.end(), Ent{});
        keys_.clear();
    }

    size_t size() const { return keys_.size(); }
    const std::vector<uint64_t> &keys() const { return keys_; }

  private:
    static constexpr uint64_t EMPTY = ~0ull;  // no packed key has all 64 bits set
    struct Ent {
        uint64_t key = EMPTY;
        int val = -1;
    };
    std::vector<Ent> tab_;
    std::vector<uint64_t> keys_;

    static uint64_t mix(uint64_t k)
    {
        k ^= k >> 33;
        k *= 0xff51afd7ed558ccdull;
        k ^= k >> 33;
        k *= 0xc4ceb9fe1a85ec53ull;
        k ^= k >> 33;
        return k;
    }

    // the slot holding k, or the empty slot where it would go
    size_t probe(uint64_t k) const
    {
        const size_t m = tab_.size() - 1;
        size_t i = mix(k) & m;
        while (tab_[i].key != EMPTY && tab_[i].key != k)
            i = (i + 1) & m;
        return i;
    }

    void rehash(size_t cap)
    {
        std::vector<Ent> old;
        old.swap(tab_);
        tab_.assign(cap, Ent{});
        for (const Ent &e : old)
            if (e.key != EMPTY)
                tab_[probe(e.key)] = e;
    }
};

}  // namespace mapk
