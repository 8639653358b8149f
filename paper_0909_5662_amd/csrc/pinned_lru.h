// Least-recently-used cache whose entries can be pinned.  Used for cached
// work-lists that hold device memory: an entry used while a stream was being
// captured into a graph is pinned, because the graph keeps the entry's device
// pointers and may be replayed at any later time; pinned entries are never
// evicted.  At most `capacity` unpinned entries are kept: inserting beyond
// that evicts the least recently used unpinned entry.
//
// Host-only C++ (no HIP types), so the rule is testable on its own.  Not
// thread-safe: the owner holds a lock around every call.
#pragma once

#include <cstddef>
#include <list>
#include <memory>
#include <utility>

namespace rot {

template <class Key, class Value>
class PinnedLru {
   public:
    explicit PinnedLru(size_t capacity) : capacity_(capacity) {}

    // The entry for `key`, made the most recent; nullptr when absent.
    Value* find(const Key& key) {
        for (auto it = entries_.begin(); it != entries_.end(); ++it)
            if (it->key == key) {
                entries_.splice(entries_.begin(), entries_, it);
                return entries_.front().value.get();
            }
        return nullptr;
    }

    // The first entry (most recent first) whose key satisfies `pred`, made
    // the most recent; nullptr when none does.
    template <class Pred>
    Value* find_if(Pred pred) {
        for (auto it = entries_.begin(); it != entries_.end(); ++it)
            if (pred(it->key)) {
                entries_.splice(entries_.begin(), entries_, it);
                return entries_.front().value.get();
            }
        return nullptr;
    }

    // Insert as the most recent entry, then evict least recently used
    // unpinned entries until at most `capacity` unpinned ones remain.
    // Returns the stored value.
    Value* insert(Key key, std::unique_ptr<Value> value) {
        entries_.push_front(Entry{std::move(key), std::move(value), false});
        Value* v = entries_.front().value.get();
        size_t unpinned = 0;
        for (const Entry& e : entries_) unpinned += e.pinned ? 0 : 1;
        for (auto it = entries_.end(); unpinned > capacity_ && it != entries_.begin();) {
            --it;
            if (!it->pinned && it->value.get() != v) {
                it = entries_.erase(it);
                unpinned--;
            }
        }
        return v;
    }

    // Keep the entry holding `value` until the cache is destroyed.
    void pin(const Value* value) {
        for (Entry& e : entries_)
            if (e.value.get() == value) e.pinned = true;
    }

    bool pinned(const Value* value) const {
        for (const Entry& e : entries_)
            if (e.value.get() == value) return e.pinned;
        return false;
    }

    size_t size() const { return entries_.size(); }

   private:
    struct Entry {
        Key key;
        std::unique_ptr<Value> value;
        bool pinned;
    };
    size_t capacity_;
    std::list<Entry> entries_;  // most recent first
};

}  // namespace rot
