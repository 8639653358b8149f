// Checks of the work-list cache's eviction rule (PinnedLru): built and run
// by tests/test_cache_policy.py with the host compiler.
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <string>

#include "pinned_lru.h"

#define CHECK(c)                                                       \
    do {                                                               \
        if (!(c)) {                                                    \
            std::printf("FAILED line %d: %s\n", __LINE__, #c);        \
            std::exit(1);                                              \
        }                                                              \
    } while (0)

struct Val {
    int id;
    static int alive;
    explicit Val(int i) : id(i) { alive++; }
    ~Val() { alive--; }
};
int Val::alive = 0;

int main() {
    {
        rot::PinnedLru<std::string, Val> c(2);
        Val* a = c.insert("a", std::make_unique<Val>(1));
        Val* b = c.insert("b", std::make_unique<Val>(2));
        CHECK(c.size() == 2 && Val::alive == 2);
        CHECK(c.find("a") == a);  // a becomes the most recent
        c.insert("c", std::make_unique<Val>(3));
        CHECK(c.size() == 2);
        CHECK(c.find("b") == nullptr);  // least recent unpinned entry evicted
        CHECK(c.find("a") == a && Val::alive == 2);
        // find_if: the first match, most recent first, made the most recent
        Val* cc = c.find_if([](const std::string& k) { return k == "c"; });
        CHECK(cc != nullptr && cc->id == 3);
        CHECK(c.find_if([](const std::string& k) { return k == "b"; }) == nullptr);
        c.insert("d", std::make_unique<Val>(4));  // evicts a (c was used last)
        CHECK(c.find("a") == nullptr && c.find("c") == cc && c.size() == 2);
        (void)b;
    }
    CHECK(Val::alive == 0);  // the cache owns and frees its values
    {
        // pinned entries are never evicted and do not count against capacity
        rot::PinnedLru<int, Val> c(2);
        Val* p1 = c.insert(1, std::make_unique<Val>(1));
        c.pin(p1);
        Val* p2 = c.insert(2, std::make_unique<Val>(2));
        c.pin(p2);
        for (int k = 3; k < 20; k++) c.insert(k, std::make_unique<Val>(k));
        CHECK(c.find(1) == p1 && c.find(2) == p2);
        CHECK(c.pinned(p1) && c.pinned(p2));
        CHECK(c.size() == 4);  // two pinned + the two most recent unpinned
        CHECK(c.find(19) != nullptr && c.find(18) != nullptr && c.find(17) == nullptr);
        CHECK(Val::alive == 4);
    }
    CHECK(Val::alive == 0);
    {
        // the entry just inserted is never the one evicted, even at capacity 0
        rot::PinnedLru<int, Val> c(0);
        Val* v = c.insert(7, std::make_unique<Val>(7));
        CHECK(c.find(7) == v && c.size() == 1);
        Val* w = c.insert(8, std::make_unique<Val>(8));
        CHECK(c.find(8) == w && c.find(7) == nullptr && c.size() == 1);
        // pinning a recently used entry after others were inserted keeps it
        rot::PinnedLru<int, Val> d(1);
        Val* x = d.insert(1, std::make_unique<Val>(1));
        d.pin(x);
        d.insert(2, std::make_unique<Val>(2));
        d.insert(3, std::make_unique<Val>(3));
        CHECK(d.find(1) == x && d.find(2) == nullptr && d.find(3) != nullptr);
    }
    CHECK(Val::alive == 0);
    std::printf("ok\n");
    return 0;
}
