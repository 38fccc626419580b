// A CPU model of the cell-queue protocol that the solve kernel without rounds runs on the GPU
// (EIK_SCHED_ASYNC): T worker threads stand in for the waves, a G x G grid of cells for the
// cells of a grid.  It reproduces the protocol's words one for one -- a per-cell word with the
// QUEUED and RUNNING bits and the tag bits, a ring of cell ids with fetch-and-add tickets on
// its head and tail and -1 for an empty position, a count of cells queued or being visited
// (decremented after a visit's own pushes) and a done word.  As on the GPU, the ring, its
// counters and the done word are relaxed atomics; only the cell word's read-modify-writes
// order memory (acquire/release), where the GPU waits for its coherent accesses.  Built with
// -fsanitize=thread, so a visit that is not ordered after the previous visit of its cell (a
// data race on the cell's own state) is reported.  It checks, for several tag patterns:
//   * no two workers visit one cell at once;
//   * no tag is lost: the last visit of every cell starts after the last tag it received;
//   * the loop ends only when nothing is queued or running, and every cell has done its work.
// Exit status 0 and a line "protocol model: ... 0 violations" on success.  Two planted mistakes
// (compile-time switches, for the tests of the model itself): PLANT_RELAXED takes the cell
// word's read-modify-writes without ordering (ThreadSanitizer must report a race on the cell's
// state), PLANT_LOST_TAG clears QUEUED again when a tag finds its cell running (the owner then
// does not re-queue it: a tag is lost).
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <thread>
#include <vector>

namespace {

#ifdef PLANT_RELAXED
constexpr std::memory_order kOwn = std::memory_order_relaxed;
#else
constexpr std::memory_order kOwn = std::memory_order_acq_rel;
#endif

constexpr uint32_t kQueued = 1u << 7;
constexpr uint32_t kRunning = 1u << 20;
constexpr uint32_t kAll = 1u << 6;

struct Model {
    int G, C, T;
    uint64_t cap;
    std::vector<std::atomic<uint32_t>> word;    // per cell: QUEUED / RUNNING / tag bits
    std::vector<std::atomic<int32_t>> ring;     // cell ids, -1 = empty
    std::atomic<uint64_t> head{0}, tail{0}, pending{0};
    std::atomic<int> done{0};
    // The cell's own state: written by the worker that owns the cell only (plain accesses).
    std::vector<int> interior, remaining, seen_tags, visits;
    // Published data that neighbours read while it may be rewritten (relaxed, as on the GPU).
    std::vector<std::atomic<int>> face;
    std::vector<std::atomic<int>> tags;         // tags received per cell
    std::vector<std::atomic<int>> visitors;     // workers inside a visit of the cell
    std::atomic<int> violations{0};
    uint64_t seed;

    Model(int g, int t, uint64_t s)
        : G(g), C(g * g), T(t), cap(2 * (uint64_t)g * g + 2 * (uint64_t)t + 64), word(C),
          ring(cap), interior(C, 0), remaining(C, 0), seen_tags(C, 0), visits(C, 0), face(C),
          tags(C), visitors(C), seed(s) {
        for (auto& r : ring) r.store(-1, std::memory_order_relaxed);
        for (int c = 0; c < C; ++c) {
            word[c].store(kAll | kQueued, std::memory_order_relaxed);
            ring[c].store(c, std::memory_order_relaxed);
            remaining[c] = 1 + (int)((c * 2654435761u + seed) % 5u);
            face[c].store(0, std::memory_order_relaxed);
            tags[c].store(1, std::memory_order_relaxed);  // the initial queueing
            visitors[c].store(0, std::memory_order_relaxed);
        }
        tail.store((uint64_t)C);
        pending.store((uint64_t)C);
    }

    uint64_t mix(uint64_t z) const {
        z += 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }

    void push(int c) {
        pending.fetch_add(1, std::memory_order_relaxed);  // before the cell can be popped
        const uint64_t pos = tail.fetch_add(1, std::memory_order_relaxed);
        std::atomic<int32_t>& slot = ring[pos % cap];
        while (slot.load(std::memory_order_relaxed) != -1) std::this_thread::yield();
        slot.store(c, std::memory_order_relaxed);
    }

    // Tag: the tag count, then the bits with QUEUED; whoever turns QUEUED on for a cell that is
    // not running pushes it (a running cell is pushed again by its owner).
    void tag(int c, uint32_t bits) {
        tags[c].fetch_add(1, std::memory_order_relaxed);
        const uint32_t old = word[c].fetch_or(bits | kQueued, kOwn);
#ifdef PLANT_LOST_TAG
        if ((old & kRunning) && !(old & kQueued)) word[c].fetch_and(~kQueued, kOwn);
#endif
        if (!(old & (kQueued | kRunning))) push(c);
    }

    int pop() {
        const uint64_t t = head.fetch_add(1, std::memory_order_relaxed);
        std::atomic<int32_t>& slot = ring[t % cap];
        for (;;) {
            const int v = slot.load(std::memory_order_relaxed);
            if (v >= 0) {
                slot.store(-1, std::memory_order_relaxed);
                return v;
            }
            if (done.load(std::memory_order_relaxed)) return -1;
            std::this_thread::yield();
        }
    }

    void visit(int c) {
        if (visitors[c].fetch_add(1, std::memory_order_relaxed) != 0) violations.fetch_add(1);
        seen_tags[c] = tags[c].load(std::memory_order_relaxed);
        ++interior[c];
        ++visits[c];
        int inflow = 0;
        const int x = c % G, y = c / G;
        const int nb[4] = {x > 0 ? c - 1 : -1, x + 1 < G ? c + 1 : -1, y > 0 ? c - G : -1,
                           y + 1 < G ? c + G : -1};
        for (int k = 0; k < 4; ++k)
            if (nb[k] >= 0) inflow += face[nb[k]].load(std::memory_order_relaxed);
        if (remaining[c] > 0) {
            --remaining[c];
            face[c].store(inflow + interior[c], std::memory_order_relaxed);
            const uint64_t r = mix(seed ^ ((uint64_t)c << 20) ^ (uint64_t)visits[c]);
            for (int k = 0; k < 4; ++k)
                if (nb[k] >= 0 && ((r >> k) & 1u)) tag(nb[k], 1u << k);
            if (remaining[c] > 0) tag(c, kAll);  // more work: re-queue itself
        }
        visitors[c].fetch_sub(1, std::memory_order_relaxed);
    }

    void worker() {
        for (;;) {
            const int c = pop();
            if (c < 0) return;
            const uint32_t old = word[c].exchange(kRunning, kOwn);
            if (!(old & kQueued) || (old & kRunning)) violations.fetch_add(1);
            visit(c);
            const uint32_t prev = word[c].fetch_and(~kRunning, kOwn);
            if (prev & kQueued) push(c);
            if (pending.fetch_sub(1, std::memory_order_relaxed) == 1)
                done.store(1, std::memory_order_relaxed);
        }
    }

    int run() {
        std::vector<std::thread> th;
        for (int t = 0; t < T; ++t) th.emplace_back([this] { worker(); });
        for (auto& t : th) t.join();
        int bad = violations.load();
        for (int c = 0; c < C; ++c) {
            if (word[c].load() != 0) ++bad;                   // left queued or running
            if (remaining[c] != 0) ++bad;                     // work not done
            if (seen_tags[c] != tags[c].load()) ++bad;        // a tag arrived after the last visit
            if (interior[c] != visits[c]) ++bad;
        }
        if (pending.load() != 0) ++bad;
        return bad;
    }
};

}  // namespace

int main() {
    int total_bad = 0;
    long total_visits = 0;
    int runs = 0;
    for (uint64_t seed = 1; seed <= 6; ++seed) {
        for (int threads : {2, 4, 8}) {
            Model m(12, threads, seed * 7919u);
            const int bad = m.run();
            for (int v : m.visits) total_visits += v;
            total_bad += bad;
            ++runs;
            if (bad) std::printf("seed %llu threads %d: %d violations\n",
                                 (unsigned long long)seed, threads, bad);
        }
    }
    std::printf("protocol model: %d runs, %ld visits, %d violations\n", runs, total_visits,
                total_bad);
    return total_bad == 0 ? 0 : 1;
}
