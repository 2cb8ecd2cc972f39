// Host test of the geometry upload cache (ss_geom_upload.hpp) with device
// operations that fail on demand: after any failed upload, a call with the
// geometry the buffer held before must upload again instead of reporting a
// cached copy, and a successful upload must leave the cache set.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ss_geom_upload.hpp"

struct FakeOps {
    int fail_dev_alloc = 0, fail_host_alloc = 0, fail_copy = 0, fail_event = 0, fail_event_sync = 0;
    int dev_allocs = 0, copies = 0, device_syncs = 0, live = 0;
    int dev_alloc(void **p, size_t bytes) {
        if (fail_dev_alloc) { --fail_dev_alloc; return 2; }
        ++dev_allocs; ++live;
        *p = std::malloc(bytes);
        return 0;
    }
    void dev_free(void *p) { --live; std::free(p); }
    int host_alloc(void **p, size_t bytes) {
        if (fail_host_alloc) { --fail_host_alloc; return 2; }
        ++live;
        *p = std::malloc(bytes);
        return 0;
    }
    void host_free(void *p) { --live; std::free(p); }
    int device_sync() { ++device_syncs; return 0; }
    int event_sync() {
        if (fail_event_sync) { --fail_event_sync; return 7; }
        return 0;
    }
    int copy_async(void *, const void *, size_t) {
        if (fail_copy) { --fail_copy; return 1; }
        ++copies;
        return 0;
    }
    int event_record() {
        if (fail_event) { --fail_event; return 3; }
        return 0;
    }
};

static int failures = 0;
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            std::printf("FAILED line %d: %s\n", __LINE__, #c);      \
            ++failures;                                             \
        }                                                           \
    } while (0)

int main() {
    using namespace ss;
    FakeOps ops;
    GeomBuffer g;
    int code = 0;
    auto fill = [](float *) {};
    std::vector<float> small(12 * 3, 1.0f), large(12 * 2000, 2.0f);
    // first upload
    CHECK(g.upload(ops, small.data(), small.size(), 1, small.size() + 8, fill, &code) == UPLOAD_OK);
    CHECK(g.holds(small.data(), small.size(), 1));
    CHECK(ops.copies == 1);
    // unchanged geometry: cached, no copy
    CHECK(g.upload(ops, small.data(), small.size(), 1, small.size() + 8, fill, &code) == UPLOAD_OK);
    CHECK(ops.copies == 1);
    // another kind: not cached
    CHECK(!g.holds(small.data(), small.size(), 0));
    // a larger geometry whose device allocation fails: error, buffers gone,
    // cache invalid; the old geometry then uploads again
    ops.fail_dev_alloc = 1;
    CHECK(g.upload(ops, large.data(), large.size(), 1, large.size() + 8, fill, &code) == UPLOAD_DEV_ALLOC);
    CHECK(code == 2);
    CHECK(g.d_geom == nullptr && g.cap == 0);
    CHECK(!g.holds(small.data(), small.size(), 1));
    CHECK(g.upload(ops, small.data(), small.size(), 1, small.size() + 8, fill, &code) == UPLOAD_OK);
    CHECK(g.d_geom != nullptr && ops.copies == 2 && g.holds(small.data(), small.size(), 1));
    // the staging allocation fails after the device allocation succeeded
    ops.fail_host_alloc = 1;
    CHECK(g.upload(ops, large.data(), large.size(), 1, large.size() + 8, fill, &code) == UPLOAD_HOST_ALLOC);
    CHECK(g.d_geom == nullptr && g.h_stage == nullptr && g.cap == 0);
    CHECK(!g.holds(small.data(), small.size(), 1));
    CHECK(g.upload(ops, small.data(), small.size(), 1, small.size() + 8, fill, &code) == UPLOAD_OK);
    CHECK(ops.copies == 3);
    // the copy fails after a successful grow: the new buffer holds nothing
    ops.fail_copy = 1;
    CHECK(g.upload(ops, large.data(), large.size(), 1, large.size() + 8, fill, &code) == UPLOAD_COPY);
    CHECK(!g.holds(large.data(), large.size(), 1) && !g.holds(small.data(), small.size(), 1));
    CHECK(g.upload(ops, small.data(), small.size(), 1, small.size() + 8, fill, &code) == UPLOAD_OK);
    CHECK(ops.copies == 4 && g.holds(small.data(), small.size(), 1));
    // the event cannot be recorded: cache invalid, device drained
    ops.fail_event = 1;
    const int syncs = ops.device_syncs;
    CHECK(g.upload(ops, large.data(), large.size(), 1, large.size() + 8, fill, &code) == UPLOAD_EVENT);
    CHECK(!g.holds(large.data(), large.size(), 1) && ops.device_syncs > syncs && !g.staged_pending);
    CHECK(g.upload(ops, large.data(), large.size(), 1, large.size() + 8, fill, &code) == UPLOAD_OK);
    CHECK(g.holds(large.data(), large.size(), 1));
    // waiting for the previous upload fails: error, cache invalid, retried next time
    ops.fail_event_sync = 1;
    CHECK(g.upload(ops, small.data(), small.size(), 1, small.size() + 8, fill, &code) == UPLOAD_SYNC);
    CHECK(code == 7 && !g.holds(large.data(), large.size(), 1) && !g.holds(small.data(), small.size(), 1));
    CHECK(g.upload(ops, small.data(), small.size(), 1, small.size() + 8, fill, &code) == UPLOAD_OK);
    CHECK(g.holds(small.data(), small.size(), 1));
    g.release(ops);
    CHECK(ops.live == 0 && !g.holds(small.data(), small.size(), 1));
    if (failures == 0) std::printf("geom upload cache: all checks passed\n");
    return failures == 0 ? 0 : 1;
}
