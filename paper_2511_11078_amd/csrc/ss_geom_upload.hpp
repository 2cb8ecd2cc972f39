// ss_geom_upload.hpp -- a context's device copy of the acquisition geometry
// and the cache that skips re-uploading an unchanged geometry.
//
// The logic is written against a small set of device operations (`Ops`) so
// that it compiles without HIP: the library instantiates it with HIP calls
// (ss_abi.cpp), the host tests with operations that fail on demand.  Ops
// provides, each returning 0 on success and a non-zero error code otherwise:
//
//   int dev_alloc(void **p, size_t bytes);   void dev_free(void *p);
//   int host_alloc(void **p, size_t bytes);  void host_free(void *p);
//   int device_sync();    // all enqueued work done (old buffers unused)
//   int event_sync();     // the last upload's read of the staging buffer done
//   int copy_async(void *dst, const void *src, size_t bytes);  // host -> device
//   int event_record();   // marks the end of that copy on the caller's stream
#pragma once

#include <cstddef>
#include <cstring>
#include <vector>

namespace ss {

enum UploadError {
    UPLOAD_OK = 0,
    UPLOAD_SYNC,        // device_sync or event_sync failed
    UPLOAD_DEV_ALLOC,   // device buffer allocation failed
    UPLOAD_HOST_ALLOC,  // pinned staging allocation failed
    UPLOAD_COPY,        // the asynchronous copy could not be enqueued
    UPLOAD_EVENT        // the completion event could not be recorded
};

struct GeomBuffer {
    float *d_geom = nullptr;       // device: view vectors, then per-view records
    float *h_stage = nullptr;      // pinned staging of the same size
    size_t cap = 0;                // floats of each buffer
    bool staged_pending = false;   // an upload may still read h_stage
    std::vector<float> last_vecs;  // the view vectors d_geom holds ...
    int last_kind = -1;            // ... and their geometry kind
    bool cached = false;           // ... valid only while this is set

    // Does d_geom hold exactly these view vectors?
    bool holds(const float *vecs, size_t nf, int kind) const {
        return cached && d_geom != nullptr && last_kind == kind && last_vecs.size() == nf &&
               std::memcmp(last_vecs.data(), vecs, nf * sizeof(float)) == 0;
    }

    // Make d_geom hold `total` floats: the nf floats of `vecs` followed by
    // what fill(h_stage) writes behind them.  Nothing happens when it already
    // holds these vectors.  The cache is invalidated before anything is
    // freed, grown or overwritten and set again only once the copy and its
    // event have been enqueued, so after any failure the next call uploads
    // again.  On failure `*code` receives the operation's error code.
    template <class Ops, class Fill>
    UploadError upload(Ops &ops, const float *vecs, size_t nf, int kind, size_t total, Fill fill, int *code) {
        if (holds(vecs, nf, kind)) return UPLOAD_OK;
        cached = false;
        int e;
        if (total > cap) {
            if (d_geom || h_stage) {
                // the old buffers may still be read by enqueued work
                if ((e = ops.device_sync()) != 0) { *code = e; return UPLOAD_SYNC; }
                release(ops);
            }
            const size_t want = total < 4096 ? 4096 : total;
            void *p = nullptr;
            if ((e = ops.dev_alloc(&p, want * sizeof(float))) != 0) { *code = e; return UPLOAD_DEV_ALLOC; }
            d_geom = static_cast<float *>(p);
            p = nullptr;
            if ((e = ops.host_alloc(&p, want * sizeof(float))) != 0) {
                ops.dev_free(d_geom);
                d_geom = nullptr;
                *code = e;
                return UPLOAD_HOST_ALLOC;
            }
            h_stage = static_cast<float *>(p);
            cap = want;
        }
        if (staged_pending) {
            if ((e = ops.event_sync()) != 0) { *code = e; return UPLOAD_SYNC; }
            staged_pending = false;
        }
        std::memcpy(h_stage, vecs, nf * sizeof(float));
        fill(h_stage);
        if ((e = ops.copy_async(d_geom, h_stage, total * sizeof(float))) != 0) { *code = e; return UPLOAD_COPY; }
        // the copy is enqueued and reads h_stage: from here on wait for it
        // before the staging buffer is written again
        staged_pending = true;
        if ((e = ops.event_record()) != 0) {
            // no event marks the copy's end: the next upload waits for the device
            staged_pending = false;
            (void)ops.device_sync();
            *code = e;
            return UPLOAD_EVENT;
        }
        last_vecs.assign(vecs, vecs + nf);
        last_kind = kind;
        cached = true;
        return UPLOAD_OK;
    }

    template <class Ops>
    void release(Ops &ops) {
        cached = false;
        if (d_geom) ops.dev_free(d_geom);
        if (h_stage) ops.host_free(h_stage);
        d_geom = nullptr;
        h_stage = nullptr;
        cap = 0;
        staged_pending = false;
    }
};

}  // namespace ss
