// Table-2 egress (vx_egress_* in include/vx.h): finished Tables 2 stream from
// HBM through pinned host staging buffers into flat plot files while the
// device goes on computing.  One writer thread per egress does everything
// that blocks -- waiting for a plot, reading its count, waiting for each
// piece's copy, write(2) -- so the caller's thread only enqueues.  Copies run
// on the egress's own stream (the DMA engines), so they overlap the caller's
// kernels; with `slots` staging buffers, the copy of piece i + slots is in
// flight while piece i is written.
#include <hip/hip_runtime.h>
#include <errno.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
#include <unistd.h>

#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "errors.h"
#include "vx.h"

namespace {

constexpr uint32_t kHeaderBytes = 128;
constexpr uint32_t kRecordBytes = 16;
static_assert(sizeof(vx_t2_record) == kRecordBytes, "Table-2 record layout");

struct Job {
    uint64_t id = 0;
    hipEvent_t ready = nullptr;  // the plot's work is done once this completes
    const vx_t2_record *t2 = nullptr;
    uint64_t cap = 0;
    const uint64_t *count = nullptr;
    uint32_t k = 0;
    uint64_t T = 0;
    uint8_t key[32] = {};
    uint32_t chunk_bits = 0, chunk = 0;
};

void put32(uint8_t *p, uint32_t v) {
    for (int i = 0; i < 4; ++i) p[i] = (uint8_t)(v >> (8 * i));
}

void put64(uint8_t *p, uint64_t v) {
    for (int i = 0; i < 8; ++i) p[i] = (uint8_t)(v >> (8 * i));
}

}  // namespace

struct vx_egress {
    int fd = -1;
    int device = 0;
    size_t slot_bytes = 0;
    uint32_t nslots = 0;
    std::vector<void *> ring;   // pinned staging buffers
    std::vector<hipEvent_t> ev;  // copy into ring[i] done
    uint64_t *count_host = nullptr;  // pinned
    hipStream_t copy = nullptr;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_job, cv_done;
    std::deque<Job> queue;
    uint64_t submitted = 0, done = 0;
    bool stop = false;
    vx_status err = VX_OK;
    char errmsg[256] = "";
    uint64_t bytes = 0;  // guarded by mu

    vx_status write_all(const void *p, size_t n, char *msg, size_t msglen) {
        if (fd >= 0) {
            const char *c = static_cast<const char *>(p);
            size_t left = n;
            while (left) {
                const ssize_t w = ::write(fd, c, left);
                if (w < 0) {
                    if (errno == EINTR) continue;
                    snprintf(msg, msglen, "plot file write: %s", strerror(errno));
                    return VX_ERR_IO;
                }
                c += w;
                left -= (size_t)w;
            }
        }
        std::lock_guard<std::mutex> g(mu);
        bytes += n;
        return VX_OK;
    }

    // Copy and write one plot file; returns the first error.
    vx_status run(const Job &j, char *msg, size_t msglen) {
#define EG_HIP(call, what)                                                              \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            snprintf(msg, msglen, "egress %s: %s", what, hipGetErrorString(e_));         \
            return VX_ERR_DEVICE;                                                       \
        }                                                                               \
    } while (0)
        EG_HIP(hipEventSynchronize(j.ready), "wait for the plot");
        EG_HIP(hipMemcpyAsync(count_host, j.count, sizeof(uint64_t), hipMemcpyDeviceToHost, copy), "count copy");
        EG_HIP(hipStreamSynchronize(copy), "count copy");
        const uint64_t cnt = *count_host;
        const uint64_t nrec = cnt < j.cap ? cnt : j.cap;
        uint8_t hdr[kHeaderBytes];
        memset(hdr, 0, sizeof(hdr));
        memcpy(hdr, "VXPLOT01", 8);
        put32(hdr + 8, kHeaderBytes);
        put32(hdr + 12, kRecordBytes);
        put32(hdr + 16, j.k);
        put32(hdr + 20, VX_BUCKET_BITS);
        put64(hdr + 24, j.T);
        put64(hdr + 32, cnt);
        put64(hdr + 40, nrec);
        memcpy(hdr + 48, j.key, 32);
        put32(hdr + 80, j.chunk_bits);
        put32(hdr + 84, j.chunk);
        vx_status st = write_all(hdr, sizeof(hdr), msg, msglen);
        if (st != VX_OK) return st;
        const uint64_t total = nrec * kRecordBytes;
        const uint64_t pieces = (total + slot_bytes - 1) / slot_bytes;
        const char *src = reinterpret_cast<const char *>(j.t2);
        auto issue = [&](uint64_t p) -> vx_status {
            const uint32_t s = (uint32_t)(p % nslots);
            const uint64_t off = p * slot_bytes;
            const uint64_t len = total - off < slot_bytes ? total - off : slot_bytes;
            EG_HIP(hipMemcpyAsync(ring[s], src + off, len, hipMemcpyDeviceToHost, copy), "record copy");
            EG_HIP(hipEventRecord(ev[s], copy), "record copy event");
            return VX_OK;
        };
        for (uint64_t p = 0; p < pieces && p < nslots; ++p)
            if ((st = issue(p)) != VX_OK) return st;
        for (uint64_t p = 0; p < pieces; ++p) {
            const uint32_t s = (uint32_t)(p % nslots);
            EG_HIP(hipEventSynchronize(ev[s]), "record copy wait");
            const uint64_t off = p * slot_bytes;
            const uint64_t len = total - off < slot_bytes ? total - off : slot_bytes;
            if ((st = write_all(ring[s], (size_t)len, msg, msglen)) != VX_OK) {
                EG_HIP(hipStreamSynchronize(copy), "drain");
                return st;
            }
            if (p + nslots < pieces && (st = issue(p + nslots)) != VX_OK) return st;
        }
        return VX_OK;
#undef EG_HIP
    }

    void loop() {
        (void)hipSetDevice(device);
        for (;;) {
            Job j;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_job.wait(lk, [&] { return stop || !queue.empty(); });
                if (queue.empty()) return;  // stop requested, nothing left
                j = queue.front();
                queue.pop_front();
            }
            char msg[256] = "";
            const vx_status st = run(j, msg, sizeof(msg));
            (void)hipEventDestroy(j.ready);
            {
                std::lock_guard<std::mutex> g(mu);
                if (st != VX_OK && err == VX_OK) {
                    err = st;
                    snprintf(errmsg, sizeof(errmsg), "%s", msg);
                }
                done = j.id;
            }
            cv_done.notify_all();
        }
    }
};

namespace {

vx_status fail(vx_status st, const char *msg) {
    vxs::set_error(msg);
    return st;
}

vx_status fail_hip(hipError_t e, const char *where) {
    char buf[256];
    snprintf(buf, sizeof(buf), "%s: %s", where, hipGetErrorString(e));
    vxs::set_error(buf);
    return VX_ERR_DEVICE;
}

void release(vx_egress *e) {
    for (void *p : e->ring)
        if (p) (void)hipHostFree(p);
    for (hipEvent_t x : e->ev)
        if (x) (void)hipEventDestroy(x);
    if (e->count_host) (void)hipHostFree(e->count_host);
    if (e->copy) (void)hipStreamDestroy(e->copy);
    delete e;
}

}  // namespace

extern "C" {

vx_status vx_egress_create(int fd, size_t slot_bytes, uint32_t slots, vx_egress **out) {
    if (!out) return fail(VX_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (slot_bytes < (1u << 20) || slot_bytes > (1ull << 30) || slot_bytes % kRecordBytes)
        return fail(VX_ERR_INVALID_ARG, "slot_bytes must be a multiple of 16 in [1 MiB, 1 GiB]");
    if (slots < 2 || slots > 64) return fail(VX_ERR_INVALID_ARG, "slots must be in [2, 64]");
    vx_egress *e = new vx_egress;
    e->fd = fd;
    e->slot_bytes = slot_bytes;
    e->nslots = slots;
    hipError_t h = hipGetDevice(&e->device);
    if (h == hipSuccess) h = hipStreamCreateWithFlags(&e->copy, hipStreamNonBlocking);
    if (h == hipSuccess) h = hipHostMalloc((void **)&e->count_host, sizeof(uint64_t), hipHostMallocDefault);
    e->ring.assign(slots, nullptr);
    e->ev.assign(slots, nullptr);
    for (uint32_t i = 0; h == hipSuccess && i < slots; ++i) {
        h = hipHostMalloc(&e->ring[i], slot_bytes, hipHostMallocDefault);
        if (h == hipSuccess) h = hipEventCreateWithFlags(&e->ev[i], hipEventDisableTiming);
    }
    if (h != hipSuccess) {
        release(e);
        return fail_hip(h, "vx_egress_create");
    }
    e->worker = std::thread([e] { e->loop(); });
    *out = e;
    return VX_OK;
}

vx_status vx_egress_submit(vx_egress *e, const vx_plot_params *params, const vx_t2_record *d_t2,
                           uint64_t t2_capacity, const uint64_t *d_t2_count, void *stream,
                           uint64_t *job) {
    return vx_egress_submit_chunk(e, params, 0, 0, d_t2, t2_capacity, d_t2_count, stream, job);
}

vx_status vx_egress_submit_chunk(vx_egress *e, const vx_plot_params *params, uint32_t chunk_bits, uint32_t chunk,
                                 const vx_t2_record *d_t2, uint64_t t2_capacity, const uint64_t *d_t2_count,
                                 void *stream, uint64_t *job) {
    if (!e || !params || !d_t2_count || (t2_capacity && !d_t2))
        return fail(VX_ERR_INVALID_ARG, "NULL egress, params or buffer");
    if (chunk_bits > 8 || chunk >= (1u << chunk_bits))
        return fail(VX_ERR_INVALID_ARG, "chunk_bits must be at most 8 and chunk below 2^chunk_bits");
    if (params->k < 1 || params->k > 32) return fail(VX_ERR_INVALID_ARG, "k must be in [1, 32]");
    if (((uintptr_t)d_t2 % 16) || ((uintptr_t)d_t2_count % 8)) return fail(VX_ERR_INVALID_ARG, "misaligned buffer");
    Job j;
    j.t2 = d_t2;
    j.cap = t2_capacity;
    j.count = d_t2_count;
    j.k = params->k;
    j.T = params->match_threshold;
    memcpy(j.key, params->key, 32);
    j.chunk_bits = chunk_bits;
    j.chunk = chunk;
    hipError_t h = hipEventCreateWithFlags(&j.ready, hipEventDisableTiming);
    if (h == hipSuccess) h = hipEventRecord(j.ready, (hipStream_t)stream);
    if (h != hipSuccess) {
        if (j.ready) (void)hipEventDestroy(j.ready);
        return fail_hip(h, "vx_egress_submit");
    }
    {
        std::lock_guard<std::mutex> g(e->mu);
        j.id = ++e->submitted;
        e->queue.push_back(j);
    }
    e->cv_job.notify_one();
    if (job) *job = j.id;
    return VX_OK;
}

vx_status vx_egress_wait(vx_egress *e, uint64_t job) {
    if (!e) return fail(VX_ERR_INVALID_ARG, "egress is NULL");
    std::unique_lock<std::mutex> lk(e->mu);
    const uint64_t target = job ? job : e->submitted;
    if (target > e->submitted) return fail(VX_ERR_INVALID_ARG, "no such egress job");
    e->cv_done.wait(lk, [&] { return e->done >= target; });
    if (e->err != VX_OK) {
        vxs::set_error(e->errmsg);
        return e->err;
    }
    return VX_OK;
}

uint64_t vx_egress_bytes(const vx_egress *e) {
    if (!e) return 0;
    std::lock_guard<std::mutex> g(const_cast<vx_egress *>(e)->mu);
    return e->bytes;
}

vx_status vx_egress_destroy(vx_egress *e) {
    if (!e) return VX_OK;
    vx_status st = vx_egress_wait(e, 0);
    {
        std::lock_guard<std::mutex> g(e->mu);
        e->stop = true;
    }
    e->cv_job.notify_all();
    if (e->worker.joinable()) e->worker.join();
    release(e);
    return st;
}

}  // extern "C"
