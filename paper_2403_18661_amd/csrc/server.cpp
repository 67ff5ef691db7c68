// Streaming server: per-stream device state, rolling PSD, continuous batching
// of window scoring across streams (the snapshotter -> whitener -> network
// ensemble of the paper's inference pipeline, Sec. VI, on one device).
//
// Per stream the device holds the recent raw strain (enough for the 64 s PSD
// background plus filter context), a ring of the segment periodograms of the
// current PSD background, the PSD and whitening response of the current and
// next hop, the recent whitened output and the recent logits.  Each PSD hop
// computes only the periodograms of the segments its background adds (8 of
// 63 at the default 8 s hop) and averages the ring in segment order, which
// gives the same PSD as a Welch estimate over the whole background.
// Whitening runs in fixed 1 s output blocks at absolute positions and PSDs on
// the fixed hop grid, so every result depends only on the stream's own data,
// never on when its chunks arrived or what else shared the batch.  A tick
// takes every pending chunk (up to a per-stream cap), advances each stream,
// then scores all new windows of all streams in one batched call and
// integrates per stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"

using namespace afm;
using Clock = std::chrono::steady_clock;

namespace {

struct Chunk {
    std::vector<double> data;   // [n_ch][n], channel-major
    int64_t n;
    Clock::time_point t;
};

struct Stream {
    bool active = false;
    // device buffers
    double* raw = nullptr;     // [n_ch][cap_raw], absolute sample raw_base at column 0
    double* pg_ring = nullptr; // [n_avg slots][n_ch][F]: periodogram of segment g in slot g % n_avg
    int64_t seg_done = 0;      // segments (of the stream's global grid) whose periodogram was taken
    double* psd = nullptr;     // [2 slots][n_ch][F]
    float* resp = nullptr;     // [2 slots][whiten_resp_floats(n_ch)]
    float* logit = nullptr;    // [cap_logit], absolute logit logit_base at 0
    // progress (absolute indices)
    int64_t raw_base = 0, raw_count = 0;
    int64_t psd_done = 0;           // hops whose response is ready
    int64_t white_base = 0, white_count = 0;
    int64_t next_window = 0;
    int64_t logit_base = 0, logit_count = 0, integ_count = 0;
    std::deque<Chunk> pending;
    // results waiting for af_server_poll
    std::vector<float> out_logits, out_integ;
    int64_t out_logit_first = 0, out_integ_first = 0;
    // per-tick scratch
    std::vector<Clock::time_point> taken_t;
    int64_t tick_first_window = 0, tick_new_windows = 0, tick_prefix = 0;
    int64_t tick_integ_first = 0, tick_new_integ = 0, tick_integ_off = 0;
};

}  // namespace

struct af_server {
    const af_net* net = nullptr;
    af_server_config cfg{};
    int device = 0;
    hipStream_t stream = nullptr;
    int n_ch = 2, window = 3072, M = 1024, F = 2049, RF = 4097;
    int64_t seg_step = 2048, n_avg = 63, hop_seg = 8;   // Welch segment grid
    int64_t n0 = 0, block = 2048;
    int64_t cap_raw = 0, cap_w = 0, cap_logit = 0, tick_cap = 0, max_tick_windows = 0;
    size_t stream_bytes = 0, shared_bytes = 0;
    // shared device buffers
    float* white = nullptr;        // [n_ch][max_streams * cap_w]
    int64_t ld_white = 0;
    void* score_ws = nullptr;
    size_t score_bytes = 0;
    int64_t* d_table = nullptr;
    float* d_logits = nullptr;     // new logits of a tick
    float* d_integ = nullptr;      // new integrated values of a tick
    void* d_tmp = nullptr;         // compaction bounce buffer
    size_t tmp_bytes = 0;
    // pinned host buffers
    double* h_stage = nullptr;
    size_t stage_elems = 0;
    int64_t* h_table = nullptr;
    float* h_logits = nullptr;
    float* h_integ = nullptr;
    std::vector<Stream> streams;
    int64_t n_active = 0;
    std::mutex mu;       // pending queues, results, latencies
    std::mutex tick_mu;  // device state: ticks, admission, release
    std::vector<double> lat_ms;
    int64_t windows_scored = 0;
};

namespace {

void free_stream(Stream& st) {
    if (st.raw) (void)hipFree(st.raw);
    if (st.pg_ring) (void)hipFree(st.pg_ring);
    if (st.psd) (void)hipFree(st.psd);
    if (st.resp) (void)hipFree(st.resp);
    if (st.logit) (void)hipFree(st.logit);
    st = Stream();
}

void free_server(af_server* s) {
    if (!s) return;
    for (Stream& st : s->streams) free_stream(st);
    if (s->white) (void)hipFree(s->white);
    if (s->score_ws) (void)hipFree(s->score_ws);
    if (s->d_table) (void)hipFree(s->d_table);
    if (s->d_logits) (void)hipFree(s->d_logits);
    if (s->d_integ) (void)hipFree(s->d_integ);
    if (s->d_tmp) (void)hipFree(s->d_tmp);
    if (s->h_stage) (void)hipHostFree(s->h_stage);
    if (s->h_table) (void)hipHostFree(s->h_table);
    if (s->h_logits) (void)hipHostFree(s->h_logits);
    if (s->h_integ) (void)hipHostFree(s->h_integ);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

// Move columns [from, to) of a [n_ch][ld] buffer (element size esz) to column 0.
af_status compact(af_server* s, void* buf, int64_t ld, int64_t from, int64_t to, size_t esz) {
    if (from < 0 || to < from) {
        set_error("internal error: compaction range [%lld, %lld)", (long long)from, (long long)to);
        return AF_EINVAL;
    }
    const int64_t len = to - from;
    if (from == 0 || len <= 0) return AF_OK;
    for (int c = 0; c < s->n_ch; ++c) {
        char* base = (char*)buf + (size_t)c * ld * esz;
        AF_HIP(hipMemcpyAsync(s->d_tmp, base + from * esz, len * esz, hipMemcpyDeviceToDevice, s->stream));
        AF_HIP(hipMemcpyAsync(base, s->d_tmp, len * esz, hipMemcpyDeviceToDevice, s->stream));
    }
    return AF_OK;
}

// Compute PSD and whitening response of hop h into slot h & 1: the
// periodograms of the background's segments not taken yet go to the ring,
// then the ring is averaged.
af_status build_hop(af_server* s, Stream& st, int64_t h) {
    const af_server_config& c = s->cfg;
    const int64_t first = h * s->hop_seg, end = first + s->n_avg;   // segments of hop h's background
    if (st.seg_done < first) st.seg_done = first;
    while (st.seg_done < end) {
        const int64_t slot = st.seg_done % s->n_avg;
        const int64_t run = std::min(end - st.seg_done, s->n_avg - slot);
        const int64_t start = st.seg_done * s->seg_step - st.raw_base;
        if (start < 0 || start + (run - 1) * s->seg_step + c.nperseg > st.raw_count - st.raw_base) {
            set_error("internal error: PSD segments of hop %lld are not in the raw buffer", (long long)h);
            return AF_EINVAL;
        }
        af_status r = welch_pgrams(st.raw + start, s->n_ch, s->cap_raw, c.prescale, c.nperseg, s->seg_step, run,
                                   st.pg_ring + (size_t)slot * s->n_ch * s->F, s->stream);
        if (r != AF_OK) return r;
        st.seg_done += run;
    }
    double* psd = st.psd + (size_t)(h & 1) * s->n_ch * s->F;
    float* resp = st.resp + (size_t)(h & 1) * whiten_resp_floats(s->n_ch);
    af_status r = welch_ring_average(st.pg_ring, s->n_ch, c.nperseg, s->n_avg, first % s->n_avg, s->n_avg, c.fs, psd,
                                     s->stream);
    if (r != AF_OK) return r;
    return whiten_build_response(psd, s->n_ch, 1, c.nperseg, c.fs, c.highpass, s->M, resp, s->stream);
}

}  // namespace

extern "C" void af_server_default_config(af_server_config* c) {
    if (!c) return;
    c->fs = 2048.0;
    c->prescale = 1e21;
    c->nperseg = 4096;
    c->noverlap = 2048;
    c->psd_len = 64 * 2048;
    c->psd_hop = 8 * 2048;
    c->fduration = 1.0;
    c->highpass = 32.0;
    c->stride = 128;
    c->integrate_width = 16;
    c->block = 2048;
    c->max_chunk = 8192;
    c->max_tick = 8 * 2048;
    c->max_streams = 64;
    c->score_batch = 2048;
    c->hbm_budget = (size_t)8 << 30;
}

extern "C" af_status af_server_create(const af_net* net, const af_server_config* cfg, af_server** out) {
    clear_error();
    AF_CHECK_ARG(net && cfg && out, "net, cfg and out must be non-null");
    const af_server_config& c = *cfg;
    AF_CHECK_ARG(c.fs > 0 && c.prescale > 0 && c.highpass >= 0, "fs, prescale > 0 and highpass >= 0 required");
    AF_CHECK_ARG(c.nperseg == 4096 || c.nperseg == 2048, "nperseg must be 2048 or 4096");
    AF_CHECK_ARG(c.noverlap >= 0 && c.noverlap < c.nperseg, "noverlap must be in [0, nperseg)");
    const double Md = c.fduration * c.fs / 2.0;
    const int M = (int)llround(Md);
    AF_CHECK_ARG(std::fabs(Md - M) < 1e-9 && M >= 2 && (M & (M - 1)) == 0 && 2 * M <= c.nperseg,
                 "fduration*fs/2 must be a power of two M with 2M <= nperseg");
    AF_CHECK_ARG(c.psd_len >= c.nperseg && c.psd_hop >= 1 && c.psd_hop % (c.nperseg - c.noverlap) == 0,
                 "psd_len >= nperseg and psd_hop a multiple of nperseg - noverlap are required");
    AF_CHECK_ARG(c.block >= 1 && c.block <= kWhitenBlockOut && c.psd_hop % c.block == 0,
                 "block must divide psd_hop and be <= %d", kWhitenBlockOut);
    AF_CHECK_ARG(c.stride >= 1 && c.integrate_width >= 1, "stride and integrate_width must be >= 1");
    AF_CHECK_ARG(c.max_chunk >= 1 && c.max_tick >= c.max_chunk && c.max_streams >= 1 && c.max_streams <= 4096 &&
                     c.score_batch >= 1,
                 "need max_chunk >= 1, max_tick >= max_chunk, 1 <= max_streams <= 4096, score_batch >= 1");
    AF_CHECK_ARG(net_in_ch(net) <= 2, "the server handles at most two detectors");
    af_server* s = new (std::nothrow) af_server();
    if (!s) { set_error("out of host memory"); return AF_ENOMEM; }
    s->net = net;
    s->cfg = c;
    s->device = net_device(net);
    s->n_ch = net_in_ch(net);
    s->window = net_window(net);
    s->M = M;
    s->F = (int)(c.nperseg / 2 + 1);
    s->RF = 8192 / 2 + 1;
    s->n0 = c.psd_len + M;
    s->seg_step = c.nperseg - c.noverlap;
    s->n_avg = (c.psd_len - c.nperseg) / s->seg_step + 1;
    s->hop_seg = c.psd_hop / s->seg_step;
    s->block = c.block;
    s->tick_cap = c.max_tick;
    s->cap_raw = c.psd_len + c.psd_hop + 2 * M + 2 * c.block + c.max_tick + c.max_chunk;
    s->cap_w = s->window + c.stride + c.max_tick + c.max_chunk + 2 * c.block;
    s->max_tick_windows = (c.max_tick + c.max_chunk + c.block) / c.stride + 2;
    s->cap_logit = c.integrate_width + s->max_tick_windows + 16;
    s->ld_white = c.max_streams * s->cap_w;
    s->stream_bytes = (size_t)s->n_ch * s->cap_raw * 8 + (size_t)(2 + s->n_avg) * s->n_ch * s->F * 8 +
                      (size_t)2 * whiten_resp_floats(s->n_ch) * 4 + (size_t)s->cap_logit * 4;
    const int64_t max_windows = c.max_streams * s->max_tick_windows;
    s->score_bytes = af_timeslide_workspace_bytes(net, 1, 1, std::min<int64_t>(c.score_batch, max_windows));
    s->tmp_bytes = std::max<size_t>((size_t)s->cap_raw * 8, (size_t)s->cap_w * 4);
    s->stage_elems = (size_t)c.max_streams * s->n_ch * (c.max_tick + c.max_chunk);
    s->shared_bytes = (size_t)s->n_ch * s->ld_white * 4 + s->score_bytes +
                      (size_t)c.max_streams * 4 * 8 + (size_t)2 * max_windows * 4 + s->tmp_bytes;
    if (s->shared_bytes > c.hbm_budget) {
        free_server(s);
        set_error("hbm_budget %zu is below the server's shared state of %zu bytes", c.hbm_budget,
                  (size_t)s->shared_bytes);
        return AF_EBUDGET;
    }
    s->streams.resize(c.max_streams);
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != s->device) { free_server(s); set_error("current device differs from the net's"); return AF_EINVAL; }
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc((void**)&s->white, (size_t)s->n_ch * s->ld_white * 4) != hipSuccess ||
        hipMalloc(&s->score_ws, s->score_bytes) != hipSuccess ||
        hipMalloc((void**)&s->d_table, (size_t)c.max_streams * 4 * 8) != hipSuccess ||
        hipMalloc((void**)&s->d_logits, (size_t)max_windows * 4) != hipSuccess ||
        hipMalloc((void**)&s->d_integ, (size_t)max_windows * 4) != hipSuccess ||
        hipMalloc(&s->d_tmp, s->tmp_bytes) != hipSuccess ||
        hipHostMalloc((void**)&s->h_stage, s->stage_elems * 8) != hipSuccess ||
        hipHostMalloc((void**)&s->h_table, (size_t)c.max_streams * 4 * 8) != hipSuccess ||
        hipHostMalloc((void**)&s->h_logits, (size_t)max_windows * 4) != hipSuccess ||
        hipHostMalloc((void**)&s->h_integ, (size_t)max_windows * 4) != hipSuccess) {
        free_server(s);
        set_error("server allocation failed");
        return AF_ENOMEM;
    }
    // whitened buffers start zeroed so that nothing uninitialised is ever read
    if (hipMemsetAsync(s->white, 0, (size_t)s->n_ch * s->ld_white * 4, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess) {
        free_server(s);
        set_error("server initialisation failed");
        return AF_EHIP;
    }
    *out = s;
    return AF_OK;
}

extern "C" void af_server_destroy(af_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->tick_mu);
        (void)hipStreamSynchronize(s->stream);
    }
    free_server(s);
}

extern "C" size_t af_server_stream_bytes(const af_server* s) { return s ? s->stream_bytes : 0; }
extern "C" size_t af_server_shared_bytes(const af_server* s) { return s ? s->shared_bytes : 0; }

extern "C" af_status af_server_admit(af_server* s, int64_t* id) {
    clear_error();
    AF_CHECK_ARG(s && id, "server and id must be non-null");
    std::lock_guard<std::mutex> lt(s->tick_mu);
    if (s->shared_bytes + (size_t)(s->n_active + 1) * s->stream_bytes > s->cfg.hbm_budget) {
        set_error("admitting another stream would exceed the HBM budget (%zu bytes for %lld streams)",
                  s->cfg.hbm_budget, (long long)(s->n_active + 1));
        return AF_EBUDGET;
    }
    int64_t slot = -1;
    for (int64_t i = 0; i < (int64_t)s->streams.size(); ++i)
        if (!s->streams[i].active) { slot = i; break; }
    if (slot < 0) {
        set_error("all %lld stream slots are in use", (long long)s->streams.size());
        return AF_EBUDGET;
    }
    Stream& st = s->streams[slot];
    st = Stream();
    if (hipMalloc((void**)&st.raw, (size_t)s->n_ch * s->cap_raw * 8) != hipSuccess ||
        hipMalloc((void**)&st.pg_ring, (size_t)s->n_avg * s->n_ch * s->F * 8) != hipSuccess ||
        hipMalloc((void**)&st.psd, (size_t)2 * s->n_ch * s->F * 8) != hipSuccess ||
        hipMalloc((void**)&st.resp, (size_t)2 * whiten_resp_floats(s->n_ch) * 4) != hipSuccess ||
        hipMalloc((void**)&st.logit, (size_t)s->cap_logit * 4) != hipSuccess) {
        free_stream(st);
        set_error("stream allocation failed");
        return AF_ENOMEM;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        st.active = true;
    }
    ++s->n_active;
    *id = slot;
    return AF_OK;
}

extern "C" af_status af_server_release(af_server* s, int64_t id) {
    clear_error();
    AF_CHECK_ARG(s && id >= 0 && id < (int64_t)s->streams.size(), "bad server or stream id");
    std::lock_guard<std::mutex> lt(s->tick_mu);
    AF_CHECK_ARG(s->streams[id].active, "stream %lld is not active", (long long)id);
    AF_HIP(hipStreamSynchronize(s->stream));
    {
        std::lock_guard<std::mutex> lk(s->mu);
        free_stream(s->streams[id]);
    }
    --s->n_active;
    return AF_OK;
}

extern "C" af_status af_server_push(af_server* s, int64_t id, const double* x, int64_t n) {
    clear_error();
    AF_CHECK_ARG(s && x && id >= 0 && id < (int64_t)s->streams.size(), "bad server, stream id or data");
    AF_CHECK_ARG(n >= 1 && n <= s->cfg.max_chunk, "chunk length must be in [1, max_chunk = %lld]",
                 (long long)s->cfg.max_chunk);
    Chunk ch;
    ch.data.assign(x, x + (size_t)s->n_ch * n);
    ch.n = n;
    ch.t = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    AF_CHECK_ARG(s->streams[id].active, "stream %lld is not active", (long long)id);
    s->streams[id].pending.push_back(std::move(ch));
    return AF_OK;
}

extern "C" af_status af_server_tick(af_server* s, int64_t* n_windows) {
    clear_error();
    AF_CHECK_ARG(s, "server must be non-null");
    std::lock_guard<std::mutex> lt(s->tick_mu);
    const af_server_config& c = s->cfg;
    const int64_t W = c.integrate_width;
    // 1. take pending chunks (whole chunks, up to max_tick samples per stream)
    std::vector<std::vector<Chunk>> taken(s->streams.size());
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (size_t i = 0; i < s->streams.size(); ++i) {
            Stream& st = s->streams[i];
            st.taken_t.clear();
            if (!st.active) continue;
            int64_t got = 0;
            while (!st.pending.empty() && got + st.pending.front().n <= s->tick_cap) {
                got += st.pending.front().n;
                taken[i].push_back(std::move(st.pending.front()));
                st.pending.pop_front();
            }
        }
    }
    // 2. advance every stream: copy in, PSD per hop, whitening blocks, new windows
    size_t stage_off = 0;
    int64_t total = 0;
    int n_entries = 0;
    for (size_t i = 0; i < s->streams.size(); ++i) {
        Stream& st = s->streams[i];
        st.tick_new_windows = 0;
        st.tick_new_integ = 0;
        if (!st.active) continue;
        int64_t incoming = 0;
        for (const Chunk& ch : taken[i]) incoming += ch.n;
        if (incoming > 0) {
            if (st.raw_count + incoming - st.raw_base > s->cap_raw) {
                // keep what the next whitening block needs (from n0 + b*block - M)
                // and what the next PSD to build needs (hop psd_done reads its
                // background from psd_done*psd_hop, which lies psd_len - psd_hop
                // before its first block's context)
                // the next block's context, and the raw data of the next
                // periodogram to take
                const int64_t b = st.white_count / s->block;
                int64_t keep = s->n0 + b * s->block - s->M;
                keep = std::min<int64_t>(keep, std::max(st.seg_done, st.psd_done * s->hop_seg) * s->seg_step);
                keep = std::min(keep, st.raw_count);
                af_status r = compact(s, st.raw, s->cap_raw, keep - st.raw_base, st.raw_count - st.raw_base, 8);
                if (r != AF_OK) return r;
                st.raw_base = keep;
            }
            AF_CHECK_ARG(st.raw_count + incoming - st.raw_base <= s->cap_raw, "stream %zu raw buffer overflow", i);
            for (const Chunk& ch : taken[i]) {
                for (int cc = 0; cc < s->n_ch; ++cc) {
                    double* dst = s->h_stage + stage_off;
                    std::memcpy(dst, ch.data.data() + (size_t)cc * ch.n, (size_t)ch.n * 8);
                    AF_HIP(hipMemcpyAsync(st.raw + (size_t)cc * s->cap_raw + (st.raw_count - st.raw_base), dst,
                                          (size_t)ch.n * 8, hipMemcpyHostToDevice, s->stream));
                    stage_off += (size_t)ch.n;
                }
                st.raw_count += ch.n;
                st.taken_t.push_back(ch.t);
            }
        }
        // whitening blocks whose input (plus M samples of context) has arrived
        while (st.raw_count >= s->n0 + (st.white_count / s->block + 1) * s->block + s->M) {
            const int64_t b = st.white_count / s->block;
            const int64_t h = (b * s->block) / c.psd_hop;
            while (st.psd_done <= h) {
                af_status r = build_hop(s, st, st.psd_done);
                if (r != AF_OK) return r;
                ++st.psd_done;
            }
            if (st.white_count + s->block - st.white_base > s->cap_w) {
                const int64_t keep = std::min(st.next_window * c.stride, st.white_count);
                af_status r = compact(s, s->white + i * s->cap_w, s->ld_white, keep - st.white_base,
                                      st.white_count - st.white_base, 4);
                if (r != AF_OK) return r;
                st.white_base = keep;
            }
            AF_CHECK_ARG(st.white_count + s->block - st.white_base <= s->cap_w, "stream %zu whitened buffer overflow", i);
            AF_CHECK_ARG(s->n0 + b * s->block - s->M >= st.raw_base,
                         "internal error: whitening context of stream %zu is not in the raw buffer", i);
            af_status r = whiten_apply(st.raw, AF_IN_F64, s->n_ch, st.raw_count - st.raw_base, s->cap_raw, c.prescale,
                                       st.resp + (size_t)(h & 1) * whiten_resp_floats(s->n_ch), 1, 0, s->M,
                                       s->n0 + b * s->block - st.raw_base, s->block,
                                       s->white + i * s->cap_w + (st.white_count - st.white_base), s->ld_white,
                                       s->stream);
            if (r != AF_OK) return r;
            st.white_count += s->block;
        }
        // new windows of this stream
        const int64_t n_w = st.white_count >= s->window ? (st.white_count - s->window) / c.stride + 1 : 0;
        if (n_w > st.next_window) {
            int64_t* e = s->h_table + 4 * n_entries;
            e[0] = (int64_t)i * s->cap_w + (st.next_window * c.stride - st.white_base);
            e[1] = s->cap_w;     // never wraps: every window lies inside the stream's buffer
            e[2] = 0;
            e[3] = total;
            st.tick_first_window = st.next_window;
            st.tick_new_windows = n_w - st.next_window;
            st.tick_prefix = total;
            total += st.tick_new_windows;
            st.next_window = n_w;
            ++n_entries;
        }
    }
    // 3. one batched scoring call over the new windows of every stream
    if (total > 0) {
        AF_HIP(hipMemcpyAsync(s->d_table, s->h_table, (size_t)n_entries * 4 * 8, hipMemcpyHostToDevice, s->stream));
        af_status r = score_table(s->net, s->white, s->ld_white, s->ld_white, c.stride, total, s->d_table, n_entries,
                                  s->d_logits, s->score_ws, s->score_bytes, s->stream);
        if (r != AF_OK) return r;
    }
    // 4. per-stream logit history and integration
    int64_t n_int_total = 0;
    for (size_t i = 0; i < s->streams.size(); ++i) {
        Stream& st = s->streams[i];
        if (!st.active || st.tick_new_windows == 0) continue;
        if (st.logit_count + st.tick_new_windows - st.logit_base > s->cap_logit) {
            const int64_t keep = std::min(st.integ_count, st.logit_count);
            if (keep > st.logit_base) {
                AF_HIP(hipMemcpyAsync(s->d_tmp, st.logit + (keep - st.logit_base), (st.logit_count - keep) * 4,
                                      hipMemcpyDeviceToDevice, s->stream));
                AF_HIP(hipMemcpyAsync(st.logit, s->d_tmp, (st.logit_count - keep) * 4, hipMemcpyDeviceToDevice,
                                      s->stream));
                st.logit_base = keep;
            }
        }
        AF_CHECK_ARG(st.logit_count + st.tick_new_windows - st.logit_base <= s->cap_logit, "logit history overflow");
        AF_HIP(hipMemcpyAsync(st.logit + (st.logit_count - st.logit_base), s->d_logits + st.tick_prefix,
                              st.tick_new_windows * 4, hipMemcpyDeviceToDevice, s->stream));
        st.logit_count += st.tick_new_windows;
        const int64_t n_int = st.logit_count >= W ? st.logit_count - W + 1 : 0;
        if (n_int > st.integ_count) {
            st.tick_integ_first = st.integ_count;
            st.tick_new_integ = n_int - st.integ_count;
            st.tick_integ_off = n_int_total;
            af_status r = af_integrate(st.logit + (st.integ_count - st.logit_base), st.logit_count - st.integ_count, W, nullptr,
                                       s->d_integ + n_int_total, s->stream);
            if (r != AF_OK) return r;
            n_int_total += st.tick_new_integ;
            st.integ_count = n_int;
        }
    }
    // 5. results to the host
    if (total > 0)
        AF_HIP(hipMemcpyAsync(s->h_logits, s->d_logits, total * 4, hipMemcpyDeviceToHost, s->stream));
    if (n_int_total > 0)
        AF_HIP(hipMemcpyAsync(s->h_integ, s->d_integ, n_int_total * 4, hipMemcpyDeviceToHost, s->stream));
    AF_HIP(hipStreamSynchronize(s->stream));
    const Clock::time_point done = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (Stream& st : s->streams) {
            if (!st.active) continue;
            if (st.tick_new_windows > 0) {
                if (st.out_logits.empty()) st.out_logit_first = st.tick_first_window;
                st.out_logits.insert(st.out_logits.end(), s->h_logits + st.tick_prefix,
                                     s->h_logits + st.tick_prefix + st.tick_new_windows);
            }
            if (st.tick_new_integ > 0) {
                if (st.out_integ.empty()) st.out_integ_first = st.tick_integ_first;
                st.out_integ.insert(st.out_integ.end(), s->h_integ + st.tick_integ_off,
                                    s->h_integ + st.tick_integ_off + st.tick_new_integ);
                // arrival -> integrated statistic on the host, for the chunks that produced it
                for (const auto& t : st.taken_t)
                    s->lat_ms.push_back(std::chrono::duration<double, std::milli>(done - t).count());
            }
        }
    }
    s->windows_scored += total;
    if (n_windows) *n_windows = total;
    return AF_OK;
}

extern "C" af_status af_server_poll(af_server* s, int64_t id, float* logits, int64_t cap_logits, int64_t* n_logits,
                                    int64_t* first_logit, float* integ, int64_t cap_integ, int64_t* n_integ,
                                    int64_t* first_integ) {
    clear_error();
    AF_CHECK_ARG(s && id >= 0 && id < (int64_t)s->streams.size() && n_logits && n_integ && first_logit && first_integ,
                 "bad arguments");
    std::lock_guard<std::mutex> lk(s->mu);
    Stream& st = s->streams[id];
    AF_CHECK_ARG(st.active, "stream %lld is not active", (long long)id);
    const int64_t nl = std::min<int64_t>((int64_t)st.out_logits.size(), logits ? cap_logits : 0);
    const int64_t ni = std::min<int64_t>((int64_t)st.out_integ.size(), integ ? cap_integ : 0);
    if (nl > 0) std::memcpy(logits, st.out_logits.data(), nl * 4);
    if (ni > 0) std::memcpy(integ, st.out_integ.data(), ni * 4);
    *first_logit = st.out_logit_first;
    *first_integ = st.out_integ_first;
    *n_logits = nl;
    *n_integ = ni;
    st.out_logits.erase(st.out_logits.begin(), st.out_logits.begin() + nl);
    st.out_integ.erase(st.out_integ.begin(), st.out_integ.begin() + ni);
    st.out_logit_first += nl;
    st.out_integ_first += ni;
    return AF_OK;
}

extern "C" af_status af_server_stats(af_server* s, double* p50_ms, double* p99_ms, int64_t* n_samples,
                                     int64_t* windows, int reset) {
    clear_error();
    AF_CHECK_ARG(s && p50_ms && p99_ms && n_samples && windows, "bad arguments");
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> v = s->lat_ms;
    *n_samples = (int64_t)v.size();
    *windows = s->windows_scored;
    *p50_ms = *p99_ms = 0.0;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto q = [&](double p) {
            const double pos = p * (double)(v.size() - 1);
            const size_t lo = (size_t)std::floor(pos), hi = std::min(lo + 1, v.size() - 1);
            return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
        };
        *p50_ms = q(0.50);
        *p99_ms = q(0.99);
    }
    if (reset) {
        s->lat_ms.clear();
        s->windows_scored = 0;
    }
    return AF_OK;
}
