// Host side of the libpolymh C ABI: argument validation, workspace carving,
// launch-shape defaults and error reporting.  Every computation is a kernel
// launch on the caller's stream; nothing here touches polygon data.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

namespace polymh {

namespace {
thread_local char g_err[512] = "";
}

polymh_status set_error(polymh_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

polymh_status check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(POLYMH_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return POLYMH_OK;
}

int cu_count()
{
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if (cache[dev] == 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
            c = 256;
        cache[dev] = c;
    }
    return cache[dev];
}

}  // namespace polymh

using namespace polymh;

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

polymh_status check_polys(const polymh_polys *p, const char *what)
{
    if (!p) return set_error(POLYMH_EINVAL, "%s: polygon set is NULL", what);
    if (p->n < 0) return set_error(POLYMH_EINVAL, "%s: negative polygon count", what);
    if (p->n > 0 && (!p->xy || !p->offsets))
        return set_error(POLYMH_EINVAL, "%s: NULL vertex or offset array", what);
    if (p->n > 0x7fffffffLL) return set_error(POLYMH_EINVAL, "%s: more than 2^31-1 polygons", what);
    return POLYMH_OK;
}

polymh_status check_box(const polymh_box &b, const char *what)
{
    if (b.xmin > b.xmax || b.ymin > b.ymax)
        return set_error(POLYMH_ERANGE, "%s: empty sampling box [%d,%d]x[%d,%d]", what, b.xmin,
                         b.xmax, b.ymin, b.ymax);
    return POLYMH_OK;
}

polymh_status check_sign_config(const polymh_sign_config &c)
{
    if (c.block_threads < 64 || c.block_threads > 512 || c.block_threads % 64)
        return set_error(POLYMH_EINVAL, "sign: block_threads must be 64..512, a multiple of 64");
    if (c.hash_block < 0) return set_error(POLYMH_EINVAL, "sign: negative hash_block");
    if (c.lds_edges < 64 || c.lds_edges > 8192)
        return set_error(POLYMH_EINVAL, "sign: lds_edges must be 64..8192");
    if (c.samples_per_lane != 1 && c.samples_per_lane != 2)
        return set_error(POLYMH_EINVAL, "sign: samples_per_lane must be 1 or 2");
    if (c.persistent && (c.blocks_per_cu < 1 || c.blocks_per_cu > 64))
        return set_error(POLYMH_EINVAL, "sign: blocks_per_cu must be 1..64");
    return POLYMH_OK;
}

struct SignWs {
    unsigned long long *queue;
    int32_t *mbr;
    int64_t *area2;
    uint32_t *flags;
    int32_t *counts;
    int32_t *order;
};

SignWs carve_sign(Carve &c, int64_t n, bool persistent)
{
    SignWs w{};
    w.queue = c.take<unsigned long long>(1);
    w.mbr = c.take<int32_t>((size_t)n * 4);
    w.area2 = c.take<int64_t>((size_t)n);
    w.flags = c.take<uint32_t>((size_t)n);
    if (persistent) {
        w.counts = c.take<int32_t>(128);
        w.order = c.take<int32_t>((size_t)n);
    }
    return w;
}

}  // namespace

extern "C" {

const char *polymh_last_error(void) { return g_err; }

int32_t polymh_version(void) { return 100; }

polymh_status polymh_check_device(void)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(POLYMH_EDEVICE, "check_device: %s", hipGetErrorString(e));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return set_error(POLYMH_EDEVICE, "check_device: %s", hipGetErrorString(e));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(POLYMH_ENOTSUP, "check_device: device %d is %s, not gfx950", dev, prop.gcnArchName);
    return POLYMH_OK;
}

polymh_status polymh_prepare(const polymh_polys *polys, int32_t *mbr, int64_t *area2,
                             uint32_t *flags, void *stream)
{
    polymh_status st = check_polys(polys, "prepare");
    if (st) return st;
    if (polys->n > 0 && !mbr) return set_error(POLYMH_EINVAL, "prepare: mbr is NULL");
    return launch_prepare(polys->xy, polys->offsets, polys->n, mbr, area2, flags, as_stream(stream));
}

polymh_status polymh_centre(const polymh_polys *polys, int32_t *xy_out, int32_t *shift,
                            int32_t *range_flag, void *stream)
{
    polymh_status st = check_polys(polys, "centre");
    if (st) return st;
    if (polys->n > 0 && !xy_out) return set_error(POLYMH_EINVAL, "centre: xy_out is NULL");
    if (polys->n > 0 && xy_out == polys->xy) return set_error(POLYMH_EINVAL, "centre: xy_out aliases the input");
    return launch_centre(polys->xy, polys->offsets, polys->n, xy_out, shift, range_flag, as_stream(stream));
}

size_t polymh_box_of_workspace_size(void) { return 256; }

polymh_status polymh_box_of(const polymh_polys *polys, void *ws, size_t ws_bytes,
                            polymh_box *out_host, void *stream)
{
    polymh_status st = check_polys(polys, "box_of");
    if (st) return st;
    if (!out_host) return set_error(POLYMH_EINVAL, "box_of: out_host is NULL");
    if (!ws || ws_bytes < polymh_box_of_workspace_size())
        return set_error(POLYMH_ECAPACITY, "box_of: workspace too small");
    if (polys->n == 0) return set_error(POLYMH_EINVAL, "box_of: empty polygon set");
    int64_t nv = 0;
    hipStream_t s = as_stream(stream);
    hipError_t e = hipMemcpyAsync(&nv, polys->offsets + polys->n, sizeof(int64_t),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(POLYMH_EDEVICE, "box_of: %s", hipGetErrorString(e));
    if (nv <= 0) return set_error(POLYMH_EINVAL, "box_of: polygon set has no vertex");
    int32_t *acc = static_cast<int32_t *>(ws);
    st = launch_box_of(polys->xy, nv, acc, s);
    if (st) return st;
    int32_t h[4];
    e = hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(POLYMH_EDEVICE, "box_of: %s", hipGetErrorString(e));
    out_host->xmin = h[0];
    out_host->ymin = h[1];
    out_host->xmax = h[2];
    out_host->ymax = h[3];
    return POLYMH_OK;
}

void polymh_sign_default_config(polymh_sign_config *cfg)
{
    if (!cfg) return;
    cfg->persistent = 1;
    cfg->block_threads = 256;
    cfg->hash_block = 0;
    cfg->lds_edges = 1024;
    cfg->samples_per_lane = 1;
    cfg->blocks_per_cu = 8;
}

size_t polymh_sign_workspace_size(int64_t n, const polymh_sign_config *cfg)
{
    polymh_sign_config c;
    if (cfg) c = *cfg;
    else polymh_sign_default_config(&c);
    if (n < 0) n = 0;
    Carve cv{nullptr, 0};
    carve_sign(cv, n, c.persistent != 0);
    return align_up(cv.used, 256);
}

polymh_status polymh_sign(const polymh_polys *polys, polymh_box box, uint64_t seed, int32_t k,
                          uint32_t cap, uint32_t *sig, const polymh_sign_config *cfg, void *ws,
                          size_t ws_bytes, void *stream)
{
    polymh_status st = check_polys(polys, "sign");
    if (st) return st;
    if ((st = check_box(box, "sign"))) return st;
    if (k < 1) return set_error(POLYMH_EINVAL, "sign: k must be >= 1");
    if (cap < 1) return set_error(POLYMH_EINVAL, "sign: cap must be >= 1");
    polymh_sign_config c;
    if (cfg) c = *cfg;
    else polymh_sign_default_config(&c);
    if ((st = check_sign_config(c))) return st;
    if (polys->n == 0) return POLYMH_OK;
    if (!sig) return set_error(POLYMH_EINVAL, "sign: sig is NULL");
    if ((int64_t)polys->n * k > (int64_t)1 << 40)
        return set_error(POLYMH_EINVAL, "sign: n * k too large");
    Carve cv{static_cast<char *>(ws), ws_bytes};
    SignWs w = carve_sign(cv, polys->n, c.persistent != 0);
    if (!cv.ok)
        return set_error(POLYMH_ECAPACITY, "sign: workspace of %zu bytes, need %zu", ws_bytes, cv.used);
    hipStream_t s = as_stream(stream);
    if ((st = launch_prepare(polys->xy, polys->offsets, polys->n, w.mbr, w.area2, w.flags, s))) return st;
    if (c.persistent) {
        if ((st = launch_sign_order(polys->offsets, w.mbr, w.area2, w.flags, polys->n, box, k, cap,
                                    w.counts, w.order, s)))
            return st;
    }
    SignLaunch L{};
    L.xy = polys->xy;
    L.off = polys->offsets;
    L.mbr = w.mbr;
    L.flags = w.flags;
    L.order = c.persistent ? w.order : nullptr;
    L.queue = c.persistent ? w.queue : nullptr;
    L.sig = sig;
    L.n = polys->n;
    L.box = box;
    L.seed = seed;
    L.k = k;
    L.cap = cap;
    L.cfg = c;
    return launch_sign(L, s);
}

}  // extern "C"

namespace {

// Scratch of polymh_sign_static: the staging polymh_sign keeps in its
// workspace (work-queue counter, MBRs, doubled areas, flags, longest-first
// order) for up to POLYMH_SIGN_STATIC_MAX_POLYS polygons, laid out as
// carve_sign lays out a workspace.  One copy per GPU, held until the process
// ends.  In host code `scratch` names a host-side stand-in, never the device
// memory: kernels get the address hipGetSymbolAddress returns for the
// current device.
constexpr size_t kStaticSignBytes = (8u << 20) + 4096;
__device__ __align__(256) unsigned char scratch[kStaticSignBytes];

// The device address of this GPU's `scratch`, looked up once per device with
// that device current.
polymh_status static_scratch(char **out)
{
    static std::mutex mu;
    static char *ptrs[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(POLYMH_EDEVICE, "sign_static: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= 64) return set_error(POLYMH_EINVAL, "sign_static: device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(mu);
    if (!ptrs[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(POLYMH_EDEVICE, "sign_static: scratch address: %s", hipGetErrorString(e));
        ptrs[dev] = static_cast<char *>(p);
    }
    *out = ptrs[dev];
    return POLYMH_OK;
}

}  // namespace

extern "C" {

polymh_status polymh_sign_static(const polymh_polys *polys, polymh_box box, uint64_t seed, int32_t k,
                                 uint32_t cap, uint32_t *sig, const polymh_sign_config *cfg, void *stream)
{
    polymh_status st = check_polys(polys, "sign_static");
    if (st) return st;
    if (polys->n > POLYMH_SIGN_STATIC_MAX_POLYS)
        return set_error(POLYMH_EINVAL, "sign_static: %lld polygons, at most %d (use polymh_sign with a workspace)",
                         (long long)polys->n, POLYMH_SIGN_STATIC_MAX_POLYS);
    polymh_sign_config c;
    if (cfg) c = *cfg;
    else polymh_sign_default_config(&c);
    Carve need{nullptr, 0};
    carve_sign(need, polys->n, c.persistent != 0);
    if (need.used > kStaticSignBytes)
        return set_error(POLYMH_EINVAL, "sign_static: staging needs %zu bytes, the scratch holds %zu", need.used,
                         kStaticSignBytes);
    char *ws = nullptr;
    if ((st = static_scratch(&ws))) return st;
    return polymh_sign(polys, box, seed, k, cap, sig, &c, ws, kStaticSignBytes, stream);
}

int64_t polymh_join_rings_size(int64_t n_vertices, int64_t n_rings, int64_t n_polys)
{
    if (n_vertices < 0 || n_rings < 0 || n_polys < 0) return -1;
    return n_vertices + 2 * (n_rings - n_polys);
}

polymh_status polymh_join_rings(const int32_t *xy, int64_t n_vertices, const int64_t *ring_offsets,
                                int64_t n_rings, const int64_t *poly_rings, int64_t n_polys, int32_t *out_xy,
                                int64_t out_capacity, int64_t *out_offsets, int32_t *bad_flag, void *stream)
{
    if (n_polys < 0 || n_rings < 0 || n_vertices < 0 || out_capacity < 0)
        return set_error(POLYMH_EINVAL, "join_rings: negative size");
    if (n_polys == 0) return POLYMH_OK;
    if (!xy || !ring_offsets || !poly_rings || !out_xy || !out_offsets)
        return set_error(POLYMH_EINVAL, "join_rings: NULL array");
    if (out_xy == xy) return set_error(POLYMH_EINVAL, "join_rings: out_xy aliases xy");
    return launch_join_rings(xy, n_vertices, ring_offsets, n_rings, poly_rings, n_polys, out_xy, out_capacity,
                             out_offsets, bad_flag, as_stream(stream));
}

size_t polymh_sign_binned_workspace_size(int64_t n, int32_t k, uint32_t cap, uint32_t horizon, int32_t bin_bits,
                                         const polymh_sign_config *cfg)
{
    (void)cfg;
    if (n < 0) n = 0;
    if (k < 1 || bin_bits < 0 || bin_bits > 6 || horizon < 1) return 0;
    if (horizon > cap) horizon = cap;
    Carve cv{nullptr, 0};
    carve_sign(cv, n, true);
    return align_up(cv.used, 256) + binned_workspace_bytes(k, horizon, bin_bits, n) + 256;
}

static polymh_status sign_binned_impl(const polymh_polys *polys, polymh_box box, uint64_t seed, int32_t k,
                                      uint32_t cap, uint32_t horizon, int32_t bin_bits, double walk_ratio,
                                      uint32_t *sig, const polymh_sign_config *cfg, void *ws, size_t ws_bytes,
                                      void *stream, bool rebin)
{
    polymh_status st = check_polys(polys, "sign_binned");
    if (st) return st;
    if ((st = check_box(box, "sign_binned"))) return st;
    if (k < 1 || k > 65535) return set_error(POLYMH_EINVAL, "sign_binned: k must be 1..65535");
    if (cap < 1) return set_error(POLYMH_EINVAL, "sign_binned: cap must be >= 1");
    if (horizon < 1) return set_error(POLYMH_EINVAL, "sign_binned: horizon must be >= 1");
    if (bin_bits < 0 || bin_bits > 6) return set_error(POLYMH_EINVAL, "sign_binned: bin_bits must be 0..6");
    if (!(walk_ratio >= 0.0)) return set_error(POLYMH_EINVAL, "sign_binned: walk_ratio must be >= 0");
    if (horizon > cap) horizon = cap;
    polymh_sign_config c;
    if (cfg) c = *cfg;
    else polymh_sign_default_config(&c);
    c.persistent = 1;
    if ((st = check_sign_config(c))) return st;
    if (polys->n == 0) return POLYMH_OK;
    if (!sig) return set_error(POLYMH_EINVAL, "sign_binned: sig is NULL");
    if ((int64_t)polys->n * k > (int64_t)1 << 40)
        return set_error(POLYMH_EINVAL, "sign_binned: n * k too large");
    Carve cv{static_cast<char *>(ws), ws_bytes};
    SignWs w = carve_sign(cv, polys->n, true);
    if (!cv.ok)
        return set_error(POLYMH_ECAPACITY, "sign_binned: workspace of %zu bytes too small", ws_bytes);
    const size_t used = align_up(cv.used, 256);
    hipStream_t s = as_stream(stream);
    if ((st = launch_prepare(polys->xy, polys->offsets, polys->n, w.mbr, w.area2, w.flags, s))) return st;
    SignLaunch L{};
    L.xy = polys->xy;
    L.off = polys->offsets;
    L.mbr = w.mbr;
    L.flags = w.flags;
    L.queue = w.queue;
    L.sig = sig;
    L.n = polys->n;
    L.box = box;
    L.seed = seed;
    L.k = k;
    L.cap = cap;
    L.cfg = c;
    if (used > ws_bytes) return set_error(POLYMH_ECAPACITY, "sign_binned: workspace too small");
    return launch_sign_binned(L, w.area2, horizon, bin_bits, walk_ratio, static_cast<char *>(ws) + used,
                              ws_bytes - used, s, rebin);
}

polymh_status polymh_sign_binned(const polymh_polys *polys, polymh_box box, uint64_t seed, int32_t k,
                                 uint32_t cap, uint32_t horizon, int32_t bin_bits, double walk_ratio, uint32_t *sig,
                                 const polymh_sign_config *cfg, void *ws, size_t ws_bytes, void *stream)
{
    return sign_binned_impl(polys, box, seed, k, cap, horizon, bin_bits, walk_ratio, sig, cfg, ws, ws_bytes, stream,
                            true);
}

polymh_status polymh_sign_binned_prebinned(const polymh_polys *polys, polymh_box box, uint64_t seed, int32_t k,
                                           uint32_t cap, uint32_t horizon, int32_t bin_bits, double walk_ratio,
                                           uint32_t *sig, const polymh_sign_config *cfg, void *ws, size_t ws_bytes,
                                           void *stream)
{
    return sign_binned_impl(polys, box, seed, k, cap, horizon, bin_bits, walk_ratio, sig, cfg, ws, ws_bytes, stream,
                            false);
}

polymh_status polymh_band(const uint32_t *sig, int64_t n, int32_t k, int32_t b, int32_t r,
                          uint64_t band_seed, uint64_t *keys, void *stream)
{
    if (n < 0 || k < 1 || b < 1 || r < 1) return set_error(POLYMH_EINVAL, "band: bad sizes");
    if ((int64_t)b * r > k) return set_error(POLYMH_EINVAL, "band: b*r = %d exceeds k = %d", b * r, k);
    if (n == 0) return POLYMH_OK;
    if (!sig || !keys) return set_error(POLYMH_EINVAL, "band: NULL array");
    return launch_band(sig, n, k, b, r, band_seed, keys, as_stream(stream));
}

size_t polymh_index_workspace_size(int64_t n, int32_t b)
{
    if (n < 0 || b < 1) return 0;
    return index_workspace_bytes(n * b);
}

polymh_status polymh_index_build(const uint64_t *keys, int64_t n, int32_t b, void *ws,
                                 size_t ws_bytes, uint64_t *sorted_keys, int32_t *sorted_ids,
                                 void *stream)
{
    if (n < 0 || b < 1) return set_error(POLYMH_EINVAL, "index_build: bad sizes");
    if (n == 0) return POLYMH_OK;
    if (!keys || !sorted_keys || !sorted_ids) return set_error(POLYMH_EINVAL, "index_build: NULL array");
    return launch_index_build(keys, n, b, ws, ws_bytes, sorted_keys, sorted_ids, as_stream(stream));
}

size_t polymh_query_workspace_size(int64_t n_data, int64_t nq)
{
    if (n_data < 0 || nq < 0) return 0;
    return query_workspace_bytes(n_data, nq);
}

polymh_status polymh_query(const uint64_t *sorted_keys, const int32_t *sorted_ids,
                           int64_t n_entries, int64_t n_data, const uint64_t *qkeys, int64_t nq,
                           int32_t b, void *ws, size_t ws_bytes, int64_t *cand_off,
                           int32_t *cand_ids, int64_t cand_cap, void *stream)
{
    if (n_entries < 0 || n_data < 0 || nq < 0 || b < 1)
        return set_error(POLYMH_EINVAL, "query: bad sizes");
    if (!cand_off) return set_error(POLYMH_EINVAL, "query: cand_off is NULL");
    if (nq > 0 && !qkeys) return set_error(POLYMH_EINVAL, "query: qkeys is NULL");
    if (n_entries > 0 && (!sorted_keys || !sorted_ids))
        return set_error(POLYMH_EINVAL, "query: NULL bucket table");
    hipStream_t s = as_stream(stream);
    if (cand_ids && cand_cap >= 0) {
        int64_t total = 0;
        hipError_t e = hipMemcpyAsync(&total, cand_off + nq, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return set_error(POLYMH_EDEVICE, "query: %s", hipGetErrorString(e));
        if (total > cand_cap)
            return set_error(POLYMH_ECAPACITY, "query: %lld candidates exceed capacity %lld",
                             (long long)total, (long long)cand_cap);
    }
    return launch_query(sorted_keys, sorted_ids, n_entries, n_data, qkeys, nq, b, ws, ws_bytes,
                        cand_off, cand_ids, s);
}

polymh_status polymh_query_capped(const uint64_t *sorted_keys, const int32_t *sorted_ids,
                                  int64_t n_entries, int64_t n_data, const uint64_t *qkeys, int64_t nq,
                                  int32_t b, void *ws, size_t ws_bytes, int64_t *cand_off,
                                  int32_t *cand_ids, int64_t cand_cap, int32_t *overflow, void *stream)
{
    if (n_entries < 0 || n_data < 0 || nq < 0 || b < 1 || cand_cap < 0)
        return set_error(POLYMH_EINVAL, "query_capped: bad sizes");
    if (!cand_off || !overflow || (cand_cap > 0 && !cand_ids))
        return set_error(POLYMH_EINVAL, "query_capped: NULL output");
    if (nq > 0 && !qkeys) return set_error(POLYMH_EINVAL, "query_capped: qkeys is NULL");
    if (n_entries > 0 && (!sorted_keys || !sorted_ids))
        return set_error(POLYMH_EINVAL, "query_capped: NULL bucket table");
    return launch_query_capped(sorted_keys, sorted_ids, n_entries, n_data, qkeys, nq, b, ws, ws_bytes,
                               cand_off, cand_ids, cand_cap, overflow, as_stream(stream));
}

polymh_status polymh_refine(const polymh_polys *data, const polymh_polys *queries,
                            const int64_t *cand_off, const int32_t *cand_ids, int64_t nq,
                            int64_t n_cand, double *cand_j, void *stream)
{
    polymh_status st = check_polys(data, "refine");
    if (st) return st;
    if ((st = check_polys(queries, "refine"))) return st;
    if (nq != queries->n) return set_error(POLYMH_EINVAL, "refine: nq differs from the query count");
    if (n_cand < 0) return set_error(POLYMH_EINVAL, "refine: negative candidate count");
    if (n_cand == 0 || nq == 0) return POLYMH_OK;
    if (!cand_off || !cand_ids || !cand_j) return set_error(POLYMH_EINVAL, "refine: NULL array");
    return launch_refine(data, queries, cand_off, cand_ids, nq, n_cand, cand_j, as_stream(stream));
}

size_t polymh_refine_workspace_size(void) { return refine_workspace_bytes(); }

polymh_status polymh_refine_ws(const polymh_polys *data, const polymh_polys *queries, const int64_t *cand_off,
                               const int32_t *cand_ids, int64_t nq, int64_t n_cand, double *cand_j,
                               uint64_t *stats, void *ws, size_t ws_bytes, void *stream)
{
    polymh_status st = check_polys(data, "refine_ws");
    if (st) return st;
    if ((st = check_polys(queries, "refine_ws"))) return st;
    if (nq != queries->n) return set_error(POLYMH_EINVAL, "refine_ws: nq differs from the query count");
    if (n_cand < 0) return set_error(POLYMH_EINVAL, "refine_ws: negative candidate count");
    if (n_cand == 0 || nq == 0) return POLYMH_OK;
    if (!cand_off || !cand_ids || !cand_j) return set_error(POLYMH_EINVAL, "refine_ws: NULL array");
    return launch_refine(data, queries, cand_off, cand_ids, nq, n_cand, cand_j, as_stream(stream),
                         reinterpret_cast<unsigned long long *>(stats), ws, ws ? ws_bytes : 0);
}

polymh_status polymh_refine_stats(const polymh_polys *data, const polymh_polys *queries,
                                  const int64_t *cand_off, const int32_t *cand_ids, int64_t nq,
                                  int64_t n_cand, double *cand_j, uint64_t *stats, void *stream)
{
    polymh_status st = check_polys(data, "refine_stats");
    if (st) return st;
    if ((st = check_polys(queries, "refine_stats"))) return st;
    if (nq != queries->n) return set_error(POLYMH_EINVAL, "refine_stats: nq differs from the query count");
    if (n_cand < 0 || !stats) return set_error(POLYMH_EINVAL, "refine_stats: bad arguments");
    if (n_cand == 0 || nq == 0) return POLYMH_OK;
    if (!cand_off || !cand_ids || !cand_j) return set_error(POLYMH_EINVAL, "refine_stats: NULL array");
    return launch_refine(data, queries, cand_off, cand_ids, nq, n_cand, cand_j, as_stream(stream),
                         reinterpret_cast<unsigned long long *>(stats));
}

polymh_status polymh_topk(const int64_t *cand_off, const int32_t *cand_ids, const double *cand_j,
                          int64_t nq, int32_t topk, int32_t *top_ids, double *top_j, void *stream)
{
    if (nq < 0 || topk < 1 || topk > 1024) return set_error(POLYMH_EINVAL, "topk: bad sizes");
    if (nq == 0) return POLYMH_OK;
    if (!cand_off || !top_ids || !top_j) return set_error(POLYMH_EINVAL, "topk: NULL array");
    return launch_topk(cand_off, cand_ids, cand_j, nq, topk, top_ids, top_j, as_stream(stream));
}

/* ------------------------------------------------------------------ scorer */

int64_t polymh_mlp_param_count(void) { return mlp_param_count(); }
int64_t polymh_mlp_bf16_count(void) { return mlp_bf16_count(); }
size_t polymh_mlp_acts_size(int64_t B) { return B < 0 ? 0 : mlp_acts_bytes_aligned(B); }
size_t polymh_mlp_scratch_size(int64_t B) { return B < 0 ? 0 : mlp_backward_scratch_bytes(B); }

polymh_status polymh_mlp_sync_bf16(const float *params, uint16_t *wbf16, void *stream)
{
    if (!params || !wbf16) return set_error(POLYMH_EINVAL, "mlp_sync_bf16: NULL array");
    return launch_mlp_sync_bf16(params, wbf16, as_stream(stream));
}

static polymh_status check_batch(int64_t B, const char *what)
{
    if (B < 0 || B % 32) return set_error(POLYMH_EINVAL, "%s: batch must be a non-negative multiple of 32", what);
    return POLYMH_OK;
}

polymh_status polymh_mlp_forward(const uint16_t *X, int64_t B, const float *params,
                                 const uint16_t *wbf16, float *y, void *acts, size_t acts_bytes,
                                 void *stream)
{
    polymh_status st = check_batch(B, "mlp_forward");
    if (st) return st;
    if (B == 0) return POLYMH_OK;
    if (!X || !params || !wbf16 || !acts) return set_error(POLYMH_EINVAL, "mlp_forward: NULL array");
    if (acts_bytes < mlp_acts_bytes_aligned(B))
        return set_error(POLYMH_ECAPACITY, "mlp_forward: activation buffer too small");
    return launch_mlp_forward(X, B, params, wbf16, y, acts, as_stream(stream));
}

polymh_status polymh_mlp_backward(const uint16_t *X, int64_t B, const float *params,
                                  const uint16_t *wbf16, void *acts, size_t acts_bytes,
                                  const float *label, float *grad, float *loss, void *scratch,
                                  size_t scratch_bytes, void *stream)
{
    polymh_status st = check_batch(B, "mlp_backward");
    if (st) return st;
    if (B == 0) return POLYMH_OK;
    if (!X || !params || !wbf16 || !acts || !label || !grad || !loss || !scratch)
        return set_error(POLYMH_EINVAL, "mlp_backward: NULL array");
    if (acts_bytes < mlp_acts_bytes_aligned(B) || scratch_bytes < mlp_backward_scratch_bytes(B))
        return set_error(POLYMH_ECAPACITY, "mlp_backward: buffer too small");
    return launch_mlp_backward(X, B, params, wbf16, acts, label, grad, loss, scratch, as_stream(stream));
}

polymh_status polymh_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step,
                              float lr, float beta1, float beta2, float eps, uint16_t *wbf16,
                              void *stream)
{
    if (!params || !grad || !m || !v || !wbf16) return set_error(POLYMH_EINVAL, "mlp_adam: NULL array");
    if (step < 1) return set_error(POLYMH_EINVAL, "mlp_adam: step counts from 1");
    return launch_mlp_adam(params, grad, m, v, step, lr, beta1, beta2, eps, wbf16, as_stream(stream));
}

polymh_status polymh_gemm_bf16(const uint16_t *A, int64_t a_row_stride, int64_t a_k_stride,
                               const uint16_t *B, int64_t b_col_stride, int64_t b_k_stride, int64_t M,
                               int64_t N, int64_t K, float *C, void *stream)
{
    if (M < 0 || N < 0 || K < 0 || M % 32 || N % 32 || K % 16)
        return set_error(POLYMH_EINVAL, "gemm_bf16: M, N multiples of 32 and K of 16 required");
    if (M == 0 || N == 0) return POLYMH_OK;
    if (!A || !B || !C) return set_error(POLYMH_EINVAL, "gemm_bf16: NULL array");
    return launch_gemm_bf16(A, a_row_stride, a_k_stride, B, b_col_stride, b_k_stride, M, N, K, C,
                            as_stream(stream));
}

polymh_status polymh_poly_features(const polymh_polys *polys, polymh_box box, float *feats, void *stream)
{
    polymh_status st = check_polys(polys, "poly_features");
    if (st) return st;
    if ((st = check_box(box, "poly_features"))) return st;
    if (polys->n > 0 && !feats) return set_error(POLYMH_EINVAL, "poly_features: feats is NULL");
    return launch_poly_features(polys, box, feats, as_stream(stream));
}

polymh_status polymh_pair_features(const uint32_t *lsig, const float *lfeat, const uint32_t *rsig,
                                   const float *rfeat, int32_t k, const int32_t *li,
                                   const int32_t *ri, int64_t R, int64_t R_pad, uint16_t *X,
                                   void *stream)
{
    if (k != 256) return set_error(POLYMH_EINVAL, "pair_features: the scorer takes k = 256 signatures");
    if (R < 0 || R_pad < R) return set_error(POLYMH_EINVAL, "pair_features: bad row counts");
    if (R_pad == 0) return POLYMH_OK;
    if (!X || (R > 0 && (!lsig || !lfeat || !rsig || !rfeat || !li || !ri)))
        return set_error(POLYMH_EINVAL, "pair_features: NULL array");
    return launch_pair_features(lsig, lfeat, rsig, rfeat, li, ri, R, R_pad, X, as_stream(stream));
}

polymh_status polymh_csr_rows(const int64_t *cand_off, int64_t nq, int32_t *rows, void *stream)
{
    if (nq < 0) return set_error(POLYMH_EINVAL, "csr_rows: negative count");
    if (nq == 0) return POLYMH_OK;
    if (!cand_off || !rows) return set_error(POLYMH_EINVAL, "csr_rows: NULL array");
    return launch_csr_rows(cand_off, nq, rows, as_stream(stream));
}

polymh_status polymh_jhat(const uint32_t *lsig, const uint32_t *rsig, int32_t k, const int32_t *li,
                          const int32_t *ri, int64_t R, float *out, void *stream)
{
    if (k < 1 || R < 0) return set_error(POLYMH_EINVAL, "jhat: bad sizes");
    if (R == 0) return POLYMH_OK;
    if (!lsig || !rsig || !li || !ri || !out) return set_error(POLYMH_EINVAL, "jhat: NULL array");
    return launch_jhat(lsig, rsig, li, ri, R, k, out, as_stream(stream));
}

polymh_status polymh_rank_head(const int64_t *cand_off, const int32_t *cand_ids, int64_t nq,
                               const float *score, int32_t M, int32_t *order, uint8_t *sorted_ok,
                               int64_t *head_off, int32_t *head_query, int64_t *head_cand,
                               int32_t *head_id, void *stream)
{
    if (nq < 0 || M < 1) return set_error(POLYMH_EINVAL, "rank_head: bad sizes");
    if (nq == 0) return POLYMH_OK;
    if (!cand_off || !cand_ids || !score || !order || !sorted_ok || !head_off || !head_query ||
        !head_cand || !head_id)
        return set_error(POLYMH_EINVAL, "rank_head: NULL array");
    hipStream_t s = as_stream(stream);
    polymh_status st = launch_rank_sort(cand_off, nq, score, order, sorted_ok, s);
    if (st) return st;
    return launch_head_select(cand_off, cand_ids, nq, order, M, head_off, head_query, head_cand,
                              head_id, s);
}

polymh_status polymh_scatter_scores(const int64_t *idx, const float *val, int64_t n, float *score,
                                    void *stream)
{
    if (n < 0) return set_error(POLYMH_EINVAL, "scatter_scores: negative count");
    if (n == 0) return POLYMH_OK;
    if (!idx || !val || !score) return set_error(POLYMH_EINVAL, "scatter_scores: NULL array");
    return launch_scatter_scores(idx, val, n, score, as_stream(stream));
}

struct RankWs {
    int32_t *order;
    uint8_t *sorted_ok, *active;
    int64_t *cursor, *roff;
    int32_t *rids, *rpos, *n_active;
    double *rj;
    unsigned long long *counters;
    char *refine_ws;      // the refinement's own workspace (pairs beyond 512 edges deferred)
};

// A round lists at most nq * F pairs; the finishing pass up to every
// candidate, so the round lists hold max(nq * F, n_cand) entries.
static RankWs carve_rank(Carve &c, int64_t nq, int64_t n_cand, int32_t F)
{
    RankWs w{};
    w.order = c.take<int32_t>((size_t)(n_cand > 0 ? n_cand : 1));
    w.sorted_ok = c.take<uint8_t>((size_t)nq + 1);
    w.active = c.take<uint8_t>((size_t)nq + 1);
    w.cursor = c.take<int64_t>((size_t)nq + 1);
    w.roff = c.take<int64_t>((size_t)nq + 1);
    const size_t per_round = std::max((size_t)nq * (size_t)F, (size_t)n_cand) + 1;
    w.rids = c.take<int32_t>(per_round);
    w.rpos = c.take<int32_t>(per_round);
    w.rj = c.take<double>(per_round);
    w.n_active = c.take<int32_t>(1);
    w.counters = c.take<unsigned long long>(2);
    w.refine_ws = c.take<char>(refine_workspace_bytes());
    return w;
}

size_t polymh_rank_workspace_size(int64_t nq, int64_t n_cand, int32_t F)
{
    if (nq < 0 || n_cand < 0 || F < 1) return 0;
    Carve cv{nullptr, 0};
    carve_rank(cv, nq, n_cand, F);
    return align_up(cv.used, 256);
}

namespace {

__global__ void k_zero_counters(unsigned long long *c)
{
    if (threadIdx.x < 2) c[threadIdx.x] = 0;
}

__global__ void k_copy_counters(const unsigned long long *c, int64_t *out)
{
    if (threadIdx.x < 2) out[threadIdx.x] = (int64_t)c[threadIdx.x];
}

// One round: per-query counts (F <= 0: everything left), their offsets, the
// round's pair list, its exact J and the merge into the running top-k.
polymh_status rank_round(const polymh_polys *data, const polymh_polys *queries, const int64_t *cand_off,
                         const int32_t *cand_ids, const float *score, int64_t nq, int32_t topk, int32_t F,
                         float margin, const RankWs &w, int32_t *top_ids, double *top_j, bool with_n_active,
                         bool finishing, hipStream_t s)
{
    polymh_status st;
    if ((st = launch_round_offsets(cand_off, nq, w.cursor, w.active, finishing ? 0 : F, w.roff, s))) return st;
    if ((st = launch_round_fill(cand_off, cand_ids, w.order, w.cursor, w.roff, nq, w.rids, w.rpos, s))) return st;
    // the pair count lives on the device: the refinement's grid is sized by
    // the round's bound (F per query; one workgroup per query for the
    // finishing pass), and workgroups of queries without pairs return at once
    const int64_t hint = finishing ? nq : nq * (int64_t)F;
    if ((st = launch_refine(data, queries, w.roff, w.rids, nq, hint, w.rj, s, nullptr, w.refine_ws,
                            refine_workspace_bytes())))
        return st;
    return launch_round_merge(cand_off, score, w.order, w.sorted_ok, w.roff, w.rids, w.rj, nq, topk,
                              finishing ? INFINITY : margin, w.cursor, w.active, top_ids, top_j,
                              with_n_active ? w.n_active : nullptr, w.counters, finishing ? 1 : 0, s);
}

polymh_status check_rank_args(const polymh_polys *data, const polymh_polys *queries, int64_t nq, int64_t n_cand,
                              int32_t topk, int32_t F, const char *who)
{
    polymh_status st = check_polys(data, who);
    if (st) return st;
    if ((st = check_polys(queries, who))) return st;
    if (nq != queries->n) return set_error(POLYMH_EINVAL, "%s: nq differs from the query count", who);
    if (topk < 1 || topk > 64 || F < 1 || n_cand < 0) return set_error(POLYMH_EINVAL, "%s: bad sizes", who);
    return POLYMH_OK;
}

}  // namespace

polymh_status polymh_rank_refine(const polymh_polys *data, const polymh_polys *queries,
                                 const int64_t *cand_off, const int32_t *cand_ids, const float *score,
                                 int64_t nq, int64_t n_cand, int32_t topk, int32_t F, float margin,
                                 int32_t max_rounds, void *ws, size_t ws_bytes, int32_t *top_ids,
                                 double *top_j, int64_t *n_refined_host, int32_t *rounds_host,
                                 void *stream)
{
    polymh_status st = check_rank_args(data, queries, nq, n_cand, topk, F, "rank_refine");
    if (st) return st;
    if (max_rounds < 1) return set_error(POLYMH_EINVAL, "rank_refine: bad sizes");
    if (nq == 0) return POLYMH_OK;
    if (!cand_off || !top_ids || !top_j || (n_cand > 0 && (!cand_ids || !score)))
        return set_error(POLYMH_EINVAL, "rank_refine: NULL array");
    Carve cv{static_cast<char *>(ws), ws_bytes};
    RankWs w = carve_rank(cv, nq, n_cand, F);
    if (!cv.ok)
        return set_error(POLYMH_ECAPACITY, "rank_refine: workspace of %zu bytes, need %zu", ws_bytes, cv.used);
    hipStream_t s = as_stream(stream);
    if ((st = launch_rank_sort(cand_off, nq, score, w.order, w.sorted_ok, s))) return st;
    if ((st = launch_rank_init(nq, topk, w.cursor, w.active, top_ids, top_j, s))) return st;
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, w.counters);
    int32_t r = 0;
    bool done = false;
    for (; r < max_rounds; r++) {
        if ((st = rank_round(data, queries, cand_off, cand_ids, score, nq, topk, F, margin, w, top_ids, top_j, true,
                             false, s)))
            return st;
        int32_t still = 0;
        hipError_t e = hipMemcpyAsync(&still, w.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return set_error(POLYMH_EDEVICE, "rank_refine: %s", hipGetErrorString(e));
        if (still == 0) {
            done = true;
            r++;
            break;
        }
    }
    // rounds exhausted with queries still active: their remaining candidates
    // are refined in full, so the top-k is always complete
    if (!done && (st = rank_round(data, queries, cand_off, cand_ids, score, nq, topk, F, margin, w, top_ids,
                                  top_j, false, true, s)))
        return st;
    if (n_refined_host) {
        unsigned long long c[2] = {0, 0};
        hipError_t e = hipMemcpyAsync(c, w.counters, sizeof(c), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return set_error(POLYMH_EDEVICE, "rank_refine: %s", hipGetErrorString(e));
        *n_refined_host = (int64_t)c[0];
    }
    if (rounds_host) *rounds_host = r;
    return POLYMH_OK;
}

polymh_status polymh_rank_jhat_order(const uint32_t *qsig, const uint32_t *dsig, int32_t k, const int64_t *cand_off,
                                     const int32_t *cand_ids, int64_t nq, float *score, int32_t *order,
                                     uint8_t *sorted_ok, void *stream)
{
    if (nq < 0 || k < 1) return set_error(POLYMH_EINVAL, "rank_jhat_order: bad sizes");
    if (nq == 0) return POLYMH_OK;
    if (!qsig || !dsig || !cand_off || !cand_ids || !score || !order || !sorted_ok)
        return set_error(POLYMH_EINVAL, "rank_jhat_order: NULL array");
    return launch_rank_jhat_sort(qsig, dsig, k, cand_off, cand_ids, nq, score, order, sorted_ok, as_stream(stream));
}

size_t polymh_sig_pack_stride(int32_t k)
{
    return (k >= 4 && k <= 256 && k % 4 == 0) ? (size_t)k * 2 : 0;
}

polymh_status polymh_sig_pack(const uint32_t *sig, int64_t n, int32_t k, void *packed, void *stream)
{
    if (n < 0 || polymh_sig_pack_stride(k) == 0) return set_error(POLYMH_EINVAL, "sig_pack: bad sizes");
    if (n == 0) return POLYMH_OK;
    if (!sig || !packed) return set_error(POLYMH_EINVAL, "sig_pack: NULL array");
    if ((reinterpret_cast<uintptr_t>(sig) & 15) || (reinterpret_cast<uintptr_t>(packed) & 7))
        return set_error(POLYMH_EINVAL, "sig_pack: misaligned array");
    return launch_sig_pack(sig, n, k, static_cast<uint16_t *>(packed), as_stream(stream));
}

polymh_status polymh_rank_jhat_order_packed(const uint32_t *qsig, const void *packed, const uint32_t *dsig,
                                            int32_t k, const int64_t *cand_off, const int32_t *cand_ids,
                                            int64_t nq, float *score, int32_t *order, uint8_t *sorted_ok,
                                            void *stream)
{
    if (nq < 0 || polymh_sig_pack_stride(k) == 0) return set_error(POLYMH_EINVAL, "rank_jhat_order_packed: bad sizes");
    if (nq == 0) return POLYMH_OK;
    if (!qsig || !packed || !dsig || !cand_off || !cand_ids || !score || !order || !sorted_ok)
        return set_error(POLYMH_EINVAL, "rank_jhat_order_packed: NULL array");
    if ((reinterpret_cast<uintptr_t>(qsig) & 15) || (reinterpret_cast<uintptr_t>(dsig) & 15) ||
        (reinterpret_cast<uintptr_t>(packed) & 7))
        return set_error(POLYMH_EINVAL, "rank_jhat_order_packed: misaligned array");
    return launch_rank_jhat_packed(qsig, static_cast<const uint16_t *>(packed), dsig, k, cand_off, cand_ids, nq,
                                   score, order, sorted_ok, as_stream(stream));
}

polymh_status polymh_rank_order(const int64_t *cand_off, int64_t nq, const float *score, int32_t *order,
                                uint8_t *sorted_ok, void *stream)
{
    if (nq < 0) return set_error(POLYMH_EINVAL, "rank_order: bad sizes");
    if (nq == 0) return POLYMH_OK;
    if (!cand_off || !score || !order || !sorted_ok) return set_error(POLYMH_EINVAL, "rank_order: NULL array");
    return launch_rank_sort(cand_off, nq, score, order, sorted_ok, as_stream(stream));
}

polymh_status polymh_rank_head_fixed(const int64_t *cand_off, const int32_t *cand_ids, int64_t nq,
                                     const int32_t *order, int32_t M, int32_t *head_query, int64_t *head_cand,
                                     int32_t *head_id, void *stream)
{
    if (nq < 0 || M < 1) return set_error(POLYMH_EINVAL, "rank_head_fixed: bad sizes");
    if (nq == 0) return POLYMH_OK;
    if (!cand_off || !cand_ids || !order || !head_query || !head_cand || !head_id)
        return set_error(POLYMH_EINVAL, "rank_head_fixed: NULL array");
    return launch_head_fixed(cand_off, cand_ids, nq, order, M, head_query, head_cand, head_id, as_stream(stream));
}

polymh_status polymh_rank_reorder_head(const int64_t *cand_off, int64_t nq, const float *score,
                                      const int32_t *order_in, int32_t M, const uint8_t *sorted_ok,
                                      int32_t *order_out, void *stream)
{
    if (nq < 0 || M < 1 || M > 64) return set_error(POLYMH_EINVAL, "rank_reorder_head: bad sizes (1 <= M <= 64)");
    if (nq == 0) return POLYMH_OK;
    if (!cand_off || !score || !order_in || !sorted_ok || !order_out)
        return set_error(POLYMH_EINVAL, "rank_reorder_head: NULL array");
    if (order_in == order_out) return set_error(POLYMH_EINVAL, "rank_reorder_head: order_out aliases order_in");
    return launch_reorder_head(cand_off, nq, score, order_in, M, sorted_ok, order_out, as_stream(stream));
}

polymh_status polymh_mlp_score_pairs(const uint32_t *lsig, const float *lfeat, const uint32_t *rsig,
                                     const float *rfeat, int32_t k, const int32_t *li, const int32_t *ri,
                                     const int64_t *out_idx, int64_t R, const float *params, const uint16_t *wbf16,
                                     float *out, void *stream)
{
    if (k != 256) return set_error(POLYMH_EINVAL, "mlp_score_pairs: the scorer takes k = 256 signatures");
    if (R < 0) return set_error(POLYMH_EINVAL, "mlp_score_pairs: negative row count");
    if (R == 0) return POLYMH_OK;
    if (!lsig || !lfeat || !rsig || !rfeat || !li || !ri || !params || !wbf16 || !out)
        return set_error(POLYMH_EINVAL, "mlp_score_pairs: NULL array");
    if ((reinterpret_cast<uintptr_t>(lsig) | reinterpret_cast<uintptr_t>(rsig) | reinterpret_cast<uintptr_t>(wbf16)) & 15)
        return set_error(POLYMH_EINVAL, "mlp_score_pairs: signatures and weights must be 16-byte aligned");
    return launch_score_pairs(lsig, lfeat, rsig, rfeat, li, ri, out_idx, R, params, wbf16, out, as_stream(stream));
}

polymh_status polymh_rank_refine_ordered(const polymh_polys *data, const polymh_polys *queries,
                                         const int64_t *cand_off, const int32_t *cand_ids, const float *score,
                                         const int32_t *order, const uint8_t *sorted_ok, int64_t nq,
                                         int64_t n_cand, int32_t topk, int32_t F, int32_t rounds, float margin,
                                         void *ws, size_t ws_bytes, int32_t *top_ids, double *top_j,
                                         int64_t *counts, void *stream)
{
    polymh_status st = check_rank_args(data, queries, nq, n_cand, topk, F, "rank_refine_ordered");
    if (st) return st;
    if (rounds < 0) return set_error(POLYMH_EINVAL, "rank_refine_ordered: bad sizes");
    if (nq == 0) return POLYMH_OK;
    if (!cand_off || !top_ids || !top_j || !order || !sorted_ok || (n_cand > 0 && (!cand_ids || !score)))
        return set_error(POLYMH_EINVAL, "rank_refine_ordered: NULL array");
    Carve cv{static_cast<char *>(ws), ws_bytes};
    RankWs w = carve_rank(cv, nq, n_cand, F);
    if (!cv.ok)
        return set_error(POLYMH_ECAPACITY, "rank_refine_ordered: workspace of %zu bytes, need %zu", ws_bytes,
                         cv.used);
    hipStream_t s = as_stream(stream);
    // the caller's order is used as given: point the workspace at it
    w.order = const_cast<int32_t *>(order);
    w.sorted_ok = const_cast<uint8_t *>(sorted_ok);
    if ((st = launch_rank_init(nq, topk, w.cursor, w.active, top_ids, top_j, s))) return st;
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, w.counters);
    // rounds 0 and 1 take up to F candidates of each active query, round
    // r >= 2 up to F * 2^(r-1): after r rounds a query has visited F * 2^(r-1)
    // of its list, so a few rounds reach deep while the first stay fine-grained
    for (int32_t r = 0; r < rounds; r++) {
        const int sh = r < 2 ? 0 : std::min(r - 1, 20);
        const int64_t Fr = std::min<int64_t>((int64_t)F << sh, (int64_t)1 << 20);
        if ((st = rank_round(data, queries, cand_off, cand_ids, score, nq, topk, (int32_t)Fr, margin, w, top_ids,
                             top_j, false, false, s)))
            return st;
    }
    if ((st = rank_round(data, queries, cand_off, cand_ids, score, nq, topk, F, margin, w, top_ids, top_j, false,
                         true, s)))
        return st;
    if (counts) hipLaunchKernelGGL(k_copy_counters, dim3(1), dim3(64), 0, s, w.counters, counts);
    return check_launch("rank_refine_ordered");
}

}  // extern "C"
