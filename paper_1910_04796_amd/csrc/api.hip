// api.hip -- the C-ABI: handles, validation, options, device memory pool.
//
// Validation of every argument happens on the host before any HIP call, so
// malformed input is rejected even on a machine without a GPU.
#include <algorithm>
#include <cstdarg>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <unordered_map>

#include "internal.h"

namespace bsmm {

// ------------------------------------------------------------------ errors
static thread_local std::string t_msg;
static thread_local int t_code = BSMM_OK;

void set_error(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_msg = buf;
    t_code = code;
}
void clear_error() {
    t_msg.clear();
    t_code = BSMM_OK;
}
int last_code() { return t_code; }

int launch_check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(BSMM_EDEVICE, "kernel launch '%s' failed: %s", what, hipGetErrorString(e));
        return BSMM_EDEVICE;
    }
    return BSMM_OK;
}

Options &options() {
    static Options o;
    return o;
}

uint64_t next_version() {
    static std::atomic<uint64_t> v{1};
    return v.fetch_add(1);
}

// ------------------------------------------------------------------- pool
namespace {
struct Provider {
    bsmm_alloc_fn alloc = nullptr;
    bsmm_dealloc_fn dealloc = nullptr;
    void *ctx = nullptr;
};
struct Block {
    void *p;
    size_t bytes;
    hipStream_t s;
    Provider prov;
};
std::mutex g_mu;
std::multimap<size_t, Block> g_free;
std::unordered_map<void *, Block> g_used;
Provider g_prov;

void *raw_alloc(size_t bytes, hipStream_t s) {
    if (g_prov.alloc) return g_prov.alloc(bytes, (void *)s, g_prov.ctx);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}
void raw_free(const Block &b) {
    if (b.prov.alloc) {
        if (b.prov.dealloc) b.prov.dealloc(b.p, b.bytes, (void *)b.s, b.prov.ctx);
    } else {
        (void)hipFree(b.p);
    }
}
size_t round_size(size_t n) {
    if (n <= 4096) return (n + 255) & ~size_t(255);
    size_t p = size_t(1) << (63 - __builtin_clzll(n));  // highest power of two <= n
    size_t step = std::max<size_t>(p / 8, 4096);
    return (n + step - 1) / step * step;
}
void release_free_locked() {
    if (g_free.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto &kv : g_free) raw_free(kv.second);
    g_free.clear();
}
}  // namespace

void *dev_alloc(size_t bytes, hipStream_t s) {
    size_t want = round_size(bytes ? bytes : 1);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_free.lower_bound(want);
    if (it != g_free.end() && it->first <= want + want / 2 + 4096) {
        Block b = it->second;
        g_free.erase(it);
        if (b.s != s) (void)hipStreamSynchronize(b.s);
        b.s = s;
        g_used[b.p] = b;
        return b.p;
    }
    void *p = raw_alloc(want, s);
    if (!p) {
        release_free_locked();
        p = raw_alloc(want, s);
    }
    if (!p) return nullptr;
    g_used[p] = Block{p, want, s, g_prov};
    return p;
}

void dev_free(void *p, hipStream_t s) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_used.find(p);
    if (it == g_used.end()) return;
    Block b = it->second;
    g_used.erase(it);
    b.s = s;
    g_free.emplace(b.bytes, b);
}

int pool_release_all() {
    std::lock_guard<std::mutex> lk(g_mu);
    release_free_locked();
    return BSMM_OK;
}

static int set_provider(bsmm_alloc_fn a, bsmm_dealloc_fn d, void *ctx) {
    std::lock_guard<std::mutex> lk(g_mu);
    release_free_locked();
    g_prov.alloc = a;
    g_prov.dealloc = a ? d : nullptr;
    g_prov.ctx = a ? ctx : nullptr;
    return BSMM_OK;
}

// ------------------------------------------------------------- validation
// Pure host checks of a block-CSR description; no HIP call.
static int validate_sizes(const char *what, int32_t nb, const int32_t *sizes) {
    if (nb < 0) {
        set_error(BSMM_EINVAL, "%s: negative block count %d", what, nb);
        return BSMM_EINVAL;
    }
    if (nb > 0 && !sizes) {
        set_error(BSMM_EINVAL, "%s: block sizes pointer is NULL", what);
        return BSMM_EINVAL;
    }
    for (int32_t i = 0; i < nb; ++i)
        if (sizes[i] < 1) {
            set_error(BSMM_EINVAL, "%s: block size %d at index %d is < 1", what, sizes[i], i);
            return BSMM_EINVAL;
        }
    return BSMM_OK;
}

static int validate_pattern(int32_t nbr, int32_t nbc, int64_t nnzb, const int64_t *rp,
                            const int32_t *ci) {
    if (nnzb < 0) {
        set_error(BSMM_EINVAL, "negative block count nnzb=%lld", (long long)nnzb);
        return BSMM_EINVAL;
    }
    if (!rp) {
        set_error(BSMM_EINVAL, "blk_row_ptr is NULL");
        return BSMM_EINVAL;
    }
    if (nnzb > 0 && !ci) {
        set_error(BSMM_EINVAL, "blk_col_ind is NULL");
        return BSMM_EINVAL;
    }
    if (nnzb > (int64_t)INT32_MAX) {
        set_error(BSMM_ERANGE, "too many blocks (%lld)", (long long)nnzb);
        return BSMM_ERANGE;
    }
    if (rp[0] != 0 || rp[nbr] != nnzb) {
        set_error(BSMM_EINDEX, "blk_row_ptr must start at 0 and end at nnzb");
        return BSMM_EINDEX;
    }
    for (int32_t i = 0; i < nbr; ++i) {
        if (rp[i + 1] < rp[i]) {
            set_error(BSMM_EINDEX, "blk_row_ptr decreases at row %d", i);
            return BSMM_EINDEX;
        }
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= nbc) {
                set_error(BSMM_EINDEX, "column index %d out of range at row %d", ci[p], i);
                return BSMM_EINDEX;
            }
            if (p > rp[i] && ci[p] <= ci[p - 1]) {
                set_error(BSMM_EINDEX, "columns not strictly ascending at row %d", i);
                return BSMM_EINDEX;
            }
        }
    }
    return BSMM_OK;
}

static thread_local bsmm_multiply_stats t_stats;
bsmm_multiply_stats &stats() { return t_stats; }

static thread_local ScratchArena *t_arena = nullptr;
ScratchArena *&scratch_arena() { return t_arena; }

// Every device buffer of a matrix belongs to the stream that last used it.
// Before work on stream s touches the matrix, s waits for the work queued
// on the buffers' current streams, and the buffers pass to s: a buffer
// released later (replaced by a grown or filtered pattern, or destroyed)
// returns to the pool under the last stream that used it, so the pool never
// hands it out while that work may still run.
int adopt_stream(bsmm_matrix_s *M, hipStream_t s) {
    DevBuf *bufs[] = {&M->b_rbs, &M->b_cbs, &M->b_row_off, &M->b_col_off, &M->b_row_map,
                      &M->b_col_map, &M->b_row_ptr, &M->b_col_ind, &M->b_blk_off, &M->b_data};
    std::vector<hipStream_t> waited;
    for (DevBuf *b : bufs) {
        if (!b->p || b->s == s) continue;
        if (std::find(waited.begin(), waited.end(), b->s) == waited.end()) {
            hipEvent_t ev;
            BSMM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            const hipError_t e1 = hipEventRecord(ev, b->s);
            const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(s, ev, 0) : e1;
            (void)hipEventDestroy(ev);
            if (e2 != hipSuccess) {
                set_error(BSMM_EDEVICE, "stream hand-over failed: %s", hipGetErrorString(e2));
                return BSMM_EDEVICE;
            }
            waited.push_back(b->s);
        }
        b->s = s;
    }
    return BSMM_OK;
}

}  // namespace bsmm

using namespace bsmm;

// ------------------------------------------------------------------- C-ABI
extern "C" int bsmm_create_matrix_typed(int32_t nbr, const int32_t *row_blk_sizes, int32_t nbc,
                                        const int32_t *col_blk_sizes, int64_t nnzb,
                                        const int64_t *blk_row_ptr, const int32_t *blk_col_ind,
                                        int32_t dtype, const void *data, int data_on_device,
                                        void *stream, bsmm_matrix *out) {
    clear_error();
    if (!out) {
        set_error(BSMM_EINVAL, "out is NULL");
        return BSMM_EINVAL;
    }
    if (dtype != BSMM_F64 && dtype != BSMM_F32) {
        set_error(BSMM_EINVAL, "unknown element type %d", dtype);
        return BSMM_EINVAL;
    }
    const size_t esize = dtype == BSMM_F32 ? sizeof(float) : sizeof(double);
    BSMM_TRY(validate_sizes("row_blk_sizes", nbr, row_blk_sizes));
    BSMM_TRY(validate_sizes("col_blk_sizes", nbc, col_blk_sizes));
    BSMM_TRY(validate_pattern(nbr, nbc, nnzb, blk_row_ptr, blk_col_ind));

    // Host-side offsets.
    std::vector<int64_t> row_off(nbr + 1, 0), col_off(nbc + 1, 0), blk_off(nnzb + 1, 0);
    for (int32_t i = 0; i < nbr; ++i) row_off[i + 1] = row_off[i] + row_blk_sizes[i];
    for (int32_t j = 0; j < nbc; ++j) col_off[j + 1] = col_off[j] + col_blk_sizes[j];
    int64_t acc = 0;
    for (int32_t i = 0; i < nbr; ++i)
        for (int64_t p = blk_row_ptr[i]; p < blk_row_ptr[i + 1]; ++p) {
            blk_off[p] = acc;
            acc += (int64_t)row_blk_sizes[i] * col_blk_sizes[blk_col_ind[p]];
            if (acc >= (int64_t(1) << 47)) {
                set_error(BSMM_ERANGE, "matrix holds 2^47 or more elements");
                return BSMM_ERANGE;
            }
        }
    blk_off[nnzb] = acc;
    if (row_off[nbr] > INT32_MAX || col_off[nbc] > INT32_MAX) {
        set_error(BSMM_ERANGE, "matrix dimension exceeds 2^31-1 rows or columns");
        return BSMM_ERANGE;
    }

    hipStream_t s = (hipStream_t)stream;
    auto *M = new (std::nothrow) bsmm_matrix_s();
    if (!M) {
        set_error(BSMM_ENOMEM, "host allocation failed");
        return BSMM_ENOMEM;
    }
    M->nbr = nbr;
    M->nbc = nbc;
    M->dtype = dtype;
    M->rbs.assign(row_blk_sizes, row_blk_sizes + nbr);
    M->cbs.assign(col_blk_sizes, col_blk_sizes + nbc);
    M->row_off = row_off;
    M->col_off = col_off;
    M->nnzb = nnzb;
    M->nelems = acc;
    M->storage = acc;
    M->max_rbs = nbr ? *std::max_element(M->rbs.begin(), M->rbs.end()) : 0;
    M->max_cbs = nbc ? *std::max_element(M->cbs.begin(), M->cbs.end()) : 0;
    M->last_stream = s;
    M->version = next_version();
    {
        int ndev = 0;
        hipError_t e1 = hipGetDeviceCount(&ndev);
        hipError_t e2 = e1 == hipSuccess && ndev > 0 ? hipGetDevice(&M->device) : e1;
        if (e1 != hipSuccess || ndev <= 0 || e2 != hipSuccess) {
            (void)hipGetLastError();
            delete M;
            set_error(BSMM_EDEVICE, "no HIP device available (%s, %d devices, %s)",
                      hipGetErrorString(e1), ndev, hipGetErrorString(e2));
            return BSMM_EDEVICE;
        }
    }

    std::vector<int2> rmap(row_off[nbr]), cmap(col_off[nbc]);
    for (int32_t i = 0; i < nbr; ++i)
        for (int32_t r = 0; r < row_blk_sizes[i]; ++r) rmap[row_off[i] + r] = make_int2(i, r);
    for (int32_t j = 0; j < nbc; ++j)
        for (int32_t c = 0; c < col_blk_sizes[j]; ++c) cmap[col_off[j] + c] = make_int2(j, c);

    auto fail = [&](int code) {
        delete M;
        return code;
    };
    int st = BSMM_OK;
    if ((st = M->b_rbs.reserve(sizeof(int32_t) * (nbr + 1), s)) ||
        (st = M->b_cbs.reserve(sizeof(int32_t) * (nbc + 1), s)) ||
        (st = M->b_row_off.reserve(sizeof(int64_t) * (nbr + 1), s)) ||
        (st = M->b_col_off.reserve(sizeof(int64_t) * (nbc + 1), s)) ||
        (st = M->b_row_map.reserve(sizeof(int2) * (rmap.size() + 1), s)) ||
        (st = M->b_col_map.reserve(sizeof(int2) * (cmap.size() + 1), s)) ||
        (st = M->b_row_ptr.reserve(sizeof(int64_t) * (nbr + 1), s)) ||
        (st = M->b_col_ind.reserve(sizeof(int32_t) * (nnzb + 1), s)) ||
        (st = M->b_blk_off.reserve(sizeof(int64_t) * (nnzb + 1), s)) ||
        (st = M->b_data.reserve(esize * (acc + 1), s)))
        return fail(st);

#define CP(dst, src, bytes)                                                                  \
    do {                                                                                     \
        if ((bytes) > 0) {                                                                   \
            hipError_t e_ = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);       \
            if (e_ != hipSuccess) {                                                          \
                set_error(BSMM_EDEVICE, "upload failed: %s", hipGetErrorString(e_));         \
                return fail(BSMM_EDEVICE);                                                   \
            }                                                                                \
        }                                                                                    \
    } while (0)
    CP(M->d_rbs(), row_blk_sizes, sizeof(int32_t) * nbr);
    CP(M->d_cbs(), col_blk_sizes, sizeof(int32_t) * nbc);
    CP(M->d_row_off(), row_off.data(), sizeof(int64_t) * (nbr + 1));
    CP(M->d_col_off(), col_off.data(), sizeof(int64_t) * (nbc + 1));
    CP(M->d_row_map(), rmap.data(), sizeof(int2) * rmap.size());
    CP(M->d_col_map(), cmap.data(), sizeof(int2) * cmap.size());
    CP(M->d_row_ptr(), blk_row_ptr, sizeof(int64_t) * (nbr + 1));
    CP(M->d_col_ind(), blk_col_ind, sizeof(int32_t) * nnzb);
    CP(M->d_blk_off(), blk_off.data(), sizeof(int64_t) * (nnzb + 1));
#undef CP
    if (acc > 0) {
        hipError_t e;
        if (data)
            e = hipMemcpyAsync(M->d_raw(), data, esize * acc,
                               data_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
        else
            e = (hipError_t)(fill_zero_bytes(M->d_raw(), esize * acc, s) == BSMM_OK ? hipSuccess
                                                                                   : hipErrorUnknown);
        if (e != hipSuccess) {
            set_error(BSMM_EDEVICE, "data upload failed: %s", hipGetErrorString(e));
            return fail(BSMM_EDEVICE);
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
        set_error(BSMM_EDEVICE, "stream synchronisation failed");
        return fail(BSMM_EDEVICE);
    }
    *out = M;
    return BSMM_OK;
}

extern "C" int bsmm_create_matrix(int32_t nbr, const int32_t *row_blk_sizes, int32_t nbc,
                                  const int32_t *col_blk_sizes, int64_t nnzb,
                                  const int64_t *blk_row_ptr, const int32_t *blk_col_ind,
                                  const double *data, int data_on_device, void *stream,
                                  bsmm_matrix *out) {
    return bsmm_create_matrix_typed(nbr, row_blk_sizes, nbc, col_blk_sizes, nnzb, blk_row_ptr,
                                    blk_col_ind, BSMM_F64, data, data_on_device, stream, out);
}

extern "C" int bsmm_matrix_dtype(bsmm_matrix m, int32_t *dtype) {
    clear_error();
    if (!m || !dtype) {
        set_error(BSMM_EINVAL, "matrix or output is NULL");
        return BSMM_EINVAL;
    }
    *dtype = m->dtype;
    return BSMM_OK;
}

extern "C" int bsmm_destroy_matrix(bsmm_matrix m) {
    clear_error();
    if (!m) return BSMM_OK;
    (void)hipStreamSynchronize(m->last_stream);
    delete m;
    return BSMM_OK;
}

extern "C" int bsmm_matrix_info(bsmm_matrix m, int32_t *nbr, int32_t *nbc, int64_t *nnzb,
                                int64_t *nelems) {
    clear_error();
    if (!m) {
        set_error(BSMM_EINVAL, "matrix is NULL");
        return BSMM_EINVAL;
    }
    if (nbr) *nbr = m->nbr;
    if (nbc) *nbc = m->nbc;
    if (nnzb) *nnzb = m->nnzb;
    if (nelems) *nelems = m->nelems;
    return BSMM_OK;
}

extern "C" int bsmm_copy_out_typed(bsmm_matrix m, int64_t *blk_row_ptr, int32_t *blk_col_ind,
                                   void *data, int data_on_device, void *stream) {
    clear_error();
    if (!m) {
        set_error(BSMM_EINVAL, "matrix is NULL");
        return BSMM_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    BSMM_TRY(adopt_stream(m, s));
    if (blk_row_ptr)
        BSMM_HIP(hipMemcpyAsync(blk_row_ptr, m->d_row_ptr(), sizeof(int64_t) * (m->nbr + 1),
                                hipMemcpyDeviceToHost, s));
    if (blk_col_ind && m->nnzb > 0)
        BSMM_HIP(hipMemcpyAsync(blk_col_ind, m->d_col_ind(), sizeof(int32_t) * m->nnzb,
                                hipMemcpyDeviceToHost, s));
    DevBuf packed, packed_off;
    if (data && m->nelems > 0 && m->holes) {
        // Storage with gaps left by a filter: the blocks are gathered into
        // packed CSR order (straight into a device destination).
        BSMM_TRY(packed_off.reserve(sizeof(int64_t) * (m->nnzb + 1), s));
        BSMM_TRY(build_block_offsets(m->d_rbs(), m->d_cbs(), m->nbr, m->d_row_ptr(), m->d_col_ind(),
                                     m->nnzb, packed_off.as<int64_t>(), nullptr, s));
        void *dst = data;
        if (!data_on_device) {
            BSMM_TRY(packed.reserve(m->esize() * m->nelems, s));
            dst = packed.p;
        }
        BSMM_TRY(relayout(m, m->d_row_ptr(), m->d_col_ind(), packed_off.as<int64_t>(), dst, s));
        if (!data_on_device)
            BSMM_HIP(hipMemcpyAsync(data, packed.p, m->esize() * m->nelems, hipMemcpyDeviceToHost, s));
    } else if (data && m->nelems > 0) {
        BSMM_HIP(hipMemcpyAsync(data, m->d_raw(), m->esize() * m->nelems,
                                data_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    }
    BSMM_HIP(hipStreamSynchronize(s));
    m->last_stream = s;
    return BSMM_OK;
}

extern "C" int bsmm_copy_out(bsmm_matrix m, int64_t *blk_row_ptr, int32_t *blk_col_ind,
                             double *data, int data_on_device, void *stream) {
    clear_error();
    if (m && m->dtype != BSMM_F64) {
        set_error(BSMM_EINVAL, "matrix holds FP32 data (bsmm_copy_out_typed copies it)");
        return BSMM_EINVAL;
    }
    return bsmm_copy_out_typed(m, blk_row_ptr, blk_col_ind, data, data_on_device, stream);
}

extern "C" int bsmm_set_allocator(bsmm_alloc_fn alloc, bsmm_dealloc_fn dealloc, void *ctx) {
    clear_error();
    if (alloc && !dealloc) {
        set_error(BSMM_EINVAL, "an allocator needs a matching deallocator");
        return BSMM_EINVAL;
    }
    return set_provider(alloc, dealloc, ctx);
}

extern "C" int bsmm_set_option(const char *key, const char *value) {
    clear_error();
    if (!key || !value) {
        set_error(BSMM_EINVAL, "key or value is NULL");
        return BSMM_EINVAL;
    }
    Options &o = options();
    std::string k(key), v(value);
    if (k == "path") {
        if (v == "auto") o.path = 0;
        else if (v == "stack") o.path = 1;
        else if (v == "dense") o.path = 2;
        else if (v == "emul") o.path = 3;
        else goto bad;
    } else if (k == "stack_kernel") {
        if (v == "plain") o.stack_kernel = 0;
        else if (v == "tuned") o.stack_kernel = 1;
        else goto bad;
    } else if (k == "stack_chunk") {
        char *end = nullptr;
        long long x = strtoll(value, &end, 10);
        if (!end || *end || x < 0) goto bad;
        o.stack_chunk = x;
    } else if (k == "stack_panel") {
        char *end = nullptr;
        long long x = strtoll(value, &end, 10);
        if (!end || *end || x < 0) goto bad;
        o.stack_panel = x;
    } else if (k == "stack_tile") {
        char *end = nullptr;
        long x = strtol(value, &end, 10);
        if (!end || *end || x < 0 || x > 65536) goto bad;
        o.stack_tile = (int)x;
    } else if (k == "jit") {
        if (v == "0") o.jit = 0;
        else if (v == "1") o.jit = 1;
        else goto bad;
    } else if (k == "stack_at") {
        if (v == "auto") o.stack_at = -1;
        else if (v == "0") o.stack_at = 0;
        else if (v == "1") o.stack_at = 1;
        else goto bad;
    } else if (k == "prescreen") {
        if (v == "0") o.prescreen = 0;
        else if (v == "1") o.prescreen = 1;
        else goto bad;
    } else if (k == "stack_sched") {
        if (v == "static") o.stack_sched = 0;
        else if (v == "dynamic") o.stack_sched = 1;
        else goto bad;
    } else if (k == "tune_db") {
        o.tune_db = v;
    } else if (k == "emul_slices") {
        char *end = nullptr;
        long x = strtol(value, &end, 10);
        if (!end || *end || x < 1 || x > 8) goto bad;
        o.emul_slices = (int)x;
    } else if (k == "stack_params") {
        int q[4] = {0, 0, 0, 0};
        if (!v.empty() && sscanf(value, "%d %d %d %d", &q[0], &q[1], &q[2], &q[3]) != 4) goto bad;
        if (!v.empty() && (q[0] < 1 || q[1] < 1 || q[2] < 0 || q[3] < 0 || q[3] > 4)) goto bad;
        for (int i = 0; i < 4; ++i) o.forced[i] = q[i];
    } else if (k == "mlp_weights") {
        o.mlp_weights = v;
    } else if (k == "dense_kb") {
        if (v == "16") o.dense_kb = 16;
        else if (v == "32") o.dense_kb = 32;
        else goto bad;
    } else if (k == "emul_kernel") {
        if (v == "t64") o.emul_kernel = 0;
        else if (v == "t128") o.emul_kernel = 1;
        else if (v == "t128k32") o.emul_kernel = 2;
        else if (v == "t128w8") o.emul_kernel = 3;
        else goto bad;
    } else if (k == "verbose") {
        if (v == "0") o.verbose = 0;
        else if (v == "1") o.verbose = 1;
        else goto bad;
    } else if (k == "plan_cache") {
        if (v == "0") o.plan_cache = 0;
        else if (v == "1") o.plan_cache = 1;
        else goto bad;
    } else if (k == "time_kernels") {
        if (v == "0") o.time_kernels = 0;
        else if (v == "1") o.time_kernels = 1;
        else goto bad;
    } else {
        set_error(BSMM_EINVAL, "unknown option '%s'", key);
        return BSMM_EINVAL;
    }
    return BSMM_OK;
bad:
    set_error(BSMM_EINVAL, "bad value '%s' for option '%s'", value, key);
    return BSMM_EINVAL;
}

extern "C" int bsmm_get_option(const char *key, char *buf, size_t len) {
    clear_error();
    if (!key || !buf || len == 0) {
        set_error(BSMM_EINVAL, "bad arguments");
        return BSMM_EINVAL;
    }
    Options &o = options();
    std::string k(key), v;
    if (k == "path") v = o.path == 0 ? "auto" : o.path == 1 ? "stack" : o.path == 2 ? "dense" : "emul";
    else if (k == "emul_slices") v = std::to_string(o.emul_slices);
    else if (k == "stack_kernel") v = o.stack_kernel ? "tuned" : "plain";
    else if (k == "stack_chunk") v = std::to_string(o.stack_chunk);
    else if (k == "stack_panel") v = std::to_string(o.stack_panel);
    else if (k == "stack_tile") v = std::to_string(o.stack_tile);
    else if (k == "stack_sched") v = o.stack_sched ? "dynamic" : "static";
    else if (k == "jit") v = std::to_string(o.jit);
    else if (k == "prescreen") v = std::to_string(o.prescreen);
    else if (k == "stack_at") v = o.stack_at < 0 ? "auto" : std::to_string(o.stack_at);
    else if (k == "tune_db") v = o.tune_db;
    else if (k == "time_kernels") v = std::to_string(o.time_kernels);
    else if (k == "verbose") v = std::to_string(o.verbose);
    else if (k == "plan_cache") v = std::to_string(o.plan_cache);
    else if (k == "dense_kb") v = std::to_string(o.dense_kb);
    else if (k == "emul_kernel") v = o.emul_kernel == 0   ? "t64"
                                        : o.emul_kernel == 1 ? "t128"
                                        : o.emul_kernel == 2 ? "t128k32"
                                                             : "t128w8";
    else if (k == "mlp_weights") v = o.mlp_weights;
    else if (k == "stack_params")
        v = o.forced[0] ? std::to_string(o.forced[0]) + " " + std::to_string(o.forced[1]) + " " +
                              std::to_string(o.forced[2]) + " " + std::to_string(o.forced[3])
                        : std::string();
    else {
        set_error(BSMM_EINVAL, "unknown option '%s'", key);
        return BSMM_EINVAL;
    }
    snprintf(buf, len, "%s", v.c_str());
    return BSMM_OK;
}

extern "C" const char *bsmm_last_error(void) { return bsmm::t_msg.c_str(); }

extern "C" int bsmm_last_stats(bsmm_multiply_stats *out) {
    if (!out) {
        set_error(BSMM_EINVAL, "out is NULL");
        return BSMM_EINVAL;
    }
    *out = bsmm::t_stats;
    return BSMM_OK;
}

// Shared by multiply.hip: argument checks of a multiply (host only).
namespace bsmm {
int validate_multiply(bsmm_matrix_s *A, bsmm_matrix_s *B, bsmm_matrix_s *C, double eps) {
    if (!A || !B || !C) {
        set_error(BSMM_EINVAL, "a matrix handle is NULL");
        return BSMM_EINVAL;
    }
    if (C == A || C == B) {
        set_error(BSMM_EINVAL, "C must not alias A or B");
        return BSMM_EINVAL;
    }
    if (A->dtype != C->dtype || B->dtype != C->dtype) {
        set_error(BSMM_EINVAL, "A, B and C hold different element types");
        return BSMM_EINVAL;
    }
    if (!(eps >= 0.0)) {
        set_error(BSMM_EINVAL, "filter_eps must be >= 0 and not NaN");
        return BSMM_EINVAL;
    }
    if (A->cbs != B->rbs) {
        set_error(BSMM_ESHAPE, "A block-column sizes differ from B block-row sizes");
        return BSMM_ESHAPE;
    }
    if (C->rbs != A->rbs || C->cbs != B->cbs) {
        set_error(BSMM_ESHAPE, "C block sizes differ from (A rows, B columns)");
        return BSMM_ESHAPE;
    }
    return BSMM_OK;
}
}  // namespace bsmm
