// C ABI of libqs: argument validation (always before anything is enqueued),
// handle and buffer management, and the dispatch of each entry point to its
// kernels. Every computation on the state runs in the library's HIP kernels.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>
#include <numeric>

#include "qs_internal.h"

namespace qs {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";

int fail(int status, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return status;
}

void clear_error() { g_err[0] = 0; }

int hip_fail(hipError_t e, const char *what)
{
    const int st = (e == hipErrorOutOfMemory) ? QS_ENOMEM : QS_EDEVICE;
    return fail(st, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Staging ring
// ---------------------------------------------------------------------------
int Staging::init(size_t bytes)
{
    cap = bytes;
    head = 0;
    QS_HIP(hipHostMalloc(reinterpret_cast<void **>(&host), bytes, hipHostMallocDefault));
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&dev), bytes);
    if (e != hipSuccess) {
        (void)hipHostFree(host);
        host = nullptr;
        return hip_fail(e, "hipMalloc(staging)");
    }
    return QS_OK;
}

void Staging::release()
{
    if (host) (void)hipHostFree(host);
    if (dev) (void)hipFree(dev);
    host = dev = nullptr;
}

int Staging::reserve(hipStream_t s, size_t bytes, void **dptr)
{
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes > cap) return fail(QS_EUNSUPPORTED, "staging request of %zu bytes too large", bytes);
    if (head + bytes > cap) {
        // wrapping: make sure no queued copy still reads the pinned ring
        QS_HIP(hipStreamSynchronize(s));
        head = 0;
    }
    *dptr = dev + head;
    head += bytes;
    return QS_OK;
}

int Staging::put(hipStream_t s, const void *src, size_t bytes, void **dptr)
{
    const size_t off0 = head;
    if (int rc = reserve(s, bytes, dptr)) return rc;
    const size_t off = size_t(static_cast<char *>(*dptr) - dev);
    (void)off0;
    std::memcpy(host + off, src, bytes);
    QS_HIP(hipMemcpyAsync(*dptr, host + off, bytes, hipMemcpyHostToDevice, s));
    return QS_OK;
}

// ---------------------------------------------------------------------------
// Handle buffers
// ---------------------------------------------------------------------------
int ensure_partials(qs_state *h, size_t count)
{
    if (h->partials_cap >= count) return QS_OK;
    if (h->partials) {
        QS_HIP(hipStreamSynchronize(h->stream));
        (void)hipFree(h->partials);
        h->partials = nullptr;
        h->partials_cap = 0;
    }
    const size_t c = std::max(count, size_t(1) << 14);
    QS_HIP(hipMalloc(reinterpret_cast<void **>(&h->partials), c * sizeof(double)));
    h->partials_cap = c;
    return QS_OK;
}

int ensure_host_out(qs_state *h, size_t bytes)
{
    if (h->host_out_cap >= bytes) return QS_OK;
    if (h->host_out) {
        QS_HIP(hipStreamSynchronize(h->stream));
        (void)hipHostFree(h->host_out);
        h->host_out = nullptr;
        h->host_out_cap = 0;
    }
    const size_t b = std::max(bytes, size_t(1) << 16);
    QS_HIP(hipHostMalloc(reinterpret_cast<void **>(&h->host_out), b, hipHostMallocDefault));
    h->host_out_cap = b;
    return QS_OK;
}

int ensure_scratch(qs_state *h)
{
    if (h->scratch) return QS_OK;
    QS_HIP(hipMalloc(&h->scratch, h->dim() * h->amp_bytes()));
    return QS_OK;
}

}  // namespace qs

using namespace qs;

namespace {

int check_handle(qs_handle h)
{
    if (!h) return fail(QS_EINVAL, "NULL handle");
    return QS_OK;
}

int validate_gate(const qs_state *h, int k, const int *targets, const double *matrix,
                  uint64_t ctrl_mask, uint64_t ctrl_vals, GateDesc &d)
{
    if (k < 1 || k > QS_MAX_K) return fail(QS_EINVAL, "gate width k=%d outside [1, %d]", k, QS_MAX_K);
    if (!targets || !matrix) return fail(QS_EINVAL, "NULL targets or matrix");
    if (k > h->n) return fail(QS_EINVAL, "gate width %d exceeds %d qubits", k, h->n);
    uint64_t tm = 0;
    for (int m = 0; m < k; ++m) {
        const int t = targets[m];
        if (t < 0 || t >= h->n) return fail(QS_EINVAL, "target %d outside [0, %d)", t, h->n);
        if ((tm >> t) & 1) return fail(QS_EINVAL, "duplicate target %d", t);
        tm |= 1ull << t;
        d.targets[m] = t;
    }
    if (h->n < 64 && (ctrl_mask >> h->n)) return fail(QS_EINVAL, "control outside the state");
    if (ctrl_mask & tm) return fail(QS_EINVAL, "control qubit is also a target");
    if (ctrl_vals & ~ctrl_mask) return fail(QS_EINVAL, "ctrl_vals has bits outside ctrl_mask");
    const size_t cnt = size_t(2) << (2 * k);
    for (size_t i = 0; i < cnt; ++i)
        if (!std::isfinite(matrix[i])) return fail(QS_EINVAL, "matrix entry %zu is not finite", i);
    d.k = k;
    d.ctrl_mask = ctrl_mask;
    d.ctrl_vals = ctrl_vals;
    return QS_OK;
}

int validate_circuit(const qs_circuit *c, int n)
{
    if (!c) return fail(QS_EINVAL, "NULL circuit");
    if (c->n_gates < 0) return fail(QS_EINVAL, "negative gate count");
    if (c->n_gates == 0) return QS_OK;
    if (!c->k || !c->targets || !c->matrices) return fail(QS_EINVAL, "NULL circuit arrays");
    size_t toff = 0;
    for (int g = 0; g < c->n_gates; ++g) {
        const int k = c->k[g];
        if (k < 1 || k > QS_MAX_K) return fail(QS_EINVAL, "gate %d: width %d outside [1, %d]", g, k, QS_MAX_K);
        uint64_t tm = 0;
        for (int m = 0; m < k; ++m) {
            const int t = c->targets[toff + size_t(m)];
            if (t < 0 || t >= n) return fail(QS_EINVAL, "gate %d: target %d outside [0, %d)", g, t, n);
            if ((tm >> t) & 1) return fail(QS_EINVAL, "gate %d: duplicate target %d", g, t);
            tm |= 1ull << t;
        }
        const uint64_t cm = c->ctrl_mask ? c->ctrl_mask[g] : 0;
        const uint64_t cv = c->ctrl_vals ? c->ctrl_vals[g] : 0;
        if (n < 64 && (cm >> n)) return fail(QS_EINVAL, "gate %d: control outside the state", g);
        if (cm & tm) return fail(QS_EINVAL, "gate %d: control qubit is also a target", g);
        if (cv & ~cm) return fail(QS_EINVAL, "gate %d: ctrl_vals outside ctrl_mask", g);
        toff += size_t(k);
    }
    return QS_OK;
}

// Device-to-device state copy: one 16-byte streaming (nontemporal) load and
// store per thread, 1024-thread blocks in chunked XCD order (runs of 64
// blocks, 1 MiB per XCD), no grid-stride loop. On a 16 GiB state this runs
// at 6.6 TB/s; four loads per thread in 256-thread blocks reach 6.1, eight
// reach 4.3, and the runtime's copy 4.9.
typedef unsigned int U4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(1024) void k_copy16(const U4 *__restrict__ src, U4 *__restrict__ dst, uint64_t n16)
{
    const uint64_t i = xcd_order<uint64_t, 64>(blockIdx.x, gridDim.x) * 1024 + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Blocks [b0, b1) of a compiled program: dense blocks sweep the whole state,
// diagonal blocks only the amplitudes whose entry is not one.
int run_blocks(qs_state *h, const qs_program_t *p, int b0, int b1)
{
    for (int b = b0; b < b1; ++b) {
        GateDesc d;
        d.k = p->k[size_t(b)];
        for (int m = 0; m < d.k; ++m) d.targets[m] = p->qubits[size_t(b)][size_t(m)];
        const void *dm = (h->dtype == QS_C128)
                             ? static_cast<const void *>(p->dmats + p->mat_off[size_t(b)])
                             : static_cast<const void *>(p->dmats32 + p->mat_off[size_t(b)]);
        int rc;
        if (p->diagonal[size_t(b)]) {
            d.cls = GC_DIAG;
            rc = launch_diag_block(h, d, dm, 1 << d.k, p->hdiag[size_t(b)].data());
        } else {
            d.cls = GC_DENSE;
            rc = launch_dense(h, d, dm);
        }
        if (rc) return rc;
    }
    return QS_OK;
}

}  // namespace

extern "C" {

const char *qs_last_error(void) { return g_err; }

int qs_version(void) { return 10000; }

int qs_alloc(int n_qubits, int dtype, void *device_buf, void *hip_stream, qs_handle *out)
{
    clear_error();
    if (!out) return fail(QS_EINVAL, "NULL output handle");
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > QS_MAX_QUBITS)
        return fail(QS_EINVAL, "n_qubits=%d outside [1, %d]", n_qubits, QS_MAX_QUBITS);
    if (dtype != QS_C64 && dtype != QS_C128) return fail(QS_EINVAL, "unknown dtype %d", dtype);
    if (device_buf && (reinterpret_cast<uintptr_t>(device_buf) & 255))
        return fail(QS_EINVAL, "device buffer not 256-byte aligned");
    qs_state *h = new (std::nothrow) qs_state();
    if (!h) return fail(QS_ENOMEM, "host allocation failed");
    h->n = n_qubits;
    h->dtype = dtype;
    h->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(QS_EDEVICE, "no HIP device");
    }
    if (int rc = h->stage.init(size_t(8) << 20)) {
        delete h;
        return rc;
    }
    if (device_buf) {
        h->psi = device_buf;
        h->borrowed = true;
    } else {
        hipError_t e = hipMalloc(&h->psi, h->dim() * h->amp_bytes());
        if (e != hipSuccess) {
            h->stage.release();
            delete h;
            return hip_fail(e, "hipMalloc(state)");
        }
        if (int rc = launch_set_basis(h, 0)) {
            (void)hipFree(h->psi);
            h->stage.release();
            delete h;
            return rc;
        }
    }
    *out = h;
    return QS_OK;
}

int qs_free(qs_handle h)
{
    clear_error();
    if (!h) return QS_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    // the library owns psi unless it was borrowed, and always owns scratch
    // (library-owned states swap the two after out-of-place passes)
    if (!h->borrowed && h->psi) (void)hipFree(h->psi);
    if (h->scratch) (void)hipFree(h->scratch);
    if (h->partials) (void)hipFree(h->partials);
    if (h->fft_roots) (void)hipFree(h->fft_roots);
    if (h->host_out) (void)hipHostFree(h->host_out);
    h->stage.release();
    delete h;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return QS_OK;
}

int qs_info(qs_handle h, int *n_qubits, int *dtype, void **device_ptr)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (n_qubits) *n_qubits = h->n;
    if (dtype) *dtype = h->dtype;
    if (device_ptr) *device_ptr = h->psi;
    return QS_OK;
}

int qs_set_zero(qs_handle h)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    return launch_set_basis(h, 0);
}

int qs_get_state(qs_handle h, void *host_dst)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!host_dst) return fail(QS_EINVAL, "NULL host buffer");
    QS_HIP(hipMemcpyAsync(host_dst, h->psi, h->dim() * h->amp_bytes(), hipMemcpyDeviceToHost,
                          h->stream));
    QS_HIP(hipStreamSynchronize(h->stream));
    return QS_OK;
}

int qs_set_state(qs_handle h, const void *host_src)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!host_src) return fail(QS_EINVAL, "NULL host buffer");
    QS_HIP(hipMemcpyAsync(h->psi, host_src, h->dim() * h->amp_bytes(), hipMemcpyHostToDevice,
                          h->stream));
    QS_HIP(hipStreamSynchronize(h->stream));
    return QS_OK;
}

int qs_load_device(qs_handle h, const void *device_src)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!device_src) return fail(QS_EINVAL, "NULL device source");
    const size_t bytes = h->dim() * h->amp_bytes();
    const char *s = static_cast<const char *>(device_src), *d = static_cast<const char *>(h->psi);
    if (s < d + bytes && d < s + bytes) return fail(QS_EINVAL, "source overlaps the state");
    const uint64_t n16 = bytes / 16;
    if (bytes % 16 == 0 && ((reinterpret_cast<uintptr_t>(s) | reinterpret_cast<uintptr_t>(d)) & 15) == 0 &&
        (n16 + 1023) / 1024 <= 0x7fffffffull) {
        hipLaunchKernelGGL(k_copy16, dim3(unsigned((n16 + 1023) / 1024)), dim3(1024), 0, h->stream,
                           reinterpret_cast<const U4 *>(s), reinterpret_cast<U4 *>(h->psi), n16);
        QS_HIP(hipGetLastError());
    } else {
        QS_HIP(hipMemcpyAsync(h->psi, device_src, bytes, hipMemcpyDeviceToDevice, h->stream));
    }
    return QS_OK;
}

int qs_get_amplitudes(qs_handle h, int count, const uint64_t *indices, void *host_dst)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (count < 0 || count > (1 << 16)) return fail(QS_EINVAL, "count=%d outside [0, 65536]", count);
    if (count == 0) return QS_OK;
    if (!indices || !host_dst) return fail(QS_EINVAL, "NULL indices or output");
    for (int i = 0; i < count; ++i)
        if (indices[i] >= h->dim()) return fail(QS_EINVAL, "index %d outside the state", i);
    return gather_amplitudes(h, count, indices, host_dst);
}

int qs_sync(qs_handle h)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    QS_HIP(hipStreamSynchronize(h->stream));
    QS_HIP(hipGetLastError());
    return QS_OK;
}

int qs_apply_gate(qs_handle h, int k, const int *targets, const double *matrix, uint64_t ctrl_mask,
                  uint64_t ctrl_vals)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    GateDesc d;
    if (int rc = validate_gate(h, k, targets, matrix, ctrl_mask, ctrl_vals, d)) return rc;
    return enqueue_gate(h, d, matrix);
}

int qs_apply_fused(qs_handle h, int n_blocks, const int *k_per_block, const int *targets_concat,
                   const double *matrices_concat)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (n_blocks < 0) return fail(QS_EINVAL, "negative block count");
    if (n_blocks == 0) return QS_OK;
    if (!k_per_block || !targets_concat || !matrices_concat) return fail(QS_EINVAL, "NULL block arrays");
    std::vector<GateDesc> ds(static_cast<size_t>(n_blocks));
    size_t toff = 0, moff = 0;
    std::vector<size_t> moffs(static_cast<size_t>(n_blocks));
    for (int b = 0; b < n_blocks; ++b) {
        const int k = k_per_block[b];
        if (k < 1 || k > QS_MAX_K) return fail(QS_EINVAL, "block %d: width %d outside [1, %d]", b, k, QS_MAX_K);
        if (int rc = validate_gate(h, k, targets_concat + toff, matrices_concat + moff, 0, 0,
                                   ds[size_t(b)]))
            return fail(rc, "block %d: %s", b, qs_last_error());
        moffs[size_t(b)] = moff;
        toff += size_t(k);
        moff += size_t(2) << (2 * k);
    }
    for (int b = 0; b < n_blocks; ++b)
        if (int rc = enqueue_gate(h, ds[size_t(b)], matrices_concat + moffs[size_t(b)])) return rc;
    return QS_OK;
}

int qs_plan_fusion(const qs_circuit *c, int n_qubits, int max_k, int *n_blocks, int *block_of_gate,
                   int *block_k, int *block_qubits)
{
    clear_error();
    if (n_qubits < 1 || n_qubits > 63) return fail(QS_EINVAL, "n_qubits=%d outside [1, 63]", n_qubits);
    if (max_k < 1 || max_k > QS_MAX_K) return fail(QS_EINVAL, "max_k=%d outside [1, %d]", max_k, QS_MAX_K);
    if (int rc = validate_circuit(c, n_qubits)) return rc;
    if (!n_blocks || (c->n_gates && (!block_of_gate || !block_k || !block_qubits)))
        return fail(QS_EINVAL, "NULL output arrays");
    Plan p;
    if (int rc = plan_fusion(n_qubits, c->n_gates, c->k, c->targets, c->ctrl_mask, max_k, p, far_qubit(16)))
        return rc;
    *n_blocks = int(p.block_gates.size());
    for (int g = 0; g < c->n_gates; ++g) block_of_gate[g] = p.block_of_gate[size_t(g)];
    for (size_t b = 0; b < p.block_gates.size(); ++b) {
        const auto &q = p.block_qubits[b];
        block_k[b] = int(q.size());
        for (int i = 0; i < QS_MAX_K; ++i)
            block_qubits[b * QS_MAX_K + size_t(i)] = i < int(q.size()) ? q[size_t(i)] : -1;
    }
    return QS_OK;
}

int qs_compile(qs_handle h, const qs_circuit *c, int max_k, qs_program *out)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!out) return fail(QS_EINVAL, "NULL output program");
    *out = nullptr;
    if (max_k < 1 || max_k > QS_MAX_K) return fail(QS_EINVAL, "max_k=%d outside [1, %d]", max_k, QS_MAX_K);
    if (int rc = validate_circuit(c, h->n)) return rc;
    for (int g = 0; g < c->n_gates; ++g) {
        const uint64_t cm = c->ctrl_mask ? c->ctrl_mask[g] : 0;
        if (c->k[g] + __builtin_popcountll(cm) > QS_MAX_K)
            return fail(QS_EUNSUPPORTED, "gate %d spans more than %d qubits with its controls", g, QS_MAX_K);
    }
    Plan p;
    if (int rc = plan_fusion(h->n, c->n_gates, c->k, c->targets, c->ctrl_mask, max_k, p, far_qubit(h->amp_bytes())))
        return rc;
    qs_program_t *pr = new (std::nothrow) qs_program_t();
    if (!pr) return fail(QS_ENOMEM, "host allocation failed");
    pr->n = h->n;
    pr->device = h->device;
    pr->n_blocks = int(p.block_gates.size());
    // host-side descriptors
    std::vector<size_t> toff(size_t(c->n_gates) + 1, 0), moff(size_t(c->n_gates) + 1, 0);
    for (int g = 0; g < c->n_gates; ++g) {
        toff[size_t(g) + 1] = toff[size_t(g)] + size_t(c->k[g]);
        moff[size_t(g) + 1] = moff[size_t(g)] + (size_t(2) << (2 * c->k[g]));
    }
    std::vector<ComposeGate> cg;
    std::vector<ComposeBlock> cb;
    std::vector<double> gm;
    int kmax = 1;
    int64_t out_off = 0;
    for (int b = 0; b < pr->n_blocks; ++b) {
        const auto &qs = p.block_qubits[size_t(b)];
        const int kb = int(qs.size());
        kmax = std::max(kmax, kb);
        auto local = [&](int q) { return int(std::lower_bound(qs.begin(), qs.end(), q) - qs.begin()); };
        ComposeBlock B;
        B.k = kb;
        B.g0 = int(cg.size());
        bool diag = true;
        for (int g : p.block_gates[size_t(b)]) {
            ComposeGate G;
            std::memset(&G, 0, sizeof G);
            G.k = c->k[g];
            for (int m = 0; m < G.k; ++m) G.local_t[m] = local(c->targets[toff[size_t(g)] + size_t(m)]);
            const uint64_t cm = c->ctrl_mask ? c->ctrl_mask[g] : 0;
            const uint64_t cv = c->ctrl_vals ? c->ctrl_vals[g] : 0;
            for (int q = 0; q < 64; ++q)
                if ((cm >> q) & 1) {
                    G.ctrl_mask |= 1u << local(q);
                    if ((cv >> q) & 1) G.ctrl_vals |= 1u << local(q);
                }
            G.mat_off = int64_t(gm.size());
            const double *src = c->matrices + moff[size_t(g)];
            const size_t cnt = size_t(2) << (2 * G.k);
            gm.insert(gm.end(), src, src + cnt);
            GateDesc tmp;
            classify(src, G.k, tmp);
            if (!(tmp.cls == GC_IDENTITY || tmp.cls == GC_PHASE1 || tmp.cls == GC_DIAG)) diag = false;
            cg.push_back(G);
        }
        B.g1 = int(cg.size());
        B.pad = 0;
        B.out_off = out_off;
        cb.push_back(B);
        pr->k.push_back(kb);
        pr->qubits.push_back(qs);
        pr->diagonal.push_back(diag ? 1 : 0);
        pr->mat_off.push_back(out_off);
        out_off += int64_t(2) << (2 * kb);
    }
    pr->mats_doubles = size_t(out_off);
    int rc = QS_OK;
    void *dcg = nullptr, *dcb = nullptr, *dgm = nullptr;
    auto cleanup = [&]() {
        if (dcg) (void)hipFree(dcg);
        if (dcb) (void)hipFree(dcb);
        if (dgm) (void)hipFree(dgm);
    };
    auto bail = [&](int r) {
        cleanup();
        if (pr->dmats) (void)hipFree(pr->dmats);
        if (pr->dmats32) (void)hipFree(pr->dmats32);
        delete pr;
        return r;
    };
    if (pr->n_blocks > 0) {
        hipError_t e = hipSuccess;
        if ((e = hipMalloc(&dcg, sizeof(ComposeGate) * cg.size())) != hipSuccess ||
            (e = hipMalloc(&dcb, sizeof(ComposeBlock) * cb.size())) != hipSuccess ||
            (e = hipMalloc(&dgm, sizeof(double) * std::max<size_t>(gm.size(), 1))) != hipSuccess ||
            (e = hipMalloc(reinterpret_cast<void **>(&pr->dmats), sizeof(double) * pr->mats_doubles)) != hipSuccess ||
            (e = hipMalloc(reinterpret_cast<void **>(&pr->dmats32), sizeof(float) * pr->mats_doubles)) != hipSuccess)
            return bail(hip_fail(e, "hipMalloc(program)"));
        if ((e = hipMemcpyAsync(dcg, cg.data(), sizeof(ComposeGate) * cg.size(), hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(dcb, cb.data(), sizeof(ComposeBlock) * cb.size(), hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(dgm, gm.data(), sizeof(double) * gm.size(), hipMemcpyHostToDevice, h->stream)) != hipSuccess)
            return bail(hip_fail(e, "hipMemcpyAsync(program)"));
        if ((rc = launch_compose(h->stream, pr->n_blocks, static_cast<ComposeBlock *>(dcb),
                                 static_cast<ComposeGate *>(dcg), static_cast<double *>(dgm),
                                 pr->dmats, kmax)))
            return bail(rc);
        if ((rc = launch_cast_f64_to_f32(h->stream, pr->dmats, pr->dmats32, pr->mats_doubles)))
            return bail(rc);
        if ((e = hipStreamSynchronize(h->stream)) != hipSuccess)
            return bail(hip_fail(e, "compose"));
    }
    // Diagonal blocks keep their composed diagonal on the host: the run
    // sweeps only the amplitudes whose entry is not one.
    pr->hdiag.resize(size_t(pr->n_blocks));
    pr->changed.assign(size_t(pr->n_blocks), 1.0);
    for (int b = 0; b < pr->n_blocks; ++b) {
        if (!pr->diagonal[size_t(b)]) continue;
        const size_t D = size_t(1) << pr->k[size_t(b)];
        std::vector<double> full(2 * D * D);
        hipError_t e = hipMemcpy(full.data(), pr->dmats + pr->mat_off[size_t(b)], full.size() * sizeof(double),
                                 hipMemcpyDeviceToHost);
        if (e != hipSuccess) return bail(hip_fail(e, "hipMemcpy(diagonal block)"));
        auto &hd = pr->hdiag[size_t(b)];
        hd.resize(2 * D);
        for (size_t j = 0; j < D; ++j) {
            hd[2 * j] = full[2 * (j * D + j)];
            hd[2 * j + 1] = full[2 * (j * D + j) + 1];
        }
        pr->changed[size_t(b)] = diag_changed_fraction(hd.data(), pr->k[size_t(b)]);
    }
    cleanup();
    *out = pr;
    return QS_OK;
}

int qs_program_info(qs_program p, int *n_blocks, int *block_k, double *amp_moves_per_run)
{
    clear_error();
    if (!p) return fail(QS_EINVAL, "NULL program");
    if (n_blocks) *n_blocks = p->n_blocks;
    if (block_k)
        for (int b = 0; b < p->n_blocks; ++b) block_k[b] = p->k[size_t(b)];
    if (amp_moves_per_run) {
        // dense blocks read and write every amplitude; diagonal blocks only
        // the ones whose entry is not one
        double f = 0.0;
        for (int b = 0; b < p->n_blocks; ++b) f += p->changed[size_t(b)];
        *amp_moves_per_run = f * 2.0 * std::ldexp(1.0, p->n);
    }
    return QS_OK;
}

int qs_program_block_kind(qs_program p, int b, int *kind, double *changed_fraction)
{
    clear_error();
    if (!p) return fail(QS_EINVAL, "NULL program");
    if (b < 0 || b >= p->n_blocks) return fail(QS_EINVAL, "block %d outside [0, %d)", b, p->n_blocks);
    const double f = p->changed[size_t(b)];
    if (kind) *kind = !p->diagonal[size_t(b)] ? QS_BLOCK_DENSE : (f == 0.0 ? QS_BLOCK_IDENTITY : QS_BLOCK_DIAGONAL);
    if (changed_fraction) *changed_fraction = f;
    return QS_OK;
}

int qs_run_program_range(qs_handle h, qs_program p, int b0, int b1)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!p) return fail(QS_EINVAL, "NULL program");
    if (p->n != h->n) return fail(QS_EINVAL, "program built for %d qubits, state has %d", p->n, h->n);
    if (b0 < 0 || b1 < b0 || b1 > p->n_blocks)
        return fail(QS_EINVAL, "block range [%d, %d) outside [0, %d]", b0, b1, p->n_blocks);
    return run_blocks(h, p, b0, b1);
}

int qs_program_block(qs_program p, int b, double *matrix_out, int *qubits_out)
{
    clear_error();
    if (!p) return fail(QS_EINVAL, "NULL program");
    if (b < 0 || b >= p->n_blocks) return fail(QS_EINVAL, "block %d outside [0, %d)", b, p->n_blocks);
    const size_t cnt = size_t(2) << (2 * p->k[size_t(b)]);
    if (matrix_out) {
        QS_HIP(hipDeviceSynchronize());
        QS_HIP(hipMemcpy(matrix_out, p->dmats + p->mat_off[size_t(b)], cnt * sizeof(double),
                         hipMemcpyDeviceToHost));
    }
    if (qubits_out)
        for (size_t i = 0; i < p->qubits[size_t(b)].size(); ++i) qubits_out[i] = p->qubits[size_t(b)][i];
    return QS_OK;
}

int qs_run_program(qs_handle h, qs_program p)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!p) return fail(QS_EINVAL, "NULL program");
    if (p->n != h->n) return fail(QS_EINVAL, "program built for %d qubits, state has %d", p->n, h->n);
    return run_blocks(h, p, 0, p->n_blocks);
}

int qs_program_free(qs_program p)
{
    clear_error();
    if (!p) return QS_OK;
    if (p->dmats || p->dmats32) (void)hipDeviceSynchronize();
    if (p->dmats) (void)hipFree(p->dmats);
    if (p->dmats32) (void)hipFree(p->dmats32);
    delete p;
    return QS_OK;
}

int qs_apply_circuit(qs_handle h, const qs_circuit *c, int max_k)
{
    qs_program p = nullptr;
    if (int rc = qs_compile(h, c, max_k, &p)) return rc;
    int rc = qs_run_program(h, p);
    qs_program_free(p);
    return rc;
}

int qs_norm2(qs_handle h, double *out)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!out) return fail(QS_EINVAL, "NULL output");
    return reduce_norm2(h, out);
}

int qs_expectation(qs_handle h, uint64_t x_mask, uint64_t y_mask, uint64_t z_mask, double *out_re,
                   double *out_im)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!out_re || !out_im) return fail(QS_EINVAL, "NULL output");
    if ((x_mask & y_mask) || (x_mask & z_mask) || (y_mask & z_mask))
        return fail(QS_EINVAL, "Pauli masks overlap");
    if (h->n < 64 && ((x_mask | y_mask | z_mask) >> h->n)) return fail(QS_EINVAL, "Pauli mask outside the state");
    return reduce_pauli(h, x_mask, y_mask, z_mask, out_re, out_im);
}

int qs_expectation_noalloc(qs_handle h, uint64_t x_mask, uint64_t y_mask, uint64_t z_mask, double *device_out)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!device_out) return fail(QS_EINVAL, "NULL device output");
    if ((x_mask & y_mask) || (x_mask & z_mask) || (y_mask & z_mask))
        return fail(QS_EINVAL, "Pauli masks overlap");
    if (h->n < 64 && ((x_mask | y_mask | z_mask) >> h->n)) return fail(QS_EINVAL, "Pauli mask outside the state");
    return reduce_pauli_noalloc(h, x_mask, y_mask, z_mask, device_out);
}

int qs_measure(qs_handle h, int m, const int *qubits, int shots, const double *uniforms,
               uint64_t *outcomes, double *probs_or_null, int collapse)
{
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (m < 1 || m > 20 || m > h->n) return fail(QS_EINVAL, "m=%d outside [1, min(20, n)]", m);
    if (!qubits) return fail(QS_EINVAL, "NULL qubit list");
    uint64_t seen = 0;
    for (int r = 0; r < m; ++r) {
        if (qubits[r] < 0 || qubits[r] >= h->n) return fail(QS_EINVAL, "qubit %d outside the state", qubits[r]);
        if ((seen >> qubits[r]) & 1) return fail(QS_EINVAL, "duplicate qubit %d", qubits[r]);
        seen |= 1ull << qubits[r];
    }
    if (shots < 0) return fail(QS_EINVAL, "negative shot count");
    if (shots > 0 && (!uniforms || !outcomes)) return fail(QS_EINVAL, "NULL uniforms or outcomes");
    for (int s = 0; s < shots; ++s)
        if (!(uniforms[s] >= 0.0 && uniforms[s] < 1.0)) return fail(QS_EINVAL, "uniform %d outside [0, 1)", s);
    if (collapse && shots < 1) return fail(QS_EINVAL, "collapse needs at least one shot");
    if (size_t(shots) * sizeof(double) > (size_t(4) << 20)) return fail(QS_EINVAL, "too many shots");
    return measure(h, m, qubits, shots, uniforms, outcomes, probs_or_null, collapse);
}

}  // extern "C"
