// Fiber scheduler of the host emulation declared in include/hip/hip_runtime.h.
#include <hip/hip_runtime.h>

#include <stdarg.h>

#include <map>
#include <random>

#include <sanitizer/common_interface_defs.h>

namespace emu {

BlockCtx *g_blk = nullptr;
Lane *g_lane = nullptr;
std::function<void()> *g_body = nullptr;

namespace {

constexpr size_t kStack = 512 * 1024;
constexpr int kWaveSize = 64;
void *g_sched_sp = nullptr;
void *g_sched_fake = nullptr;
const void *g_sched_stack_bottom = nullptr;
size_t g_sched_stack_size = 0;
std::vector<unsigned char *> g_stacks;  // reused between workgroups
std::mt19937_64 g_rng;
int g_order = 0;  // 0 forward, 1 reverse, 2 shuffled
bool g_order_read = false;
uint64_t g_blocks = 0;

void read_order()
{
    if (g_order_read) return;
    g_order_read = true;
    const char *e = getenv("EMU_ORDER");
    if (!e || !strcmp(e, "fwd")) return;
    if (!strcmp(e, "rev")) {
        g_order = 1;
        return;
    }
    g_order = 2;
    g_rng.seed(strtoull(e, nullptr, 10));
}

}  // namespace

void fail(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    fprintf(stderr, "emu: ");
    vfprintf(stderr, fmt, ap);
    if (g_blk)
        fprintf(stderr, " (block %u,%u,%u of %u,%u,%u, %u threads)", g_blk->bid.x, g_blk->bid.y, g_blk->bid.z,
                g_blk->gdim.x, g_blk->gdim.y, g_blk->gdim.z, g_blk->bdim.x);
    fprintf(stderr, "\n");
    va_end(ap);
    abort();
}

}  // namespace emu

// Context switch (System V x86-64): saves the callee-saved registers on the
// current stack, stores the stack pointer to *save and continues on `load`.
extern "C" void emu_ctx_switch(void **save, void *load);
asm(R"(
.text
.globl emu_ctx_switch
.type emu_ctx_switch,@function
emu_ctx_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
.size emu_ctx_switch, .-emu_ctx_switch
)");

namespace emu {

namespace {

void fiber_main()
{
    __sanitizer_finish_switch_fiber(nullptr, &g_sched_stack_bottom, &g_sched_stack_size);
    (*g_body)();
    g_lane->state = kDone;
    __sanitizer_start_switch_fiber(nullptr, g_sched_stack_bottom, g_sched_stack_size);
    void *dead;
    emu_ctx_switch(&dead, g_sched_sp);
    abort();  // never resumed
}

void init_fiber(Lane &L)
{
    unsigned char *top = L.stack + kStack;
    top = reinterpret_cast<unsigned char *>(reinterpret_cast<uintptr_t>(top) & ~uintptr_t(15));
    void **sp = reinterpret_cast<void **>(top);
    *--sp = nullptr;                                          // fake return address of fiber_main
    *--sp = reinterpret_cast<void *>(&fiber_main);            // popped by ret
    for (int r = 0; r < 6; ++r) *--sp = nullptr;              // rbp rbx r12 r13 r14 r15
    L.sp = sp;
}

void resume(Lane &L)
{
    g_lane = &L;
    __sanitizer_start_switch_fiber(&g_sched_fake, L.stack, kStack);
    emu_ctx_switch(&g_sched_sp, L.sp);
    __sanitizer_finish_switch_fiber(g_sched_fake, nullptr, nullptr);
    g_lane = nullptr;
}

// Resolves the wave operation that the waiting lanes of one wave share.
void resolve_wave(std::vector<Lane> &lanes, int w0, int w1)
{
    std::vector<int> at;
    for (int i = w0; i < w1; ++i)
        if (lanes[i].state == kWave) at.push_back(i);
    if (at.empty()) return;
    const int op = lanes[at[0]].op;
    for (int i : at)
        if (lanes[i].op != op) fail("lanes of one wave wait at different wave operations (%d, %d)", op, lanes[i].op);
    auto lane_of = [&](int l) -> Lane * {
        const int i = w0 + l;
        return i < w1 ? &lanes[i] : nullptr;
    };
    auto value_of = [&](int l, const char *what) -> uint64_t {
        Lane *L = lane_of(l);
        if (!L || L->state != kWave) fail("%s reads lane %d, which is not at the operation", what, l);
        return L->a;
    };
    uint64_t ballot = 0;
    for (int i : at)
        if (lanes[i].a) ballot |= uint64_t(1) << (i - w0);
    for (int i : at) {
        Lane &L = lanes[i];
        const int l = i - w0;
        switch (op) {
        case kSync: L.result = 0; break;
        case kBallot: L.result = ballot; break;
        case kShflXor: L.result = value_of(l ^ int(L.b), "shfl_xor"); break;
        case kShflIdx: L.result = value_of(int(L.b) & 63, "shfl"); break;
        case kShflUp: L.result = l >= int(L.b) ? value_of(l - int(L.b), "shfl_up") : L.a; break;
        case kReadlane: {
            for (int j : at)
                if (lanes[j].b != L.b) fail("readlane with a lane index that differs across lanes");
            L.result = value_of(int(L.b) & 63, "readlane");
            break;
        }
        case kRor1: L.result = value_of((l + 63) & 63, "row rotate"); break;
        case kReadFirst: L.result = lanes[at[0]].a; break;
        case kInvBallot: {
            for (int j : at)
                if (lanes[j].a != L.a) fail("inverse ballot of a mask that differs across lanes");
            L.result = (L.a >> l) & 1;
            break;
        }
        default: fail("unknown wave operation %d", op);
        }
    }
    for (int i : at) lanes[i].state = kRun;
}

}  // namespace

void yield_to_scheduler()
{
    Lane *L = g_lane;
    __sanitizer_start_switch_fiber(&L->fake, g_sched_stack_bottom, g_sched_stack_size);
    emu_ctx_switch(&L->sp, g_sched_sp);
    __sanitizer_finish_switch_fiber(L->fake, &g_sched_stack_bottom, &g_sched_stack_size);
    g_lane = L;
}

void run_grid(std::function<void()> body, dim3 grid, dim3 block, size_t dyn_lds)
{
    read_order();
    const int nthreads = int(block.x * block.y * block.z);
    if (nthreads < 1 || nthreads > 1024) fail("workgroup of %d threads", nthreads);
    if (block.y != 1 || block.z != 1) fail("only one-dimensional workgroups are emulated");
    while (int(g_stacks.size()) < nthreads) g_stacks.push_back(static_cast<unsigned char *>(malloc(kStack)));
    const int nwaves = (nthreads + kWaveSize - 1) / kWaveSize;
    for (unsigned bz = 0; bz < grid.z; ++bz)
        for (unsigned by = 0; by < grid.y; ++by)
            for (unsigned bx = 0; bx < grid.x; ++bx) {
                BlockCtx B;
                B.bid = dim3(bx, by, bz);
                B.bdim = block;
                B.gdim = grid;
                B.lds_bytes = dyn_lds;
                B.lds = dyn_lds ? static_cast<unsigned char *>(malloc(dyn_lds)) : nullptr;
                if (B.lds) memset(B.lds, 0xA5, dyn_lds);  // garbage, as LDS starts
                B.dma.resize(nwaves);
                B.lanes.resize(nthreads);
                for (int t = 0; t < nthreads; ++t) {
                    Lane &L = B.lanes[t];
                    L.tid = dim3(unsigned(t));
                    L.index = t;
                    L.stack = g_stacks[t];
                    init_fiber(L);
                }
                g_blk = &B;
                g_body = &body;
                std::vector<int> order(nwaves);
                for (int w = 0; w < nwaves; ++w) order[w] = g_order == 1 ? nwaves - 1 - w : w;
                for (;;) {
                    if (g_order == 2) std::shuffle(order.begin(), order.end(), g_rng);
                    for (int w : order) {
                        const int w0 = w * kWaveSize, w1 = std::min(nthreads, w0 + kWaveSize);
                        for (;;) {
                            for (int i = w0; i < w1; ++i)
                                if (B.lanes[i].state == kRun) resume(B.lanes[i]);
                            bool waiting = false;
                            for (int i = w0; i < w1; ++i) waiting |= B.lanes[i].state == kWave;
                            if (!waiting) break;
                            resolve_wave(B.lanes, w0, w1);
                        }
                    }
                    int live = 0, at_barrier = 0;
                    for (auto &L : B.lanes) {
                        live += L.state != kDone;
                        at_barrier += L.state == kBarrier;
                    }
                    if (live == 0) break;
                    if (at_barrier != live) fail("no progress: %d live threads, %d at a barrier", live, at_barrier);
                    B.barrier_or_result = B.barrier_or;
                    B.barrier_or = 0;
                    for (auto &L : B.lanes)
                        if (L.state == kBarrier) L.state = kRun;
                }
                for (auto &q : B.dma)
                    if (!q.empty()) fail("direct LDS loads never waited for");
                g_blk = nullptr;
                free(B.lds);
                ++g_blocks;
            }
}

}  // namespace emu

void emu_waitcnt_vmem(int keep)
{
    auto &q = ::emu::g_blk->dma[::emu::g_lane->index / 64];
    const int me = ::emu::g_lane->index;
    const uint64_t issued = ::emu::g_lane->dma_issued;
    size_t out = 0;
    for (size_t k = 0; k < q.size(); ++k) {
        const auto &d = q[k];
        if (d.lane == me && d.seq + uint64_t(keep) < issued)
            memcpy(d.dst, d.src, d.bytes);
        else
            q[out++] = d;
    }
    q.resize(out);
}

void emu_amdgcn_global_load_lds(const void *src, void *lds, int size, int offset, int aux)
{
    (void)aux;
    auto *B = ::emu::g_blk;
    unsigned char *dst = static_cast<unsigned char *>(lds) + offset + size_t(size) * (::emu::g_lane->index & 63);
    if (dst < B->lds || dst + size > B->lds + B->lds_bytes)
        ::emu::fail("direct LDS load of %d bytes at LDS offset %td, dynamic LDS is %zu bytes", size, dst - B->lds,
                    B->lds_bytes);
    volatile unsigned char probe = *static_cast<const volatile unsigned char *>(src);  // checked read
    (void)probe;
    ::emu::Lane *L = ::emu::g_lane;
    B->dma[L->index / 64].push_back({dst, static_cast<const unsigned char *>(src), size_t(size), L->index,
                                     L->dma_issued++});
}

namespace {
std::map<const void *, int> g_allowed;
}

void emu_allow_lds(const void *kernel, int bytes)
{
    if (bytes > 160 * 1024) ::emu::fail("dynamic LDS of %d bytes exceeds 160 KiB", bytes);
    g_allowed[kernel] = bytes;
}

void emu_check_lds(const void *kernel, size_t bytes)
{
    auto it = g_allowed.find(kernel);
    const size_t limit = it == g_allowed.end() ? 64 * 1024 : size_t(it->second);
    if (bytes > limit) ::emu::fail("launch with %zu bytes of dynamic LDS, %zu allowed", bytes, limit);
}

extern "C" {
void *emu_alloc(size_t bytes) { return malloc(bytes ? bytes : 1); }
void emu_free(void *p) { free(p); }
unsigned long long emu_blocks_run(void) { return ::emu::g_blocks; }
}
