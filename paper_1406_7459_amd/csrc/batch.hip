// batch.hip -- many independent grids of uneven sizes (for example the
// points of a field sweep) stepped together.  Every pass of every instance
// runs through the same kernel bodies as a single plan (demag_kernels.hpp,
// stage_body.hpp); a batched launch covers one pass kind for all instances
// that share the transform length of that pass, reading its workgroups'
// (instance, block) coordinates from a task table (column passes read it
// through the XCD mapping of layout.hpp, so neighbouring tasks share an
// L2).  A whole RK4 step is a
// fixed sequence of such launches and is captured once into a HIP graph.
//
// Two launch modes.  Merged: one launch per pass kind over every instance
// and every transform length (512 threads a workgroup for the row and
// column passes, 128 or 256 for the products), a task naming its instance,
// block and length; each length runs in the radix order of at most 12
// values per thread (order 1 for 3 2^a lengths; 5 2^a lengths take 20); the
// product passes take one launch per register class (the z products of at
// most 8 values per thread; the y products of nz = 1 instances and the
// 12-value z products; the products of 5 2^a lengths), so the many short z
// products of thin films are sized for neither the larger schedules'
// registers nor the long y products' LDS; tasks are ordered longest
// transform first.  At most 8 launches per stage, 7 without 5 2^a lengths.
// Grouped: one launch
// per (pass kind, transform length), each group with its own tuned tile in
// the default radix orders.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "demag_kernels.hpp"
#include "mm_internal.hpp"
#include "stage_body.hpp"

namespace mmk {

struct BInst {
    float *M;      // caller state (bound per call)
    float *Sa, *Sb, *H, *kacc;
    float *Hout;   // output of the inverse x pass: H for a step, caller H for mm_batch_demag
    float2 *X1, *X2;
    const float *Kt;
    const float2 *tw0, *tw1, *tw2;
    int nx, ny, nz, pad;
    int Lx, Ly, Lz;  // padded transform lengths (>= 2n; Lz = 1 when nz = 1)
    StageCoef c;
};

__device__ __forceinline__ float *bsel(const BInst &I, int s) { return s == 0 ? I.M : (s == 1 ? I.Sa : I.Sb); }

template <int L, int V>
__global__ __launch_bounds__(1024) void kb_xfwd(const BInst *__restrict__ B, const int4 *__restrict__ T, int sel,
                                                int lp2)
{
    const int4 t = T[blockIdx.x];
    const BInst &I = B[t.x];
    xfwd_body<L, V>(bsel(I, sel), I.X1, I.nz * I.ny, I.nx, lp2, I.tw0, t.y);
}
template <int L, int V>
__global__ __launch_bounds__(1024) void kb_yfwd(const BInst *__restrict__ B, const int4 *__restrict__ T, int lp2)
{
    const int4 t = T[xcd_block(blockIdx.x, gridDim.x)];
    const BInst &I = B[t.x];
    yfwd_body<L, V>(I.X1, I.X2, I.Lx / 2 + 1, I.ny, lp2, I.tw1, t.y, t.z);
}
template <int L, bool Z>
__global__ __launch_bounds__(conv_max_threads<L>()) void kb_reg3(const BInst *__restrict__ B,
                                                                  const int4 *__restrict__ T, int lp2)
{
    const int4 t = T[xcd_block(blockIdx.x, gridDim.x)];
    const BInst &I = B[t.x];
    conv_reg3_body<L, Z>(Z ? I.X2 : I.X1, I.Kt, I.Lx / 2 + 1, I.Ly / 2, Z ? I.nz : I.ny, lp2, Z ? I.tw2 : I.tw1, t.y,
                         t.z);
}
template <int L, int V, bool Z>
__global__ __launch_bounds__(1024) void kb_split(const BInst *__restrict__ B, const int4 *__restrict__ T, int lp2)
{
    const int4 t = T[xcd_block(blockIdx.x, gridDim.x)];
    const BInst &I = B[t.x];
    conv_split_body<L, V, Z>(Z ? I.X2 : I.X1, I.Kt, I.Lx / 2 + 1, I.Ly / 2, Z ? I.nz : I.ny, lp2, Z ? I.tw2 : I.tw1,
                             t.y, t.z);
}
template <int L, int V>
__global__ __launch_bounds__(1024) void kb_yinv(const BInst *__restrict__ B, const int4 *__restrict__ T, int lp2)
{
    const int4 t = T[xcd_block(blockIdx.x, gridDim.x)];
    const BInst &I = B[t.x];
    yinv_body<L, V>(I.X2, I.X1, I.Lx / 2 + 1, I.ny, lp2, I.tw1, t.y, t.z);
}
template <int L, int V>
__global__ __launch_bounds__(1024) void kb_xinv(const BInst *__restrict__ B, const int4 *__restrict__ T, int lp2)
{
    const int4 t = T[blockIdx.x];
    const BInst &I = B[t.x];
    xinv_body<L, V>(I.X1, I.Hout, I.nz * I.ny, I.nx, lp2, I.tw0, t.y);
}
// state of buffer ssel -> buffer osel, with the step's base state Mn in
// buffer msel (M for the RK4 stages; the second step of an Euler pair starts
// from Sa)
template <int STAGE>
__global__ __launch_bounds__(256) void kb_stage(const BInst *__restrict__ B, const int2 *__restrict__ T, int ssel,
                                                int osel, int msel)
{
    const int2 t = T[blockIdx.x];
    const BInst &I = B[t.x];
    stage_body<STAGE>(bsel(I, ssel), I.H, bsel(I, msel), I.kacc, bsel(I, osel), I.nx, I.ny, I.nz, I.c,
                      (unsigned)t.y * 256u + threadIdx.x);
}
// single Euler step: the new state, written to Sa, becomes M
__global__ __launch_bounds__(256) void kb_copy(const BInst *__restrict__ B, const int2 *__restrict__ T)
{
    const int2 t = T[blockIdx.x];
    const BInst &I = B[t.x];
    const size_t n3 = 3 * (size_t)I.nx * I.ny * I.nz;
    for (size_t i = (size_t)t.y * 768 + threadIdx.x; i < n3 && i < (size_t)(t.y + 1) * 768; i += 256) I.M[i] = I.Sa[i];
}

// ------------------------------------------------------------- merged ---
// Threads of a merged launch: the row and column passes 512, so a long
// transform still gets several columns (rows) per workgroup for coalesced
// access; the products 256 (long y products, 12-value z products), which
// bounds their ping-pong LDS (proportional to values per thread x threads),
// and 128 for the short z products, whose P = 128 / Q columns per task stay
// within the half spectra of small films.  Every length of a launch runs P
// = threads / Q transforms of Q = L / E threads each.

// Schedule variant of length L in the merged launches: radix order 1 (radix
// 3 then 4s, 12 values per thread) for 3 2^a lengths, the default otherwise;
// the y passes also take order 1 (radix 16 first, 16 values per thread) for
// 2^a lengths >= 512, which halves their threads per column and doubles
// the columns (contiguous bytes of each row) a 512-thread task covers.
// KIND: 0 x passes, 1 y passes, 2 products.
template <int L> constexpr bool bm_alt() { return L >= 24 && L % 3 == 0; }
template <int L, int KIND> constexpr bool bm_o1()
{
    return bm_alt<L>() || (KIND == 1 && L >= 512 && (L & (L - 1)) == 0);
}
template <int L, int KIND> constexpr int bm_v()
{
    return bm_o1<L, KIND>() ? (KIND == 2 ? 3 : 2) : 0;  // tile variant of radix order 1
}
template <int L, int KIND> constexpr int bm_e()
{
    if constexpr (bm_o1<L, KIND>()) return Factors<L, 1>::E;
    else return Factors<L>::E;
}
template <int T, int L, int KIND> constexpr int bm_lp2()
{
    int lp = 0;
    while ((1 << lp) * (L / bm_e<L, KIND>()) < T) ++lp;
    return lp;
}

// Launch slots of the merged mode: the x and y passes one launch each; the
// product passes by register class of their schedules: A the z products of
// at most 8 values per thread, B the y products (nz = 1) and the z products
// of 12 (3 2^a lengths), C every product of a 5 2^a length (20 values per
// thread).  Small-length z products (the bulk of the tasks of thin films)
// then share neither the larger schedules' registers nor the long y
// products' LDS, and slot C is empty unless a grid pads to 5 2^a.
enum {
    MS_XFWD = 0, MS_YFWD = 1, MS_CONV_A = 2, MS_CONV_B = 3, MS_CONV_C = 4, MS_YINV = 5, MS_XINV = 6, MS_COUNT = 7
};
template <int L> constexpr bool bm_five() { return L % 5 == 0; }
// product slot of a length: 0 (A), 1 (B), 2 (C); y products use B or C
template <int L> constexpr int bm_class() { return bm_five<L>() ? 2 : (bm_e<L, 2>() > 8 ? 1 : 0); }
__host__ __device__ constexpr bool bm_conv(int slot) { return slot == MS_CONV_A || slot == MS_CONV_B || slot == MS_CONV_C; }
__host__ __device__ constexpr int bm_threads(int slot)
{
    return slot == MS_CONV_A ? 128 : (bm_conv(slot) ? 256 : 512);
}
constexpr int BM_YCONV = 1 << 16;  // task flag: product along y (nz = 1)
constexpr int BM_EDGE = 1 << 17;   // task flag: edge workgroup (the last kx column, column_of)
constexpr int BM_LEN = (1 << 16) - 1;

// t = (instance, block, plane or ky (an edge task: row group), transform
// length [| BM_YCONV] [| BM_EDGE])
template <int SLOT, int L>
__device__ __forceinline__ void bm_run(const BInst &I, const int4 &t, int sel)
{
    constexpr int KIND = bm_conv(SLOT) ? 2 : ((SLOT == MS_YFWD || SLOT == MS_YINV) ? 1 : 0);
    constexpr int V = bm_v<L, KIND>(), lp2 = bm_lp2<bm_threads(SLOT), L, KIND>();
    static_assert((1 << lp2) * (L / bm_e<L, KIND>()) == bm_threads(SLOT), "P transforms fill the workgroup exactly");
    if constexpr (SLOT == MS_XFWD) xfwd_body<L, V>(bsel(I, sel), I.X1, I.nz * I.ny, I.nx, lp2, I.tw0, t.y);
    else if constexpr (SLOT == MS_YFWD)
        yfwd_body<L, V>(I.X1, I.X2, I.Lx / 2 + 1, I.ny, lp2, I.tw1, t.y, t.z, (t.w & BM_EDGE) ? 3 * I.nz : 0);
    else if constexpr (SLOT == MS_YINV)
        yinv_body<L, V>(I.X2, I.X1, I.Lx / 2 + 1, I.ny, lp2, I.tw1, t.y, t.z, (t.w & BM_EDGE) ? 3 * I.nz : 0);
    else if constexpr (SLOT == MS_XINV) xinv_body<L, V>(I.X1, I.Hout, I.nz * I.ny, I.nx, lp2, I.tw0, t.y);
    else {
        // product slots (bm_class): y products in B or C, z products in
        // the slot of their class
        constexpr int O = bm_o1<L, 2>() ? 1 : 0;
        const bool y = (t.w & BM_YCONV) != 0;
        if constexpr ((SLOT == MS_CONV_B && bm_class<L>() < 2) || (SLOT == MS_CONV_C && bm_class<L>() == 2)) {
            if (y) conv_reg3_body<L, false, O>(I.X1, I.Kt, I.Lx / 2 + 1, I.Ly / 2, I.ny, lp2, I.tw1, t.y, 0);
        }
        if constexpr (bm_class<L>() == SLOT - MS_CONV_A) {
            if (!y)
                conv_reg3_body<L, true, O>(I.X2, I.Kt, I.Lx / 2 + 1, I.Ly / 2, I.nz, lp2, I.tw2, t.y, t.z,
                                           (t.w & BM_EDGE) ? I.Ly : 0);
        }
    }
}

#define MMK_BM_LENGTHS(X)                                                                                \
    X(2) X(4) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(128) \
        X(160) X(192) X(256) X(320) X(384) X(512) X(640) X(768) X(1024)

template <int SLOT>
__global__ __launch_bounds__(bm_threads(SLOT)) void kb_merged(const BInst *__restrict__ B, const int4 *__restrict__ T,
                                                         int sel)
{
    const bool rows = SLOT == MS_XFWD || SLOT == MS_XINV;
    const int4 t = T[rows ? blockIdx.x : xcd_block(blockIdx.x, gridDim.x)];
    const BInst &I = B[t.x];
    switch (t.w & BM_LEN) {
#define MMK_CASE(LEN) case LEN: bm_run<SLOT, LEN>(I, t, sel); break;
        MMK_BM_LENGTHS(MMK_CASE)
#undef MMK_CASE
    default: break;
    }
}

// P, variant and tile of length L in the merged launches (host side)
// P (transforms per workgroup) of length L in merged slot `slot`, and the
// schedule variant of `pass` there
static int bm_P(int slot, int L)
{
    switch (L) {
#define MMK_CASE(LEN) \
    case LEN:                                                                  \
        return slot == MS_CONV_A   ? (1 << bm_lp2<bm_threads(MS_CONV_A), LEN, 2>())                   \
               : bm_conv(slot)     ? (1 << bm_lp2<bm_threads(MS_CONV_B), LEN, 2>())                   \
               : (slot == MS_YFWD || slot == MS_YINV) ? (1 << bm_lp2<bm_threads(MS_YFWD), LEN, 1>()) \
                                   : (1 << bm_lp2<bm_threads(MS_XFWD), LEN, 0>());
        MMK_BM_LENGTHS(MMK_CASE)
#undef MMK_CASE
    default: return 0;
    }
}
static int bm_variant(int pass, int L)
{
    switch (L) {
#define MMK_CASE(LEN) \
    case LEN:                                                            \
        return pass == MM_PASS_ZCONV || pass == MM_PASS_YCONV ? bm_v<LEN, 2>() \
               : (pass == MM_PASS_YFWD || pass == MM_PASS_YINV) ? bm_v<LEN, 1>() : bm_v<LEN, 0>();
        MMK_BM_LENGTHS(MMK_CASE)
#undef MMK_CASE
    default: return 0;
    }
}
// LDS bytes of P transforms of length L for `pass` in variant var: linear in
// P (twiddles plus P transforms' slots), taken from the shapes at P = 1, 2
static size_t bm_lds(int pass, int L, int var, int P)
{
    int t1, t2, m;
    size_t l1 = 0, l2 = 0;
    shape_for(pass, L, 1 + 256 * var, t1, l1, m);
    shape_for(pass, L, 2 + 256 * var, t2, l2, m);
    return l1 + (size_t)(P - 1) * (l2 - l1);
}

// register class of length L (0: at most 8 values per thread, 1: 12)
static int bm_class_of(int L)
{
    switch (L) {
#define MMK_CASE(LEN) case LEN: return bm_class<LEN>();
        MMK_BM_LENGTHS(MMK_CASE)
#undef MMK_CASE
    default: return 0;
    }
}

// ---------------------------------------------------------------- host ---
struct BGroup {
    int pass = 0, L = 0, tile = 0;
    int threads = 0;
    size_t lds = 0;
    std::vector<int4> tasks;
    int4 *d = nullptr;
    size_t cap = 0;  // device table capacity: the most tasks any candidate tile makes
};

struct BatchImpl {
    int count = 0;
    std::vector<mm_plan> plans;
    std::vector<BInst> inst;
    BInst *d_inst = nullptr, *d_io = nullptr;
    std::vector<BGroup> groups;
    std::vector<int2> stage_tasks, copy_tasks;
    int2 *d_stage = nullptr, *d_copy = nullptr;
    size_t lds_limit = 65536;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    std::string key;
    std::vector<float *> bound_M;
    std::string bound_params;
    size_t bytes = 0;                // workspace bytes
    std::vector<size_t> plan_bytes;  // per-instance plan workspace
    char *ws = nullptr;              // bound workspace (nullptr: unbound)
    bool merged = true;              // launch mode
    BGroup mg[MS_COUNT];             // merged launch per slot (tile unused)
};

static int pass_len_of(const BInst &I, int pass)
{
    switch (pass) {
    case MM_PASS_XFWD:
    case MM_PASS_XINV: return I.Lx;
    case MM_PASS_YFWD:
    case MM_PASS_YINV: return I.nz > 1 ? I.Ly : 0;
    case MM_PASS_ZCONV: return I.nz > 1 ? I.Lz : 0;
    case MM_PASS_YCONV: return I.nz == 1 ? I.Ly : 0;
    default: return 0;
    }
}

static int launch_group(const BGroup &g, const BInst *table, int sel, hipStream_t s, bool raise_only);

// tile variants in the default radix order: single-component passes 0, 1;
// product passes 0, 1, 2
static bool default_order(int pass, int tile)
{
    const int var = tile >> 8;
    return (pass == MM_PASS_ZCONV || pass == MM_PASS_YCONV) ? var <= 2 : var <= 1;
}

static void make_tasks(const BatchImpl &b, const BGroup &g, int tile, std::vector<int4> &tasks)
{
    const int P = tile & 255;
    tasks.clear();
    for (int i = 0; i < b.count; ++i) {
        const BInst &I = b.inst[i];
        if (pass_len_of(I, g.pass) != g.L) continue;
        const int nxc = I.Lx / 2 + 1, ncr = I.nz * I.ny;
        switch (g.pass) {
        case MM_PASS_XFWD:
        case MM_PASS_XINV: {
            const int pairs = 3 * ((ncr + 1) / 2);
            for (int bx = 0; bx < (pairs + P - 1) / P; ++bx) tasks.push_back(make_int4(i, bx, 0, 0));
            break;
        }
        case MM_PASS_YFWD:
        case MM_PASS_YINV:
            for (int pl = 0; pl < 3 * I.nz; ++pl)
                for (int bx = 0; bx < (nxc + P - 1) / P; ++bx) tasks.push_back(make_int4(i, bx, pl, 0));
            break;
        case MM_PASS_ZCONV:  // the two rows of a mirror pair next to each other, then the tile
            for (int m = 0; m < I.Ly / 2; ++m)
                for (int bx = 0; bx < (nxc + P - 1) / P; ++bx)
                    for (int h = 0; h < 2; ++h)
                        tasks.push_back(make_int4(i, bx, ky_of_slot(2 * m + h, I.Ly / 2), 0));
            break;
        case MM_PASS_YCONV:
            for (int bx = 0; bx < (nxc + P - 1) / P; ++bx) tasks.push_back(make_int4(i, bx, 0, 0));
            break;
        default: break;
        }
    }
}

// Task table of a group for its current tile, uploaded into the group's
// slice of the workspace (sized at set-up for the largest candidate table).
static int build_tasks(BatchImpl &b, BGroup &g)
{
    make_tasks(b, g, g.tile, g.tasks);
    if (g.tasks.size() > g.cap) return fail(MM_EINVAL, "batch: task table over its capacity");
    MMK_HIP(hipMemcpy(g.d, g.tasks.data(), sizeof(int4) * g.tasks.size(), hipMemcpyHostToDevice));
    int maxt;
    shape_for(g.pass, g.L, g.tile, g.threads, g.lds, maxt);
    return launch_group(g, nullptr, 0, nullptr, true);  // raise the LDS limit if this tile needs it
}

// Task table of merged launch slot `slot`: every instance with the pass
// active (and, for a product slot, its product in that slot),
// longest transform first, each with its length's tile; the launch's LDS is
// the largest any of its lengths needs.
static void make_merged(BatchImpl &b, int slot)
{
    BGroup &g = b.mg[slot];
    g.tasks.clear();
    g.lds = 0;
    const bool conv = bm_conv(slot);
    auto pass_of = [&](const BInst &I) {
        switch (slot) {
        case MS_XFWD: return (int)MM_PASS_XFWD;
        case MS_YFWD: return (int)MM_PASS_YFWD;
        case MS_YINV: return (int)MM_PASS_YINV;
        case MS_XINV: return (int)MM_PASS_XINV;
        default: return I.nz > 1 ? (int)MM_PASS_ZCONV : (int)MM_PASS_YCONV;
        }
    };
    auto len_of = [&](const BInst &I) {
        const int L = pass_len_of(I, pass_of(I));
        // z products by register class; every y product in slot B
        if (conv && L) {
            const int cls = bm_class_of(L);
            const int want = I.nz > 1 ? cls : (cls == 2 ? 2 : 1);  // y products: B, or C for 5 2^a
            if (want != slot - MS_CONV_A) return 0;
        }
        return L;
    };
    std::vector<int> order;
    for (int i = 0; i < b.count; ++i)
        if (len_of(b.inst[i])) order.push_back(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return len_of(b.inst[a]) > len_of(b.inst[c]); });
    for (int i : order) {
        const BInst &I = b.inst[i];
        const int pass = pass_of(I);
        const int L = len_of(I);
        const int P = bm_P(slot, L);
        g.lds = std::max(g.lds, bm_lds(pass, L, bm_variant(pass, L), P));
        const int nxc = I.Lx / 2 + 1, ncr = I.nz * I.ny;
        // column passes: when P divides the Lx/2 columns below the last,
        // tiles over those and edge tasks (dispatched first) for the last
        const bool edge = P > 1 && (I.Lx / 2) % P == 0;
        const int ntm = edge ? (I.Lx / 2) / P : (nxc + P - 1) / P;
        auto edges = [&](int nrows) {
            if (edge)
                for (int e = 0; e < (nrows + P - 1) / P; ++e) g.tasks.push_back(make_int4(i, 0, e, L | BM_EDGE));
        };
        switch (pass) {
        case MM_PASS_XFWD:
        case MM_PASS_XINV: {
            const int pairs = 3 * ((ncr + 1) / 2);
            for (int bx = 0; bx < (pairs + P - 1) / P; ++bx) g.tasks.push_back(make_int4(i, bx, 0, L));
            break;
        }
        case MM_PASS_YFWD:
        case MM_PASS_YINV:
            edges(3 * I.nz);
            for (int pl = 0; pl < 3 * I.nz; ++pl)
                for (int bx = 0; bx < ntm; ++bx) g.tasks.push_back(make_int4(i, bx, pl, L));
            break;
        case MM_PASS_ZCONV:
            edges(I.Ly);
            for (int m = 0; m < I.Ly / 2; ++m)
                for (int bx = 0; bx < ntm; ++bx)
                    for (int h = 0; h < 2; ++h)
                        g.tasks.push_back(make_int4(i, bx, ky_of_slot(2 * m + h, I.Ly / 2), L));
            break;
        case MM_PASS_YCONV:
            for (int bx = 0; bx < (nxc + P - 1) / P; ++bx) g.tasks.push_back(make_int4(i, bx, 0, L | BM_YCONV));
            break;
        default: break;
        }
    }
    g.cap = g.tasks.size();
}

static int ilog2i(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

template <typename K>
static void raise_if_needed(K kern, size_t lds)
{
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int L>
static void launch_group_len(const BGroup &g, const BInst *table, int sel, hipStream_t s, bool raise_only)
{
    const int P = g.tile & 255, var = g.tile >> 8, lp2 = ilog2i(P);
    const dim3 grid((unsigned)g.tasks.size()), block(g.threads);
    const size_t lds = g.lds;
    switch (g.pass) {
    case MM_PASS_XFWD:
        if (var == 0) { if (raise_only) raise_if_needed(kb_xfwd<L, 0>, lds); else hipLaunchKernelGGL((kb_xfwd<L, 0>), grid, block, lds, s, table, g.d, sel, lp2); }
        else { if (raise_only) raise_if_needed(kb_xfwd<L, 1>, lds); else hipLaunchKernelGGL((kb_xfwd<L, 1>), grid, block, lds, s, table, g.d, sel, lp2); }
        break;
    case MM_PASS_YFWD:
        if (var == 0) { if (raise_only) raise_if_needed(kb_yfwd<L, 0>, lds); else hipLaunchKernelGGL((kb_yfwd<L, 0>), grid, block, lds, s, table, g.d, lp2); }
        else { if (raise_only) raise_if_needed(kb_yfwd<L, 1>, lds); else hipLaunchKernelGGL((kb_yfwd<L, 1>), grid, block, lds, s, table, g.d, lp2); }
        break;
    case MM_PASS_YINV:
        if (var == 0) { if (raise_only) raise_if_needed(kb_yinv<L, 0>, lds); else hipLaunchKernelGGL((kb_yinv<L, 0>), grid, block, lds, s, table, g.d, lp2); }
        else { if (raise_only) raise_if_needed(kb_yinv<L, 1>, lds); else hipLaunchKernelGGL((kb_yinv<L, 1>), grid, block, lds, s, table, g.d, lp2); }
        break;
    case MM_PASS_XINV:
        if (var == 0) { if (raise_only) raise_if_needed(kb_xinv<L, 0>, lds); else hipLaunchKernelGGL((kb_xinv<L, 0>), grid, block, lds, s, table, g.d, lp2); }
        else { if (raise_only) raise_if_needed(kb_xinv<L, 1>, lds); else hipLaunchKernelGGL((kb_xinv<L, 1>), grid, block, lds, s, table, g.d, lp2); }
        break;
    case MM_PASS_ZCONV:
    case MM_PASS_YCONV: {
        const bool z = g.pass == MM_PASS_ZCONV;
        if (var == 0) {
            if (z) { if (raise_only) raise_if_needed(kb_reg3<L, true>, lds); else hipLaunchKernelGGL((kb_reg3<L, true>), grid, block, lds, s, table, g.d, lp2); }
            else { if (raise_only) raise_if_needed(kb_reg3<L, false>, lds); else hipLaunchKernelGGL((kb_reg3<L, false>), grid, block, lds, s, table, g.d, lp2); }
        } else if (var == 1) {
            if (z) { if (raise_only) raise_if_needed(kb_split<L, 0, true>, lds); else hipLaunchKernelGGL((kb_split<L, 0, true>), grid, block, lds, s, table, g.d, lp2); }
            else { if (raise_only) raise_if_needed(kb_split<L, 0, false>, lds); else hipLaunchKernelGGL((kb_split<L, 0, false>), grid, block, lds, s, table, g.d, lp2); }
        } else {
            if (z) { if (raise_only) raise_if_needed(kb_split<L, 1, true>, lds); else hipLaunchKernelGGL((kb_split<L, 1, true>), grid, block, lds, s, table, g.d, lp2); }
            else { if (raise_only) raise_if_needed(kb_split<L, 1, false>, lds); else hipLaunchKernelGGL((kb_split<L, 1, false>), grid, block, lds, s, table, g.d, lp2); }
        }
        break;
    }
    default: break;
    }
}

#define MMK_BATCH_LENGTHS(X)                                                                             \
    X(2) X(4) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(128) \
        X(160) X(192) X(256) X(320) X(384) X(512) X(640) X(768) X(1024)

static int launch_group(const BGroup &g, const BInst *table, int sel, hipStream_t s, bool raise_only)
{
    if (g.tasks.empty()) return MM_OK;
    switch (g.L) {
#define MMK_CASE(LEN) case LEN: launch_group_len<LEN>(g, table, sel, s, raise_only); break;
        MMK_BATCH_LENGTHS(MMK_CASE)
#undef MMK_CASE
    default: return fail(MM_EINVAL, "batch: unsupported length");
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MM_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
    return MM_OK;
}

static const int DEMAG_ORDER[6] = {MM_PASS_XFWD, MM_PASS_YFWD, MM_PASS_ZCONV, MM_PASS_YCONV, MM_PASS_YINV,
                                   MM_PASS_XINV};

static int merged_launch(const BatchImpl &b, int slot, const BInst *table, int sel, hipStream_t s)
{
    const BGroup &g = b.mg[slot];
    if (g.tasks.empty()) return MM_OK;
    const dim3 grid((unsigned)g.tasks.size()), block((unsigned)bm_threads(slot));
    switch (slot) {
    case MS_XFWD: hipLaunchKernelGGL(kb_merged<MS_XFWD>, grid, block, g.lds, s, table, g.d, sel); break;
    case MS_YFWD: hipLaunchKernelGGL(kb_merged<MS_YFWD>, grid, block, g.lds, s, table, g.d, sel); break;
    case MS_CONV_A: hipLaunchKernelGGL(kb_merged<MS_CONV_A>, grid, block, g.lds, s, table, g.d, sel); break;
    case MS_CONV_B: hipLaunchKernelGGL(kb_merged<MS_CONV_B>, grid, block, g.lds, s, table, g.d, sel); break;
    case MS_CONV_C: hipLaunchKernelGGL(kb_merged<MS_CONV_C>, grid, block, g.lds, s, table, g.d, sel); break;
    case MS_YINV: hipLaunchKernelGGL(kb_merged<MS_YINV>, grid, block, g.lds, s, table, g.d, sel); break;
    case MS_XINV: hipLaunchKernelGGL(kb_merged<MS_XINV>, grid, block, g.lds, s, table, g.d, sel); break;
    default: break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MM_EHIP, std::string("batch merged launch: ") + hipGetErrorString(e));
    return MM_OK;
}

static int batch_demag_enqueue(BatchImpl &b, const BInst *table, int sel, hipStream_t s)
{
    if (b.merged) {
        for (int slot = 0; slot < MS_COUNT; ++slot) {
            int rc = merged_launch(b, slot, table, sel, s);
            if (rc != MM_OK) return rc;
        }
        return MM_OK;
    }
    for (int pass : DEMAG_ORDER)
        for (const BGroup &g : b.groups)
            if (g.pass == pass) {
                int rc = launch_group(g, table, sel, s, false);
                if (rc != MM_OK) return rc;
            }
    return MM_OK;
}

template <int STAGE>
static int batch_stage(BatchImpl &b, int ssel, int osel, hipStream_t s, int msel = 0)
{
    hipLaunchKernelGGL(kb_stage<STAGE>, dim3((unsigned)b.stage_tasks.size()), dim3(256), 0, s, b.d_inst, b.d_stage,
                       ssel, osel, msel);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MM_EHIP, std::string("batch stage: ") + hipGetErrorString(e));
    return MM_OK;
}

// One step, or (euler_pair) two Euler steps M -> Sa -> M, which alternate
// between the two buffers and copy nothing.
static int batch_step_enqueue(BatchImpl &b, int integrator, hipStream_t s, bool euler_pair = false)
{
    int rc;
    if (integrator == MM_EULER && euler_pair) {
        if ((rc = batch_demag_enqueue(b, b.d_inst, 0, s)) != MM_OK) return rc;
        if ((rc = batch_stage<0>(b, 0, 1, s)) != MM_OK) return rc;
        if ((rc = batch_demag_enqueue(b, b.d_inst, 1, s)) != MM_OK) return rc;
        return batch_stage<0>(b, 1, 0, s, 1);
    }
    if (integrator == MM_EULER) {
        if ((rc = batch_demag_enqueue(b, b.d_inst, 0, s)) != MM_OK) return rc;
        if ((rc = batch_stage<0>(b, 0, 1, s)) != MM_OK) return rc;
        hipLaunchKernelGGL(kb_copy, dim3((unsigned)b.copy_tasks.size()), dim3(256), 0, s, b.d_inst, b.d_copy);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? MM_OK : fail(MM_EHIP, std::string("batch copy: ") + hipGetErrorString(e));
    }
    // stage states: S1 = M, S2 = Sa, S3 = Sb, S4 = Sa; stage 4 writes M
    if ((rc = batch_demag_enqueue(b, b.d_inst, 0, s)) != MM_OK) return rc;
    if ((rc = batch_stage<1>(b, 0, 1, s)) != MM_OK) return rc;
    if ((rc = batch_demag_enqueue(b, b.d_inst, 1, s)) != MM_OK) return rc;
    if ((rc = batch_stage<2>(b, 1, 2, s)) != MM_OK) return rc;
    if ((rc = batch_demag_enqueue(b, b.d_inst, 2, s)) != MM_OK) return rc;
    if ((rc = batch_stage<3>(b, 2, 1, s)) != MM_OK) return rc;
    if ((rc = batch_demag_enqueue(b, b.d_inst, 1, s)) != MM_OK) return rc;
    return batch_stage<4>(b, 1, 0, s);
}

static void drop_graph(BatchImpl &b)
{
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
    b.key.clear();
}

static void free_batch(BatchImpl *b)
{
    if (!b) return;
    drop_graph(*b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (mm_plan p : b->plans) mm_destroy(p);
    delete b;
}

static void raise_merged_lds(BatchImpl &b)
{
    const void *k[MS_COUNT] = {(const void *)kb_merged<MS_XFWD>,   (const void *)kb_merged<MS_YFWD>,
                               (const void *)kb_merged<MS_CONV_A>, (const void *)kb_merged<MS_CONV_B>,
                               (const void *)kb_merged<MS_CONV_C>, (const void *)kb_merged<MS_YINV>,
                               (const void *)kb_merged<MS_XINV>};
    for (int slot = 0; slot < MS_COUNT; ++slot)
        if (b.mg[slot].lds > 65536)
            (void)hipFuncSetAttribute(k[slot], hipFuncAttributeMaxDynamicSharedMemorySize, (int)b.mg[slot].lds);
}

}  // namespace mmk

using namespace mmk;

struct mm_batch_s {
    BatchImpl *impl;
};

extern "C" {

int mm_batch_setup(int count, const int *nx, const int *ny, const int *nz, const double *dx, const double *dy,
                   const double *dz, mm_batch *out)
{
    if (!out) return fail(MM_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !nx || !ny || !nz || !dx || !dy || !dz) return fail(MM_EINVAL, "batch: bad arguments");
    BatchImpl *b = new BatchImpl();
    b->count = count;
    int rc = MM_OK;
    for (int i = 0; i < count && rc == MM_OK; ++i) {
        mm_plan p = nullptr;
        rc = mm_demag_setup(nx[i], ny[i], nz[i], dx[i], dy[i], dz[i], &p);
        if (rc == MM_OK) b->plans.push_back(p);
    }
    if (rc != MM_OK) {
        free_batch(b);
        return rc;
    }
    b->lds_limit = plan_of(b->plans[0])->lds_limit;
    for (int i = 0; i < count; ++i) {
        const Plan &p = *plan_of(b->plans[i]);
        if (p.lds_limit < b->lds_limit) b->lds_limit = p.lds_limit;
        BInst I{};
        I.nx = p.nx; I.ny = p.ny; I.nz = p.nz;
        I.Lx = p.Lx; I.Ly = p.Ly; I.Lz = p.Lz;
        b->inst.push_back(I);
        const size_t n = (size_t)p.cells();
        for (size_t blk = 0; blk < (n + 255) / 256; ++blk) b->stage_tasks.push_back(make_int2(i, (int)blk));
        for (size_t blk = 0; blk < (3 * n + 767) / 768; ++blk) b->copy_tasks.push_back(make_int2(i, (int)blk));
    }
    // one group per (pass, length) present in the batch; its device table
    // holds the largest task list any candidate tile makes
    std::vector<int4> scratch;
    for (int pass : DEMAG_ORDER) {
        std::vector<int> lens;
        for (const BInst &I : b->inst) {
            const int L = pass_len_of(I, pass);
            if (L && std::find(lens.begin(), lens.end(), L) == lens.end()) lens.push_back(L);
        }
        std::sort(lens.begin(), lens.end());
        for (int L : lens) {
            BGroup g;
            g.pass = pass;
            g.L = L;
            g.tile = default_tile_for(pass, L, b->lds_limit);
            for (int t : tile_candidates_for(pass, L, b->lds_limit)) {
                if (!default_order(pass, t)) continue;  // the groups run the default radix orders
                make_tasks(*b, g, t, scratch);
                g.cap = std::max(g.cap, scratch.size());
            }
            make_tasks(*b, g, g.tile, scratch);
            g.cap = std::max(g.cap, scratch.size());
            b->groups.push_back(g);
        }
    }
    for (int slot = 0; slot < MS_COUNT; ++slot) make_merged(*b, slot);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t total = 0;
    for (int slot = 0; slot < MS_COUNT; ++slot) total += al(sizeof(int4) * b->mg[slot].tasks.size());
    for (int i = 0; i < count; ++i) {
        size_t pb = 0;
        mm_plan_workspace_bytes(b->plans[i], &pb);
        b->plan_bytes.push_back(al(pb));
        total += al(pb);
    }
    for (const BGroup &g : b->groups) total += al(sizeof(int4) * g.cap);
    total += 2 * al(sizeof(BInst) * count) + al(sizeof(int2) * b->stage_tasks.size()) +
             al(sizeof(int2) * b->copy_tasks.size());
    b->bytes = total;
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        free_batch(b);
        return fail(MM_EHIP, "batch stream");
    }
    *out = new mm_batch_s{b};
    return MM_OK;
}

int mm_batch_workspace_bytes(mm_batch batch, size_t *bytes)
{
    if (!batch || !batch->impl || !bytes) return fail(MM_EINVAL, "NULL batch or bytes");
    *bytes = batch->impl->bytes;
    return MM_OK;
}

int mm_batch_bind_workspace(mm_batch batch, void *ws, size_t bytes)
{
    if (!batch || !batch->impl || !ws) return fail(MM_EINVAL, "NULL batch or workspace");
    BatchImpl &b = *batch->impl;
    if ((uintptr_t)ws % 256 != 0) return fail(MM_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < b.bytes)
        return fail(MM_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes; the batch needs " +
                                   std::to_string(b.bytes));
    drop_graph(b);
    b.ws = nullptr;
    b.bound_M.clear();
    b.bound_params.clear();
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    char *cur = (char *)ws;
    int rc;
    for (int i = 0; i < b.count; ++i) {
        if ((rc = mm_plan_bind_workspace(b.plans[i], cur, b.plan_bytes[i])) != MM_OK) return rc;
        cur += b.plan_bytes[i];
        const Plan &p = *plan_of(b.plans[i]);
        BInst &I = b.inst[i];
        I.M = nullptr;
        I.Sa = p.Sa; I.Sb = p.Sb; I.H = p.H; I.kacc = p.kacc; I.Hout = p.H;
        I.X1 = p.X1; I.X2 = p.X2; I.Kt = p.Kt;
        I.tw0 = p.tw[0]; I.tw1 = p.tw[1]; I.tw2 = p.tw[2];
    }
    for (BGroup &g : b.groups) {
        g.d = (int4 *)cur;
        cur += al(sizeof(int4) * g.cap);
        if ((rc = build_tasks(b, g)) != MM_OK) return rc;
    }
    for (int slot = 0; slot < MS_COUNT; ++slot) {
        BGroup &g = b.mg[slot];
        g.d = (int4 *)cur;
        cur += al(sizeof(int4) * g.tasks.size());
        if (!g.tasks.empty())
            MMK_HIP(hipMemcpy(g.d, g.tasks.data(), sizeof(int4) * g.tasks.size(), hipMemcpyHostToDevice));
        if (g.lds > b.lds_limit) return fail(MM_EINVAL, "batch: merged launch needs more LDS than the device has");
    }
    raise_merged_lds(b);
    b.d_inst = (BInst *)cur; cur += al(sizeof(BInst) * b.count);
    b.d_io = (BInst *)cur; cur += al(sizeof(BInst) * b.count);
    b.d_stage = (int2 *)cur; cur += al(sizeof(int2) * b.stage_tasks.size());
    b.d_copy = (int2 *)cur;
    MMK_HIP(hipMemcpy(b.d_inst, b.inst.data(), sizeof(BInst) * b.count, hipMemcpyHostToDevice));
    MMK_HIP(hipMemcpy(b.d_io, b.inst.data(), sizeof(BInst) * b.count, hipMemcpyHostToDevice));
    MMK_HIP(hipMemcpy(b.d_stage, b.stage_tasks.data(), sizeof(int2) * b.stage_tasks.size(), hipMemcpyHostToDevice));
    MMK_HIP(hipMemcpy(b.d_copy, b.copy_tasks.data(), sizeof(int2) * b.copy_tasks.size(), hipMemcpyHostToDevice));
    MMK_HIP(hipDeviceSynchronize());
    b.ws = (char *)ws;
    return MM_OK;
}

static int batch_ready(mm_batch batch)
{
    if (!batch || !batch->impl) return fail(MM_EINVAL, "NULL batch");
    if (!batch->impl->ws) return fail(MM_EINVAL, "batch has no workspace: call mm_batch_bind_workspace first");
    return MM_OK;
}

void mm_batch_destroy(mm_batch batch)
{
    if (!batch) return;
    free_batch(batch->impl);
    delete batch;
}

int mm_batch_demag(mm_batch batch, const float *const *M, float *const *H, void *stream)
{
    int rc0 = batch_ready(batch);
    if (rc0 != MM_OK) return rc0;
    if (!M || !H) return fail(MM_EINVAL, "NULL pointer table");
    BatchImpl &b = *batch->impl;
    std::vector<BInst> io = b.inst;
    for (int i = 0; i < b.count; ++i) {
        if (!M[i] || !H[i] || (const void *)M[i] == (const void *)H[i])
            return fail(MM_EINVAL, "batch demag: NULL or aliased field of instance " + std::to_string(i));
        io[i].M = const_cast<float *>(M[i]);
        io[i].Hout = H[i];
    }
    hipStream_t s = (hipStream_t)stream;
    MMK_HIP(hipStreamSynchronize(s));  // the table may still feed an earlier call
    MMK_HIP(hipMemcpy(b.d_io, io.data(), sizeof(BInst) * b.count, hipMemcpyHostToDevice));
    return batch_demag_enqueue(b, b.d_io, 0, s);
}

int mm_batch_step(mm_batch batch, const mm_llg_params *params, float *const *M, int nsteps, void *stream)
{
    int rc0 = batch_ready(batch);
    if (rc0 != MM_OK) return rc0;
    if (!params || !M) return fail(MM_EINVAL, "NULL params or M table");
    if (nsteps < 0) return fail(MM_EINVAL, "nsteps < 0");
    BatchImpl &b = *batch->impl;
    const int integrator = params[0].integrator;
    for (int i = 0; i < b.count; ++i) {
        if (!M[i]) return fail(MM_EINVAL, "NULL M of instance " + std::to_string(i));
        if (params[i].integrator != integrator) return fail(MM_EINVAL, "batch: one integrator for all instances");
        if (!(params[i].Ms > 0.0) || !std::isfinite(params[i].dt)) return fail(MM_EINVAL, "batch: bad params");
        if (params[i].demag_mode != MM_EXACT) return fail(MM_EINVAL, "batch: exact demag only");
    }
    if (nsteps == 0) return MM_OK;
    hipStream_t s = (hipStream_t)stream;
    std::string pkey((const char *)params, sizeof(mm_llg_params) * b.count);
    std::vector<float *> mv(M, M + b.count);
    if (mv != b.bound_M || pkey != b.bound_params) {
        for (int i = 0; i < b.count; ++i) {
            b.inst[i].M = M[i];
            b.inst[i].Hout = b.inst[i].H;
            b.inst[i].c = stage_coef(*plan_of(b.plans[i]), params[i]);
        }
        MMK_HIP(hipStreamSynchronize(s));
        MMK_HIP(hipDeviceSynchronize());
        MMK_HIP(hipMemcpy(b.d_inst, b.inst.data(), sizeof(BInst) * b.count, hipMemcpyHostToDevice));
        b.bound_M = mv;
        b.bound_params = pkey;
        drop_graph(b);
    }
    // Euler: the graph holds a pair of steps (no copy); an odd count ends
    // with one copying step launched directly
    const bool pair = integrator == MM_EULER;
    const int unit = pair ? 2 : 1;
    if (nsteps < unit) return batch_step_enqueue(b, integrator, s);
    std::string key = std::to_string(integrator) + (b.merged ? "m" : "g");
    for (const BGroup &g : b.groups) key += "," + std::to_string(g.tile);
    if (!b.exec || b.key != key) {
        drop_graph(b);
        MMK_HIP(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
        int rc = batch_step_enqueue(b, integrator, b.cap, pair);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b.cap, &g);
        if (rc != MM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(MM_EHIP, std::string("batch capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            b.exec = nullptr;
            return fail(MM_EHIP, std::string("batch instantiate: ") + hipGetErrorString(e));
        }
        b.graph = g;
        b.key = key;
    }
    for (int i = 0; i + unit <= nsteps; i += unit) MMK_HIP(hipGraphLaunch(b.exec, s));
    if (nsteps % unit) return batch_step_enqueue(b, integrator, s);
    return MM_OK;
}

int mm_batch_autotune(mm_batch batch, int reps, void *stream)
{
    int rc0 = batch_ready(batch);
    if (rc0 != MM_OK) return rc0;
    BatchImpl &b = *batch->impl;
    if (reps < 1) reps = 1;
    hipStream_t s = (hipStream_t)stream;
    // time on the internal buffers: the x pass reads Sa (its content does not
    // change the timing), the others read what the previous pass left
    for (int i = 0; i < b.count; ++i) {
        const Plan &p = *plan_of(b.plans[i]);
        MMK_HIP(hipMemsetAsync(p.Sa, 0, sizeof(float) * 3 * (size_t)p.cells(), s));
    }
    MMK_HIP(hipStreamSynchronize(s));
    hipEvent_t e0, e1;
    MMK_HIP(hipEventCreate(&e0));
    MMK_HIP(hipEventCreate(&e1));
    int rc = MM_OK, tuned = 0;
    const bool was_merged = b.merged;
    b.merged = false;  // the groups' tiles are what there is to tune
    // a candidate is timed as `reps` complete batched demag evaluations
    // (every group launched in step order, events only around the loop), so
    // it is judged in the cache state and launch overlap of a real step
    for (BGroup &g : b.groups) {
        const int keep = g.tile;
        float best = 1e30f;
        int best_tile = keep;
        for (int t : tile_candidates_for(g.pass, g.L, b.lds_limit)) {
            if (!default_order(g.pass, t)) continue;  // the groups run the default radix orders
            g.tile = t;
            if ((rc = build_tasks(b, g)) != MM_OK) break;
            if ((rc = batch_demag_enqueue(b, b.d_inst, 1, s)) != MM_OK) break;
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps && rc == MM_OK; ++r) rc = batch_demag_enqueue(b, b.d_inst, 1, s);
            (void)hipEventRecord(e1, s);
            if (rc != MM_OK || hipEventSynchronize(e1) != hipSuccess) {
                if (rc == MM_OK) rc = fail(MM_EHIP, "batch autotune event");
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) {
                best = ms;
                best_tile = t;
            }
            ++tuned;
        }
        if (rc != MM_OK) break;
        g.tile = best_tile;
        if ((rc = build_tasks(b, g)) != MM_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b.merged = was_merged;
    drop_graph(b);
    if (rc != MM_OK) return rc;
    return tuned ? MM_OK : fail(MM_ETUNE, "batch: no candidate ran");
}

int mm_batch_query(mm_batch batch, int *groups, int *launches_per_step, long long *cells)
{
    if (!batch || !batch->impl) return fail(MM_EINVAL, "NULL batch");
    BatchImpl &b = *batch->impl;
    int kinds = 0;
    for (int slot = 0; slot < MS_COUNT; ++slot) kinds += b.mg[slot].tasks.empty() ? 0 : 1;
    if (groups) *groups = b.merged ? kinds : (int)b.groups.size();
    if (launches_per_step) *launches_per_step = 4 * ((b.merged ? kinds : (int)b.groups.size()) + 1);
    if (cells) {
        long long c = 0;
        for (const BInst &I : b.inst) c += (long long)I.nx * I.ny * I.nz;
        *cells = c;
    }
    return MM_OK;
}

int mm_batch_set_mode(mm_batch batch, int mode)
{
    if (!batch || !batch->impl) return fail(MM_EINVAL, "NULL batch");
    if (mode != MM_BATCH_GROUPED && mode != MM_BATCH_MERGED) return fail(MM_EINVAL, "unknown batch mode");
    batch->impl->merged = mode == MM_BATCH_MERGED;
    drop_graph(*batch->impl);
    return MM_OK;
}

int mm_batch_group_tile(mm_batch batch, int index, int *pass, int *length, int *tile)
{
    if (!batch || !batch->impl) return fail(MM_EINVAL, "NULL batch");
    BatchImpl &b = *batch->impl;
    if (index < 0 || index >= (int)b.groups.size()) return fail(MM_EINVAL, "group index");
    if (pass) *pass = b.groups[index].pass;
    if (length) *length = b.groups[index].L;
    if (tile) *tile = b.groups[index].tile;
    return MM_OK;
}

}  // extern "C"
