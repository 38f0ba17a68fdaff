// rs_blocks.hip -- the block networks BTN and OET at device scale (Section 2;
// Section 3, Eqs. Tb and To): the n keys are cut into p runs of
// N = ceil(n/p) keys held in HBM (the tail padded with the largest key),
// every run is sorted by one workgroup (the segmented sort's per-segment
// paths), then the network's merge-split stages run, each one pass over all
// runs: BTN's lg p (lg p + 1)/2 stages of Batcher's bitonic sorter on p
// wires, or OET's p rounds of neighbour pairs.
//
// A merge-split of runs A (the lower index) and B leaves the N smallest keys
// of their union, in order, in one run and the N largest in the other; ties
// are taken from A first.  Each pair's 2N outputs are cut into chunks of
// MS_C.  First the co-rank of every chunk boundary d -- how many of the
// first d outputs come from A -- is found by one binary search per boundary
// (all boundaries of the stage in parallel).  Then one workgroup per chunk
// loads its slices of A and B into LDS, each thread finds its own co-rank
// inside them and merges MS_ITEMS outputs, and the chunk is written back with
// consecutive threads on consecutive addresses.
#include <vector>

#include "rs_internal.hpp"

namespace rs {
namespace {

// 8 outputs per thread: a shorter merge per thread after its co-rank search
// (measured at 2^27 keys: 0.243 ms a stage against 0.285 with 256 x 16 and
// 0.318 with 1,024 x 4)
constexpr int MS_NT = 512;
constexpr int MS_ITEMS = 8;
constexpr uint32_t MS_C = MS_NT * MS_ITEMS;  // outputs per merge workgroup

struct Stage {
    uint32_t oet;     // 0: a BTN stage, 1: an OET round
    uint32_t k, lj;   // BTN: merge size k, partner distance 1 << lj
    uint32_t parity;  // OET: the lower run of the round's first pair
    uint32_t pairs;
};

// Pair q of a stage: runs a < b, and whether a keeps the smaller half (BTN:
// the pair sorts ascending when bit k of a is clear).
__device__ __forceinline__ void pair_of(const Stage& s, uint32_t q, uint32_t& a, uint32_t& b, bool& asc) {
    if (s.oet) {
        a = s.parity + 2 * q;
        b = a + 1;
        asc = true;
    } else {
        const uint32_t j = 1u << s.lj;
        a = ((q >> s.lj) << (s.lj + 1)) | (q & (j - 1));
        b = a | j;
        asc = (a & s.k) == 0;
    }
}

// Co-rank of output d in the merge of A (la keys) and B (lb keys) with ties
// from A: the largest x in [max(0, d - lb), min(d, la)] with
// A[x-1] <= B[d-x].  For x above the lower end d - x < lb, so B[d-x] exists.
__device__ __forceinline__ uint32_t corank(const uint32_t* A, uint32_t la, const uint32_t* B, uint32_t lb,
                                           uint32_t d) {
    uint32_t lo = d > lb ? d - lb : 0u, hi = d < la ? d : la;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (A[mid - 1] <= B[d - mid]) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Segment bounds of the runs for the local sorts: i*N clipped to n.
__global__ void k_run_offsets(int64_t* __restrict__ off, uint32_t p, uint64_t N, uint64_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= p) {
        const uint64_t o = (uint64_t)i * N;
        off[i] = (int64_t)(o < n ? o : n);
    }
}

// cr[q (nch + 1) + c] = co-rank of output min(c MS_C, 2N) of pair q.
__global__ void k_corank(const uint32_t* __restrict__ src, uint32_t N, Stage s, uint32_t nch,
                         uint32_t* __restrict__ cr) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= s.pairs * (nch + 1)) return;
    const uint32_t q = t / (nch + 1), c = t - q * (nch + 1);
    uint32_t a, b;
    bool asc;
    pair_of(s, q, a, b, asc);
    const uint64_t d = (uint64_t)c * MS_C;
    const uint32_t dd = (uint32_t)(d < 2ull * N ? d : 2ull * N);
    cr[t] = corank(src + (size_t)a * N, N, src + (size_t)b * N, N, dd);
}

// One chunk of one pair's merge-split: outputs [d0, d1) of the merged pair;
// output o < N is position o of the run keeping the smaller half, o >= N
// position o - N of the other.  Only positions below `limit` are written
// (the last stage writes the caller's n keys).
__global__ __launch_bounds__(MS_NT) void k_merge_split(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                       uint32_t N, uint64_t limit, Stage s, uint32_t nch,
                                                       const uint32_t* __restrict__ cr) {
    __shared__ uint32_t sm[MS_C];
    const uint32_t tid = threadIdx.x;
    const uint32_t q = blockIdx.x / nch, c = blockIdx.x - q * nch;
    uint32_t a, b;
    bool asc;
    pair_of(s, q, a, b, asc);
    const uint32_t d0 = c * MS_C;
    const uint32_t d1 = 2 * N - d0 < MS_C ? 2 * N : d0 + MS_C;
    const uint32_t x0 = cr[q * (nch + 1) + c], x1 = cr[q * (nch + 1) + c + 1];
    const uint32_t la = x1 - x0, lb = (d1 - x1) - (d0 - x0), L = d1 - d0;
    const uint32_t* __restrict__ A = src + (size_t)a * N + x0;
    const uint32_t* __restrict__ B = src + (size_t)b * N + (d0 - x0);
    // the chunk's L = la + lb inputs, A's slice then B's, all loads in flight
    {
        uint32_t v[MS_ITEMS];
#pragma unroll
        for (int r = 0; r < MS_ITEMS; ++r) {
            const uint32_t i = r * MS_NT + tid;
            v[r] = i < la ? A[i] : (i < L ? B[i - la] : 0u);
        }
#pragma unroll
        for (int r = 0; r < MS_ITEMS; ++r) {
            const uint32_t i = r * MS_NT + tid;
            if (i < L) sm[i] = v[r];
        }
    }
    __syncthreads();
    uint32_t v[MS_ITEMS];
    const uint32_t dt = tid * MS_ITEMS;
    if (dt < L) {
        uint32_t x = corank(sm, la, sm + la, lb, dt);
        uint32_t y = dt - x;
#pragma unroll
        for (int r = 0; r < MS_ITEMS; ++r) {
            if (dt + r < L) {
                const bool from_a = y >= lb || (x < la && sm[x] <= sm[la + y]);
                v[r] = from_a ? sm[x++] : sm[la + y++];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < MS_ITEMS; ++r)
        if (dt + r < L) sm[dt + r] = v[r];
    __syncthreads();
    const uint32_t lo_run = asc ? a : b, hi_run = asc ? b : a;
    for (uint32_t i = tid; i < L; i += MS_NT) {
        const uint32_t o = d0 + i;
        const uint64_t g = o < N ? (uint64_t)lo_run * N + o : (uint64_t)hi_run * N + (o - N);
        if (g < limit) dst[g] = sm[i];
    }
}

uint32_t log2u(uint32_t p) {
    uint32_t l = 0;
    while ((1u << l) < p) ++l;
    return l;
}

}  // namespace

// The MBSP cost model of the device-scale networks (Section 3, Eqs. TbG and
// ToG, a processor read as a workgroup).  Defaults: the calibration on one
// MI355X by the BTN runs themselves -- a run's radix sort costs 68 G per key
// with G = 55 ps (stable for runs of 2^19 to 2^23 keys), and a merge-split
// stage, spread over the whole device, 1.67 ps per key of the array plus
// 17.2 us (a least-squares fit, relative error, of the BTN and OET stage
// times at 2^23, 2^25 and 2^27 keys); 512 workgroups resident.
static rs_block_model g_block_model = {3.74, 1.67, 17.2, 512};

const rs_block_model& block_model() { return g_block_model; }
void block_model_set(const rs_block_model& m) { g_block_model = m; }

double block_model_ns(const rs_block_model& m, size_t n, int algo, uint32_t p) {
    const double N = (double)((n + p - 1) / p);
    const double waves = (double)((p + (uint32_t)m.resident_runs - 1) / (uint32_t)m.resident_runs);
    const double local = m.local_ns_per_key * N * waves;
    const double stage = m.stage_ps_per_key * 1e-3 * (double)p * N + m.stage_fixed_us * 1e3;
    return local + (double)block_stages(algo, p) * stage;
}

uint32_t block_default_p(size_t n, int algo) {
    // candidates: 2 <= p <= 4096, at least 64 keys per run (p = 2 always),
    // powers of two for BTN; the model's minimum, the smaller p on a tie
    uint64_t pmax = n / 64;
    if (pmax > 4096) pmax = 4096;
    if (pmax < 2) pmax = 2;
    const rs_block_model& m = block_model();
    uint32_t best = 2;
    double tbest = block_model_ns(m, n, algo, 2);
    for (uint32_t p = 3; p <= pmax; ++p) {
        if (algo == RS_ALGO_BTN && (p & (p - 1))) continue;
        const double t = block_model_ns(m, n, algo, p);
        if (t < tbest) {
            tbest = t;
            best = p;
        }
    }
    return best;
}

bool block_plan(size_t n, int algo, uint32_t p, BlockPlan* bp) {
    if (algo != RS_ALGO_BTN && algo != RS_ALGO_OET) return false;
    if (p < 2 || p > 4096 || n == 0) return false;
    if (algo == RS_ALGO_BTN && (p & (p - 1))) return false;
    BlockPlan q;
    q.p = p;
    q.N = (n + p - 1) / p;
    if ((uint64_t)p * q.N >= (1ull << 32)) return false;  // 32-bit positions
    q.nch = (uint32_t)((2 * q.N + MS_C - 1) / MS_C);
    // one workgroup per run: the local sort of the paper's processors
    if (!seg_plan(p, (int64_t)n, &q.seg, false)) return false;
    size_t off = 0;
    q.off_seg = off;
    off += align_up(q.seg.total);
    q.off_off = off;
    off += align_up(sizeof(int64_t) * (p + 1));
    q.off_x = off;
    off += align_up(sizeof(uint32_t) * (size_t)p * q.N);
    q.off_y = off;
    off += align_up(sizeof(uint32_t) * (size_t)p * q.N);
    q.off_cr = off;
    off += align_up(sizeof(uint32_t) * (size_t)(p / 2 + 1) * (q.nch + 1));
    q.total = off;
    *bp = q;
    return true;
}

int64_t block_stages(int algo, uint32_t p) {
    const int64_t lg = log2u(p);
    return algo == RS_ALGO_BTN ? lg * (lg + 1) / 2 : (int64_t)p;
}

rs_status block_run(const BlockPlan& bp, int algo, const uint32_t* in, uint32_t* out, size_t n,
                    const SegTable& table, void* ws_, hipStream_t st) {
    unsigned char* ws = static_cast<unsigned char*>(ws_);
    const uint32_t p = bp.p, N = (uint32_t)bp.N;
    const uint64_t pn = (uint64_t)p * N;
    int64_t* off = reinterpret_cast<int64_t*>(ws + bp.off_off);
    uint32_t* X = reinterpret_cast<uint32_t*>(ws + bp.off_x);
    uint32_t* Y = reinterpret_cast<uint32_t*>(ws + bp.off_y);
    uint32_t* cr = reinterpret_cast<uint32_t*>(ws + bp.off_cr);

    // local sorts: run i = keys [i N, (i+1) N) of the input, one workgroup each
    hipLaunchKernelGGL(k_run_offsets, dim3((p + 256) / 256), dim3(256), 0, st, off, p, (uint64_t)N, (uint64_t)n);
    rs_status rc = launch_status();
    if (rc != RS_OK) return rc;
    if ((rc = seg_run(bp.seg, in, X, off, p, (int64_t)n, table, ws + bp.off_seg, st)) != RS_OK) return rc;
    if (pn > n && (rc = fill_u32(X + n, pn - n, 0xFFFFFFFFu, st)) != RS_OK) return rc;

    // the network's stages, alternating between X and Y; the last writes out
    std::vector<Stage> stages;
    if (algo == RS_ALGO_BTN) {
        for (uint32_t k = 2; k <= p; k <<= 1)
            for (uint32_t j = k >> 1; j >= 1; j >>= 1) stages.push_back(Stage{0u, k, log2u(j), 0u, p / 2});
    } else {
        for (uint32_t t = 0; t < p; ++t) stages.push_back(Stage{1u, 0u, 0u, t & 1u, (p - (t & 1u)) / 2});
    }
    const uint32_t* src = X;
    for (size_t i = 0; i < stages.size(); ++i) {
        const Stage& s = stages[i];
        const bool last = i + 1 == stages.size();
        uint32_t* dst = last ? out : (src == X ? Y : X);
        const uint64_t limit = last ? (uint64_t)n : pn;
        prof(st, KID_BLOCK_MERGE, 0);
        if (s.pairs) {
            const uint64_t nb = (uint64_t)s.pairs * (bp.nch + 1);
            hipLaunchKernelGGL(k_corank, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, src, N, s, bp.nch, cr);
            hipLaunchKernelGGL(k_merge_split, dim3(s.pairs * bp.nch), dim3(MS_NT), 0, st, src, dst, N, limit, s,
                               bp.nch, cr);
        }
        // OET: the runs no pair of this round holds move unchanged
        if (s.oet) {
            const uint32_t first_free = s.parity ? 0u : p;          // run 0 when the pairs start at 1
            const uint32_t last_free = ((p - s.parity) & 1u) ? p - 1 : p;
            for (uint32_t r : {first_free, last_free}) {
                if (r >= p || (uint64_t)r * N >= limit) continue;
                const uint64_t m = limit - (uint64_t)r * N < N ? limit - (uint64_t)r * N : N;
                hipError_t e = hipMemcpyAsync(dst + (size_t)r * N, src + (size_t)r * N, m * sizeof(uint32_t),
                                              hipMemcpyDeviceToDevice, st);
                if (e != hipSuccess) return hip_fail(e);
            }
        }
        prof(st, KID_BLOCK_MERGE, 1);
        if ((rc = launch_status()) != RS_OK) return rc;
        src = dst;
    }
    return RS_OK;
}

}  // namespace rs
