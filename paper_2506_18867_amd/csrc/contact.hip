// contact.hip -- conversion of contact Hessians and gradients from the triangle contact mesh
// embedded in the B-spline surface to the control points (Sec. 4.3, contact barrier, Eq.
// "gradient and hessian of contact barrier"; Sec. 5.2, Alg. "Contact Hessian conversion and
// assembly").
//
// Mesh vertex a sits at fixed parametric coordinates, so x_a = sum_m w_a[m] C^{i(a,m)} over the
// 9 CPs of the span it lies in (Eq. "trig mesh node from control points"). By the chain rule the
// CP Hessian block (i, j) is sum over vertex pairs (a, b) of w_a[m] w_b[m'] H(a, b), and the CP
// gradient i is sum_a w_a[m] g_a. The paper builds this on the CPU with hash maps filled per
// spatial block (to limit write conflicts). Here both levels are a sort by key plus a segmented
// sum, with no atomics and a fixed summation order (results are bitwise reproducible):
//   1. expand every contact pair into its (vertex, vertex) block entries, radix-sort them by the
//      vertex pair, run-length encode, and sum each run: the vertex-level Hessian H_lin;
//   2. expand every distinct vertex pair into the CP pairs of its two 3x3 CP supports (weight
//      products that are exactly zero are skipped), radix-sort by CP pair, run-length encode, and
//      sum each run w_a[m] w_b[m'] H_lin: the CP-level blocks, already in CSR order;
//   3. row pointers by binary search over the sorted CP-pair keys; the gradient as a gather over
//      the vertices of the 3x3 spans around each CP.
#include <cstring>
#include <rocprim/rocprim.hpp>

#include "bsc_internal.h"

namespace bsc {
namespace {

typedef unsigned long long u64;
typedef unsigned int u32;

constexpr int kCtBlock = 256;

inline unsigned bit_width(u64 v) {
    unsigned b = 0;
    while (v) { ++b; v >>= 1; }
    return b;
}

// Step 1 expansion: entry t = 16 c + 4 s + s' for slots s, s' of pair c. Key (a << vbits) | b,
// or the sentinel (all used bits set, sorted after every valid key) for unused slots.
// Out-of-range vertex indices raise the error flag and are skipped.
__global__ void k_ct_expand_v(int n_pairs, int n_vert, unsigned vbits, const int32_t *__restrict__ verts, u64 sent,
                              u64 *__restrict__ key, u32 *__restrict__ val, int32_t *__restrict__ flag) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 16 * n_pairs) return;
    const int c = t >> 4, s = (t >> 2) & 3, s2 = t & 3;
    const int va = verts[4 * c + s], vb = verts[4 * c + s2];
    const bool bad = va < -1 || vb < -1 || va >= n_vert || vb >= n_vert;
    if (bad) atomicOr(flag, 1);
    const bool ok = !bad && va >= 0 && vb >= 0;
    key[t] = ok ? (u64(va) << vbits) | u64(vb) : sent;
    val[t] = u32(t);
}

__global__ void k_ct_zero(double *__restrict__ p, size_t n) {
    const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

// Step 1 sums: one thread per distinct vertex pair u, summing the 3x3 blocks of its run in the
// sorted (stable, hence original) order. Also records the pair's vertices and its span-pair key
// (e_a << ebits) | e_b, and, for the diagonal pair (a, a), the pair gradients of the slots
// holding a.
__global__ void k_ct_vpair_sum(int n1, unsigned vbits, unsigned ebits, const u64 *__restrict__ ukey, const u32 *__restrict__ cnt,
                               const u32 *__restrict__ off, const u32 *__restrict__ val, const double *__restrict__ pair_hess,
                               const double *__restrict__ pair_grad, const int32_t *__restrict__ vspan, double *__restrict__ hlin,
                               int32_t *__restrict__ pa, int32_t *__restrict__ pb, u64 *__restrict__ spkey, u32 *__restrict__ spval,
                               double *__restrict__ glin) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n1) return;
    double h[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, g[3] = {0, 0, 0};
    const u32 o = off[u], n = cnt[u];
    for (u32 q = o; q < o + n; ++q) {
        const u32 t = val[q];
        const int c = int(t >> 4), s = int((t >> 2) & 3), s2 = int(t & 3);
        const double *H = pair_hess + size_t(c) * 144;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) h[3 * r + k] += H[(3 * s + r) * 12 + 3 * s2 + k];
        if (pair_grad && s == s2) {
#pragma unroll
            for (int r = 0; r < 3; ++r) g[r] += pair_grad[size_t(c) * 12 + 3 * s + r];
        }
    }
#pragma unroll
    for (int r = 0; r < 9; ++r) hlin[size_t(u) * 9 + r] = h[r];
    const u64 k = ukey[u];
    const int a = int(k >> vbits), b = int(k & ((u64(1) << vbits) - 1));
    pa[u] = a;
    pb[u] = b;
    spkey[u] = (u64(vspan[a]) << ebits) | u64(vspan[b]);
    spval[u] = u32(u);
    if (pair_grad && a == b) {
#pragma unroll
        for (int r = 0; r < 3; ++r) glin[size_t(a) * 3 + r] = g[r];
    }
}

// Vertex-pair data in span-pair order (so that the vertex pairs of one span pair are contiguous).
__global__ void k_ct_permute(int n1, const u32 *__restrict__ spv, const double *__restrict__ hlin, const int32_t *__restrict__ pa,
                             const int32_t *__restrict__ pb, double *__restrict__ hsp, int32_t *__restrict__ pas,
                             int32_t *__restrict__ pbs) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n1) return;
    const u32 v = spv[r];
#pragma unroll
    for (int e = 0; e < 9; ++e) hsp[size_t(r) * 9 + e] = hlin[size_t(v) * 9 + e];
    pas[r] = pa[v];
    pbs[r] = pb[v];
}

// Step 2 expansion: entry t = 81 w + 9 m + m' for the CPs m, m' of the two spans of span pair w.
// Valid only if some vertex pair of the span pair has a nonzero weight product there.
template <typename K>
__global__ void k_ct_expand_cp(int n2, unsigned ebits, unsigned cbits, int n_u, int Nu, const u64 *__restrict__ ukeysp,
                               const u32 *__restrict__ cntsp, const u32 *__restrict__ offsp, const int32_t *__restrict__ pas,
                               const int32_t *__restrict__ pbs, const double *__restrict__ vw, K sent, K *__restrict__ key,
                               u32 *__restrict__ val) {
    const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= size_t(n2) * 81) return;
    const int w = int(t / 81), mm = int(t % 81), m = mm / 9, m2 = mm % 9;
    bool nz = false;
    const u32 o = offsp[w], n = cntsp[w];
    for (u32 q = o; q < o + n && !nz; ++q) nz = vw[size_t(pas[q]) * 9 + m] * vw[size_t(pbs[q]) * 9 + m2] != 0.0;
    const u64 k = ukeysp[w];
    const int ea = int(k >> ebits), eb = int(k & ((u64(1) << ebits) - 1));
    const int i = (ea / Nu + m / 3) * n_u + (ea % Nu + m % 3);
    const int j = (eb / Nu + m2 / 3) * n_u + (eb % Nu + m2 % 3);
    key[t] = nz ? (K(i) << cbits) | K(j) : sent;
    val[t] = u32(t);
}

// Step 2 sums: a group of kCtLanes lanes per CP block. Lane l takes the entries l, l + kCtLanes,
// ... of the block's run (each entry sums over the vertex pairs of its span pair in their sorted
// order), then the group adds its lanes in a fixed tree. The order depends only on the run, so
// the result is reproducible; the lanes hide the latency of the dependent loads of each entry.
constexpr int kCtLanes = 8;

template <typename K>
__global__ void __launch_bounds__(kCtBlock) k_ct_cpair_sum(int nnzb, unsigned cbits, const K *__restrict__ ukey2,
                                                           const u32 *__restrict__ cnt2, const u32 *__restrict__ off2,
                                                           const u32 *__restrict__ val2, const u32 *__restrict__ cntsp,
                                                           const u32 *__restrict__ offsp, const int32_t *__restrict__ pas,
                                                           const int32_t *__restrict__ pbs, const double *__restrict__ vw,
                                                           const double *__restrict__ hsp,
                                                           int32_t *__restrict__ col, double *__restrict__ out) {
    const int gid = int((size_t(blockIdx.x) * blockDim.x + threadIdx.x) / kCtLanes);
    const int lane = threadIdx.x % kCtLanes;
    const bool live = gid < nnzb;
    double h[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (live) {
        const u32 o = off2[gid], n = cnt2[gid];
        for (u32 q = o + lane; q < o + n; q += kCtLanes) {
            const u32 t = val2[q];
            const int w = int(t / 81), mm = int(t % 81), m = mm / 9, m2 = mm % 9;
            const u32 o2 = offsp[w], n2 = cntsp[w];
            for (u32 r = o2; r < o2 + n2; ++r) {
                const double wt = vw[size_t(pas[r]) * 9 + m] * vw[size_t(pbs[r]) * 9 + m2];
                const double *H = hsp + size_t(r) * 9;
#pragma unroll
                for (int e = 0; e < 9; ++e) h[e] += wt * H[e];
            }
        }
    }
#pragma unroll
    for (int d = kCtLanes / 2; d > 0; d >>= 1)
#pragma unroll
        for (int e = 0; e < 9; ++e) h[e] += __shfl_xor(h[e], d, kCtLanes);
    if (live && lane == 0) {
        col[gid] = int32_t(ukey2[gid] & ((K(1) << cbits) - 1));
#pragma unroll
        for (int r = 0; r < 9; ++r) out[size_t(gid) * 9 + r] = h[r];
    }
}

// CSR row pointers: row_ptr[i] = first block whose row is >= i (lower bound over sorted keys).
template <typename K>
__global__ void k_ct_rowptr(int n_cp, int nnzb, unsigned cbits, const K *__restrict__ ukey2, int32_t *__restrict__ row_ptr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n_cp) return;
    const K target = K(i) << cbits;
    int lo = 0, hi = nnzb;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ukey2[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    row_ptr[i] = lo;
}

// CP gradient: gather over the vertices of the (up to) 3x3 spans whose CP set holds CP i.
__global__ void k_ct_grad(int n_u, int n_v, int Nu, int Nv, const int32_t *__restrict__ voff, const int32_t *__restrict__ vlist,
                          const double *__restrict__ vw, const double *__restrict__ glin, double *__restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_cp = n_u * n_v;
    if (i >= n_cp) return;
    const int ci = i % n_u, cj = i / n_u;
    double g[3] = {0.0, 0.0, 0.0};
    for (int l = max(0, cj - 2); l <= min(cj, Nv - 1); ++l)
        for (int k = max(0, ci - 2); k <= min(ci, Nu - 1); ++k) {
            const int e = l * Nu + k, m = 3 * (cj - l) + (ci - k);
            for (int q = voff[e]; q < voff[e + 1]; ++q) {
                const int a = vlist[q];
                const double w = vw[size_t(a) * 9 + m];
#pragma unroll
                for (int r = 0; r < 3; ++r) g[r] += w * glin[size_t(a) * 3 + r];
            }
        }
#pragma unroll
    for (int r = 0; r < 3; ++r) grad[size_t(r) * n_cp + i] = g[r];
}

inline unsigned grid(size_t n) { return unsigned((n + kCtBlock - 1) / kCtBlock); }

// Key widths: vertex pairs (a << vbits) | b; span pairs (e_a << ebits) | e_b; CP pairs
// (i << cbits) | j, held in 32 bits when they fit.
struct CtBits {
    unsigned vbits, ebits, cbits;
    bool cp32;
};
inline CtBits ct_bits(const bsc_ctx *c) {
    CtBits b;
    // bit_width(n) > bit_width(n - 1) when n is a power of two: indices stay below the all-ones
    // pattern, so the sentinel key (all used bits set) never equals a valid key
    b.vbits = bit_width(u64(c->ct_nvert));
    b.ebits = bit_width(u64(c->n_elem));
    b.cbits = bit_width(u64(c->n_cp));
    b.cp32 = 2 * b.cbits <= 32;
    return b;
}

// Step 2 (span pairs onward) for the CP-key type K. Returns the block count in *nnzb.
template <typename K>
bsc_status ct_step2(bsc_ctx *c, int n1, const CtBits &bits, int32_t cap_blocks, int32_t *d_col_idx, double *d_vals,
                    int32_t *d_row_ptr, int *nnzb_out) {
    const ContactBufs &B = c->ct;
    hipStream_t st = c->stream;
    auto ok = [&](hipError_t e, const char *what) { return hip_check(c, e, what); };
    bsc_status s;
    size_t tb;
    u32 host_small[4] = {0, 0, 0, 0};
    K *key2a = (K *)B.key2a, *key2b = (K *)B.key2b, *ukey2 = (K *)B.ukey2;
    const K sent2 = K((u64(1) << (2 * bits.cbits)) - 1);
    int nnzb = 0;
    if (n1 > 0) {
        // 2a. vertex pairs grouped by span pair
        tb = B.tmp_bytes;
        if ((s = ok(rocprim::radix_sort_pairs(B.tmp, tb, B.spk, B.spk_s, B.spv, B.spv_s, unsigned(n1), 0, 2 * bits.ebits, st),
                    "contact sort span pairs")) != BSC_OK) return s;
        tb = B.tmp_bytes;
        if ((s = ok(rocprim::run_length_encode(B.tmp, tb, B.spk_s, unsigned(n1), B.uksp, B.cntsp, B.small + 3, st),
                    "contact runs span pairs")) != BSC_OK) return s;
        if ((s = ok(hipMemcpyAsync(host_small, B.small, 16, hipMemcpyDeviceToHost, st), "contact read 2a")) != BSC_OK) return s;
        if ((s = ok(hipStreamSynchronize(st), "contact sync 2a")) != BSC_OK) return s;
        const int n2 = int(host_small[3]);
        tb = B.tmp_bytes;
        if ((s = ok(rocprim::exclusive_scan(B.tmp, tb, B.cntsp, B.offsp, u32(0), size_t(n2), rocprim::plus<u32>(), st),
                    "contact scan span pairs")) != BSC_OK) return s;
        k_ct_permute<<<grid(n1), kCtBlock, 0, st>>>(n1, B.spv_s, B.hlin, B.pa, B.pb, B.hsp, B.pas, B.pbs);
        if ((s = ok(hipGetLastError(), "contact permute")) != BSC_OK) return s;
        // 2b. CP-pair entries, sorted; runs
        const unsigned e2 = 81u * unsigned(n2);
        k_ct_expand_cp<K><<<grid(e2), kCtBlock, 0, st>>>(n2, bits.ebits, bits.cbits, c->n_u, c->Nu, B.uksp, B.cntsp, B.offsp,
                                                         B.pas, B.pbs, B.vw, sent2, key2a, B.val2a);
        if ((s = ok(hipGetLastError(), "contact expand 2")) != BSC_OK) return s;
        tb = B.tmp_bytes;
        if ((s = ok(rocprim::radix_sort_pairs(B.tmp, tb, key2a, key2b, B.val2a, B.val2b, e2, 0, 2 * bits.cbits, st),
                    "contact sort 2")) != BSC_OK) return s;
        tb = B.tmp_bytes;
        if ((s = ok(rocprim::run_length_encode(B.tmp, tb, key2b, e2, ukey2, B.cnt2, B.small + 1, st), "contact runs 2")) != BSC_OK)
            return s;
        if ((s = ok(hipMemcpyAsync(host_small, B.small, 16, hipMemcpyDeviceToHost, st), "contact read 2")) != BSC_OK) return s;
        if ((s = ok(hipStreamSynchronize(st), "contact sync 2")) != BSC_OK) return s;
        nnzb = int(host_small[1]);
        K last = 0;
        if (nnzb > 0) {
            if ((s = ok(hipMemcpy(&last, ukey2 + (nnzb - 1), sizeof(K), hipMemcpyDeviceToHost), "contact read last")) != BSC_OK)
                return s;
            if (last == sent2) --nnzb;
        }
        if (nnzb > cap_blocks) {
            *nnzb_out = nnzb;
            return fail(c, BSC_E_NOMEM, "more CP blocks than cap_blocks (nnzb holds the count needed)");
        }
        if (nnzb > 0) {
            // 2c. sums
            tb = B.tmp_bytes;
            if ((s = ok(rocprim::exclusive_scan(B.tmp, tb, B.cnt2, B.off2, u32(0), size_t(nnzb), rocprim::plus<u32>(), st),
                        "contact scan 2")) != BSC_OK) return s;
            k_ct_cpair_sum<K><<<grid(size_t(nnzb) * kCtLanes), kCtBlock, 0, st>>>(
                nnzb, bits.cbits, ukey2, B.cnt2, B.off2, B.val2b, B.cntsp, B.offsp, B.pas, B.pbs, B.vw, B.hsp, d_col_idx, d_vals);
            if ((s = ok(hipGetLastError(), "contact sum 2")) != BSC_OK) return s;
        }
    }
    k_ct_rowptr<K><<<grid(size_t(c->n_cp) + 1), kCtBlock, 0, st>>>(c->n_cp, nnzb, bits.cbits, ukey2, d_row_ptr);
    if ((s = ok(hipGetLastError(), "contact row pointers")) != BSC_OK) return s;
    *nnzb_out = nnzb;
    return BSC_OK;
}

template <typename K>
size_t sort_tmp(unsigned n) {
    size_t s = 0, need = 0;
    const K *k = nullptr;
    K *ko = nullptr;
    const u32 *v = nullptr;
    u32 *vo = nullptr;
    (void)rocprim::radix_sort_pairs(nullptr, s, k, ko, v, vo, n, 0, 8 * unsigned(sizeof(K)), hipStream_t(0));
    need = std::max(need, s);
    s = 0;
    (void)rocprim::run_length_encode(nullptr, s, k, n, ko, vo, vo, hipStream_t(0));
    need = std::max(need, s);
    s = 0;
    (void)rocprim::exclusive_scan(nullptr, s, v, vo, u32(0), size_t(n), rocprim::plus<u32>(), hipStream_t(0));
    return std::max(need, s);
}

}  // namespace

// Layout of the contact workspace; base == nullptr only sizes it.
size_t contact_layout(const bsc_ctx *c, ContactBufs *b, char *base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += (bytes + 255) & ~size_t(255);
        return p;
    };
    const size_t nv = c->ct_nvert, e1 = size_t(16) * c->ct_max_pairs, u1 = c->ct_max_vpairs, e2 = size_t(81) * u1;
    ContactBufs t{};
    t.vspan = (int32_t *)take(4 * nv);
    t.vw = (double *)take(72 * nv);
    t.voff = (int32_t *)take(4 * (size_t(c->n_elem) + 1));
    t.vlist = (int32_t *)take(4 * nv);
    t.key1a = (u64 *)take(8 * e1);
    t.key1b = (u64 *)take(8 * e1);
    t.val1a = (u32 *)take(4 * e1);
    t.val1b = (u32 *)take(4 * e1);
    t.ukey1 = (u64 *)take(8 * e1);
    t.cnt1 = (u32 *)take(4 * e1);
    t.off1 = (u32 *)take(4 * e1);
    t.hlin = (double *)take(72 * u1);
    t.hsp = (double *)take(72 * u1);
    t.pas = (int32_t *)take(4 * u1);
    t.pbs = (int32_t *)take(4 * u1);
    t.pa = (int32_t *)take(4 * u1);
    t.pb = (int32_t *)take(4 * u1);
    t.spk = (u64 *)take(8 * u1);
    t.spk_s = (u64 *)take(8 * u1);
    t.spv = (u32 *)take(4 * u1);
    t.spv_s = (u32 *)take(4 * u1);
    t.uksp = (u64 *)take(8 * u1);
    t.cntsp = (u32 *)take(4 * u1);
    t.offsp = (u32 *)take(4 * u1);
    t.glin = (double *)take(24 * nv);
    t.key2a = (u64 *)take(8 * e2);
    t.key2b = (u64 *)take(8 * e2);
    t.val2a = (u32 *)take(4 * e2);
    t.val2b = (u32 *)take(4 * e2);
    t.ukey2 = (u64 *)take(8 * e2);
    t.cnt2 = (u32 *)take(4 * e2);
    t.off2 = (u32 *)take(4 * e2);
    t.small = (u32 *)take(256);                     // [0] runs 1, [1] runs 2, [2] error flag, [3] span-pair runs
    t.tmp = take(c->ct_tmp_bytes);
    t.tmp_bytes = c->ct_tmp_bytes;
    if (b) *b = t;
    return off;
}

// Temporary storage that the sorts, run-length encodings and scans need at the largest sizes.
size_t contact_tmp_bytes(int max_pairs, int max_vpairs) {
    const unsigned e1 = unsigned(16 * max_pairs), u1 = unsigned(max_vpairs), e2 = 81u * u1;
    size_t need = std::max(sort_tmp<u64>(e1), sort_tmp<u64>(u1));
    need = std::max(need, std::max(sort_tmp<u64>(e2), sort_tmp<u32>(e2)));
    return need + 256;
}

}  // namespace bsc

using namespace bsc;

extern "C" {

bsc_status bsc_contact_setup(bsc_ctx *c, int32_t n_vert, const double *uv, int32_t max_pairs, int32_t max_vpairs) {
    if (!c) return BSC_E_INVAL;
    if (n_vert < 1 || !uv || max_pairs < 1 || max_pairs > (1 << 20) || max_vpairs < 0)
        return fail(c, BSC_E_INVAL, "bad contact-mesh sizes");
    if (max_vpairs == 0) max_vpairs = 16 * max_pairs;
    if (int64_t(max_vpairs) * 81 >= (int64_t(1) << 31) || int64_t(n_vert) * n_vert >= (int64_t(1) << 62))
        return fail(c, BSC_E_INVAL, "contact capacities too large");
    const double Lu = c->hu * c->Nu, Lv = c->hv * c->Nv;
    std::vector<int32_t> span(n_vert);
    std::vector<double> w(size_t(9) * n_vert);
    for (int a = 0; a < n_vert; ++a) {
        const double u = uv[2 * a], v = uv[2 * a + 1];
        if (!(u >= 0.0 && u <= Lu && v >= 0.0 && v <= Lv)) return fail(c, BSC_E_INVAL, "contact vertex outside the parameter rectangle");
        const double su = u / c->hu, sv = v / c->hv;      // span units
        const int k = std::min(int(std::floor(su)), c->Nu - 1), l = std::min(int(std::floor(sv)), c->Nv - 1);
        double Nu3[3], Nv3[3], D[3], D2[3];
        host_pieces(k == 0 ? 0 : (k == c->Nu - 1 ? 2 : 1), su - k, Nu3, D, D2);
        host_pieces(l == 0 ? 0 : (l == c->Nv - 1 ? 2 : 1), sv - l, Nv3, D, D2);
        span[a] = l * c->Nu + k;
        for (int b = 0; b < 3; ++b)
            for (int aa = 0; aa < 3; ++aa) w[size_t(a) * 9 + 3 * b + aa] = Nu3[aa] * Nv3[b];
    }
    // vertices grouped by span (for the gradient gather)
    std::vector<int32_t> voff(c->n_elem + 1, 0), vlist(n_vert);
    for (int a = 0; a < n_vert; ++a) voff[span[a] + 1]++;
    for (int e = 0; e < c->n_elem; ++e) voff[e + 1] += voff[e];
    std::vector<int32_t> cur(voff.begin(), voff.end() - 1);
    for (int a = 0; a < n_vert; ++a) vlist[cur[span[a]]++] = a;
    c->ct_nvert = n_vert;
    c->ct_max_pairs = max_pairs;
    c->ct_max_vpairs = max_vpairs;
    c->ct_span.swap(span);
    c->ct_w.swap(w);
    c->ct_voff.swap(voff);
    c->ct_vlist.swap(vlist);
    c->ct_tmp_bytes = contact_tmp_bytes(max_pairs, max_vpairs);
    c->ct_ws = nullptr;
    c->ct_ws_bytes = 0;
    return BSC_OK;
}

bsc_status bsc_contact_workspace_size(const bsc_ctx *c, size_t *bytes) {
    if (!c || !bytes) return BSC_E_INVAL;
    if (c->ct_nvert == 0) return BSC_E_STATE;
    *bytes = contact_layout(c, nullptr, nullptr);
    return BSC_OK;
}

bsc_status bsc_contact_bind_workspace(bsc_ctx *c, void *d_ws, size_t bytes) {
    if (!c || !d_ws) return BSC_E_INVAL;
    if (c->ct_nvert == 0) return fail(c, BSC_E_STATE, "call bsc_contact_setup first");
    if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0) return fail(c, BSC_E_INVAL, "workspace must be 256-byte aligned");
    if (bytes < contact_layout(c, nullptr, nullptr)) return fail(c, BSC_E_NOMEM, "contact workspace too small");
    ContactBufs &B = c->ct;
    contact_layout(c, &B, (char *)d_ws);
    struct Up { void *dst; const void *src; size_t n; } ups[] = {
        {B.vspan, c->ct_span.data(), 4 * c->ct_span.size()}, {B.vw, c->ct_w.data(), 8 * c->ct_w.size()},
        {B.voff, c->ct_voff.data(), 4 * c->ct_voff.size()}, {B.vlist, c->ct_vlist.data(), 4 * c->ct_vlist.size()},
    };
    for (const Up &u : ups) {
        bsc_status st = hip_check(c, hipMemcpyAsync(u.dst, u.src, u.n, hipMemcpyHostToDevice, c->stream), "upload contact tables");
        if (st != BSC_OK) return st;
    }
    bsc_status st = hip_check(c, hipStreamSynchronize(c->stream), "bind contact workspace");
    if (st != BSC_OK) return st;
    c->ct_ws = (char *)d_ws;
    c->ct_ws_bytes = bytes;
    return BSC_OK;
}

bsc_status bsc_contact_hessian(bsc_ctx *c, int32_t n_pairs, const int32_t *d_pair_verts, const double *d_pair_hess,
                               const double *d_pair_grad, int32_t cap_blocks, int32_t *d_row_ptr, int32_t *d_col_idx,
                               double *d_vals, int32_t *nnzb_out, double *d_grad) {
    if (!c || !nnzb_out) return BSC_E_INVAL;
    *nnzb_out = 0;
    if (!c->ct_ws) return fail(c, BSC_E_STATE, "bind a contact workspace first");
    if (n_pairs < 0 || n_pairs > c->ct_max_pairs) return fail(c, BSC_E_INVAL, "n_pairs outside [0, max_pairs]");
    if (cap_blocks < 0 || !d_row_ptr || (n_pairs > 0 && (!d_pair_verts || !d_pair_hess)) ||
        (cap_blocks > 0 && (!d_col_idx || !d_vals)))
        return fail(c, BSC_E_INVAL, "null or negative argument");
    const ContactBufs &B = c->ct;
    hipStream_t st = c->stream;
    const int n_vert = c->ct_nvert;
    const CtBits bits = ct_bits(c);
    const u64 sent1 = (u64(1) << (2 * bits.vbits)) - 1;
    size_t tb = B.tmp_bytes;
    auto ok = [&](hipError_t e, const char *what) { return hip_check(c, e, what); };
    bsc_status s;
    u32 host_small[4] = {0, 0, 0, 0};

    // vertex gradients start at zero (vertices in no contact keep zero)
    if (d_grad) {
        k_ct_zero<<<grid(size_t(3) * n_vert), kCtBlock, 0, st>>>(B.glin, size_t(3) * n_vert);
        if ((s = ok(hipGetLastError(), "contact zero")) != BSC_OK) return s;
    }
    if ((s = ok(hipMemsetAsync(B.small, 0, 16, st), "contact flags")) != BSC_OK) return s;
    int n1 = 0;
    if (n_pairs > 0) {
        // 1. vertex-pair entries, sorted; runs; sums
        const unsigned e1 = unsigned(16 * n_pairs);
        k_ct_expand_v<<<grid(e1), kCtBlock, 0, st>>>(n_pairs, n_vert, bits.vbits, d_pair_verts, sent1, B.key1a, B.val1a,
                                                     (int32_t *)(B.small + 2));
        if ((s = ok(hipGetLastError(), "contact expand 1")) != BSC_OK) return s;
        tb = B.tmp_bytes;
        if ((s = ok(rocprim::radix_sort_pairs(B.tmp, tb, B.key1a, B.key1b, B.val1a, B.val1b, e1, 0, 2 * bits.vbits, st),
                    "contact sort 1")) != BSC_OK) return s;
        tb = B.tmp_bytes;
        if ((s = ok(rocprim::run_length_encode(B.tmp, tb, B.key1b, e1, B.ukey1, B.cnt1, B.small, st), "contact runs 1")) != BSC_OK)
            return s;
        if ((s = ok(hipMemcpyAsync(host_small, B.small, 16, hipMemcpyDeviceToHost, st), "contact read 1")) != BSC_OK) return s;
        if ((s = ok(hipStreamSynchronize(st), "contact sync 1")) != BSC_OK) return s;
        if (host_small[2]) return fail(c, BSC_E_INVAL, "contact pair vertex index out of range");
        n1 = int(host_small[0]);
        // the sentinel run, if any, is the last one
        u64 last = 0;
        if (n1 > 0) {
            if ((s = ok(hipMemcpy(&last, B.ukey1 + (n1 - 1), 8, hipMemcpyDeviceToHost), "contact read last")) != BSC_OK) return s;
            if (last == sent1) --n1;
        }
        if (n1 > c->ct_max_vpairs) return fail(c, BSC_E_NOMEM, "more distinct vertex pairs than max_vpairs");
        if (n1 > 0) {
            tb = B.tmp_bytes;
            if ((s = ok(rocprim::exclusive_scan(B.tmp, tb, B.cnt1, B.off1, u32(0), size_t(n1), rocprim::plus<u32>(), st),
                        "contact scan 1")) != BSC_OK) return s;
            k_ct_vpair_sum<<<grid(n1), kCtBlock, 0, st>>>(n1, bits.vbits, bits.ebits, B.ukey1, B.cnt1, B.off1, B.val1b, d_pair_hess,
                                                          d_grad ? d_pair_grad : nullptr, B.vspan, B.hlin, B.pa, B.pb, B.spk,
                                                          B.spv, B.glin);
            if ((s = ok(hipGetLastError(), "contact sum 1")) != BSC_OK) return s;
        }
    }
    int nnzb = 0;
    s = bits.cp32 ? ct_step2<u32>(c, n1, bits, cap_blocks, d_col_idx, d_vals, d_row_ptr, &nnzb)
                  : ct_step2<u64>(c, n1, bits, cap_blocks, d_col_idx, d_vals, d_row_ptr, &nnzb);
    if (s != BSC_OK) {
        *nnzb_out = nnzb;
        return s;
    }
    if (d_grad) {
        k_ct_grad<<<grid(c->n_cp), kCtBlock, 0, st>>>(c->n_u, c->n_v, c->Nu, c->Nv, B.voff, B.vlist, B.vw, B.glin, d_grad);
        if ((s = ok(hipGetLastError(), "contact gradient")) != BSC_OK) return s;
    }
    *nnzb_out = nnzb;
    return BSC_OK;
}

}  // extern "C"
