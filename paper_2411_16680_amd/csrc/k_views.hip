// k_views.hip -- render of a decoded intermediate LDM into every input view
// (Sec. 3.2.2 "Decoding and rendering the intermediate LDM", Eq. 2): the
// projection operator, the transpose of the bilinear back-projection, splats
// each layer-pixel's colour and density into the four view pixels around its
// reprojection (per layer, per view, unnormalised), then each view composites
// its projected layers front to back.
//
// Two forms.  The binned form (up to 128 layers) never writes the projected
// layers: every (view, layer-pixel) becomes a record in the bin of the view
// tile its taps reach, and one workgroup per tile adds its records into LDS
// and composites the tile (see "Binned form" below).  The planes form, for
// more layers: a fill kernel clears the projected layers (no
// hipMemsetAsync, so the call can be captured in a graph); k_splat, one
// thread per (view, layer-pixel), scatters with float atomics regrouped
// through LDS so that eight adjacent lanes add the four channels of a tap
// and of its right neighbour (32 contiguous bytes) instead of 64 lanes
// hitting 64 scattered words; k_views_composite, one thread per view pixel.
// Both forms form the same products of tap weight and payload and the same
// composite; only the order of the float additions into a view pixel
// differs.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "uf_params.h"

// multiply-adds fused within an expression only: the binned form's counting
// and writing passes evaluate the same reprojection and must round it alike
#pragma clang fp contract(on)

namespace qk {
namespace {

__global__ void __launch_bounds__(256) k_views_zero(const ViewsParams p) {
    const int64_t n4 = p.ws_floats >> 2;
    float4 *w = reinterpret_cast<float4 *>(p.ws);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256)
        w[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Per wave: 64 layer-pixels x 2 tap rows = 128 entries -- the float index
// in ws of the row's left and right taps (-1 = dropped) and their weights --
// and the 64 payloads (r, g, b, alpha).  A row's two taps are neighbours in
// the plane, so one entry is 32 contiguous bytes.
struct SplatSlice {
    int4 e[128];         // dst_left, dst_right, weight bits left, right
    float4 val[64];
};

__global__ void __launch_bounds__(256) k_splat(const ViewsParams p) {
    __shared__ SplatSlice sl[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    SplatSlice &s = sl[wave];
    // one (view, 256 layer-pixels) chunk per workgroup, views slowest, in an
    // XCD-aware order (workgroups are dispatched round-robin over the 8 XCDs:
    // workgroup i takes chunk (i % 8) * per + i / 8), so each XCD scatters
    // the rows of one layer into one view at a time and the band of the
    // view's plane those rows reach stays in its L2
    const int64_t bpv = (p.N + 255) / 256, n = bpv * p.V;
    int64_t chunk;
    {
        const int64_t i = blockIdx.x, xcd = i & 7, loc = i >> 3, q8 = n >> 3, rem = n & 7;
        chunk = (xcd < rem) ? xcd * (q8 + 1) + loc : rem * (q8 + 1) + (xcd - rem) * q8 + loc;
    }
    const int m = (int)(chunk / bpv);
    const int64_t q = (chunk - (int64_t)m * bpv) * 256 + threadIdx.x;   // layer-pixel
    const bool live = q < p.N;
    const int64_t hw = (int64_t)p.H * p.W;
    const int l = live ? (int)(q / hw) : 0;
    const int64_t r = live ? q - (int64_t)l * hw : 0;
    const int y = (int)(r / p.W), x = (int)(r - (int64_t)y * p.W);
    const double u = (double)x + 0.5, v = (double)y + 0.5;
    int4 row0 = make_int4(-1, -1, 0, 0), row1 = make_int4(-1, -1, 0, 0);
    if (live) {
        s.val[lane] = make_float4(p.color[q * 3 + 0], p.color[q * 3 + 1], p.color[q * 3 + 2],
                                  p.alpha[q]);
        const double invd = 1.0 / (double)p.depth[q];
        const double *A = p.cam[m];
        const int vw = p.vW[m], vh = p.vH[m];
        const double pz = fma(A[6], u, fma(A[7], v, fma(A[11], invd, A[8])));
        const double qx = fma(A[0], u, fma(A[1], v, fma(A[9], invd, A[2])));
        const double qy = fma(A[3], u, fma(A[4], v, fma(A[10], invd, A[5])));
        const double rz = 1.0 / pz;
        const double fxc = qx * rz - 0.5, fyc = qy * rz - 0.5;
        if ((pz > 1e-6) && (fxc > -2.0) && (fxc < (double)(vw + 1)) && (fyc > -2.0) &&
            (fyc < (double)(vh + 1))) {
            const double xf = floor(fxc), yf = floor(fyc);
            const float fx = (float)(fxc - xf), fy = (float)(fyc - yf);
            const int ix = (int)xf, iy = (int)yf;
            const int64_t base = p.sbase[m] + (int64_t)l * vh * vw * 4;
            const bool vx0 = (unsigned)ix < (unsigned)vw, vx1 = (unsigned)(ix + 1) < (unsigned)vw;
            const bool vy0 = (unsigned)iy < (unsigned)vh, vy1 = (unsigned)(iy + 1) < (unsigned)vh;
            const int64_t o0 = base + ((int64_t)iy * vw + ix) * 4, o1 = o0 + (int64_t)vw * 4;
            row0 = make_int4((vx0 && vy0) ? (int)o0 : -1, (vx1 && vy0) ? (int)o0 + 4 : -1,
                             __float_as_int((1.0f - fx) * (1.0f - fy)),
                             __float_as_int(fx * (1.0f - fy)));
            row1 = make_int4((vx0 && vy1) ? (int)o1 : -1, (vx1 && vy1) ? (int)o1 + 4 : -1,
                             __float_as_int((1.0f - fx) * fy), __float_as_int(fx * fy));
        }
    }
    s.e[2 * lane] = row0;
    s.e[2 * lane + 1] = row1;
    __syncthreads();
    // lanes 8k..8k+7 add entry 8 j + k: the left tap's four channels, then
    // the right tap's
    const int c = lane & 3, right = (lane >> 2) & 1;
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
        const int en = 8 * j + (lane >> 3);
        const int4 ent = s.e[en];
        const int d = right ? ent.y : ent.x;
        if (d >= 0) {
            const float4 pv = s.val[en >> 1];
            const float val = c == 0 ? pv.x : c == 1 ? pv.y : c == 2 ? pv.z : pv.w;
            unsafeAtomicAdd(p.ws + d + c, __int_as_float(right ? ent.w : ent.z) * val);
        }
    }
}

__global__ void __launch_bounds__(256) k_views_composite(const ViewsParams p) {
    const int m = blockIdx.y;
    const int64_t np = (int64_t)p.vH[m] * p.vW[m];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= np) return;
    const float4 *S = reinterpret_cast<const float4 *>(p.ws + p.sbase[m]);
    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    for (int l = 0; l < p.L; ++l) {
        const float4 s = S[(int64_t)l * np + i];
        const float w = T * s.w;
        c0 = fmaf(w, s.x, c0);
        c1 = fmaf(w, s.y, c1);
        c2 = fmaf(w, s.z, c2);
        T *= 1.0f - s.w;
    }
    float *rgb = p.rgb[m];
    rgb[i * 3 + 0] = c0;
    rgb[i * 3 + 1] = c1;
    rgb[i * 3 + 2] = c2;
    if (p.acc[m] != nullptr) p.acc[m][i] = 1.0f - T;
}


// ---------------------------------------------------------------------------
// Binned form.
//
//   k_vbin_zero    clears the bin counts
//   k_vbin_count   a workgroup takes 1024 layer-pixels of one view: their
//                  records' bins, counted in an LDS hash table, then one
//                  global add per distinct bin
//   k_vbin_scan    one workgroup: exclusive prefix sums of the counts, the
//                  write cursors
//   k_vbin_write   the same records; per distinct bin of the workgroup one
//                  global add on the bin's cursor reserves a run of slots,
//                  a record's slot is that base plus its rank in the bin
//   k_vbin_tile    one workgroup per (view, tile): adds the taps of its
//                  records that fall inside the tile into LDS (all layers of
//                  the tile) and composites each pixel front to back
//
// The tile sums are 64-bit fixed point (2^-32 units) added with integer LDS
// atomics: on this chip a float atomic add in LDS costs several times an
// integer one, and integer sums are exact, so the result does not depend on
// the order in which records arrive (the render is bitwise reproducible).
// Each contribution (tap weight times payload, rounded to float as in the
// planes form) is rounded to the nearest 2^-32; a sum stays below 2^31 in
// magnitude unless more than 2^31 records reach one view pixel of a layer.
//
// A record is binned by the tile holding (ix + 1, iy + 1), the right column
// and bottom row of its taps; its left column (ix) may then lie in the tile
// to the left and its top row (iy) in the tile above.  Each tile has four
// bins by which of the two its records cross (bit 0 left, bit 1 top), so a
// tile's workgroup reads its own four bins and only the crossing bins of
// the tiles to its right, below and below right: every record is stored
// once and read by at most four workgroups.
// ---------------------------------------------------------------------------

constexpr int kVbKpt = 4;                       // records per thread
constexpr int kVbChunk = 256 * kVbKpt;          // records per workgroup
constexpr int kVbHashBits = 11;
constexpr int kVbHash = 1 << kVbHashBits;       // LDS hash slots, > kVbChunk keys
constexpr float kVbFix = 4294967296.0f;         // fixed-point scale of the tile sums, 2^32
constexpr float kVbUnfix = 2.3283064365386963e-10f;   // 2^-32

// 1 / x in double: the hardware reciprocal refined by one Newton step (its
// relative error squares, far below what the coordinates need).  The binned
// passes all reproject through it, so they agree bit for bit.
__device__ inline double recip_d(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// The record of layer-pixel q in view m: its bin, or -1 when no tap lies in
// the view.  The reprojection of k_splat (reciprocals as above); a sample
// with fxc <= -1 or fxc >= vW (likewise y) has no tap inside.  Every binned
// pass calls it: the tile pass recomputes a record's footprint from the
// layer-pixel index the write pass stored.
// (The binned form runs only while V L H W < 2^31, so a layer-pixel index
// and its divisions fit 32 bits.)
__device__ inline int vbin_record(const ViewsParams &p, int m, int q, float &fx, float &fy,
                                  int &ix, int &iy, int &l) {
    const uint32_t hw = (uint32_t)p.H * (uint32_t)p.W, uq = (uint32_t)q;
    l = (int)(uq / hw);
    const uint32_t r = uq - (uint32_t)l * hw;
    const int y = (int)(r / (uint32_t)p.W), x = (int)(r - (uint32_t)y * (uint32_t)p.W);
    const double u = (double)x + 0.5, v = (double)y + 0.5;
    const double invd = recip_d((double)p.depth[q]);
    const double *A = p.cam[m];
    const int vw = p.vW[m], vh = p.vH[m];
    const double pz = fma(A[6], u, fma(A[7], v, fma(A[11], invd, A[8])));
    const double qx = fma(A[0], u, fma(A[1], v, fma(A[9], invd, A[2])));
    const double qy = fma(A[3], u, fma(A[4], v, fma(A[10], invd, A[5])));
    const double rz = recip_d(pz);
    const double fxc = qx * rz - 0.5, fyc = qy * rz - 0.5;
    if (!((pz > 1e-6) && (fxc > -1.0) && (fxc < (double)vw) && (fyc > -1.0) && (fyc < (double)vh)))
        return -1;
    const double xf = floor(fxc), yf = floor(fyc);
    fx = (float)(fxc - xf);
    fy = (float)(fyc - yf);
    ix = (int)xf;
    iy = (int)yf;
    const int tx = min((ix + 1) / p.tw, p.ntx[m] - 1), ty = min((iy + 1) / p.th, p.nty[m] - 1);
    const int cls = (ix == tx * p.tw - 1 ? 1 : 0) | (iy == ty * p.th - 1 ? 2 : 0);
    return 4 * (p.tbase[m] + ty * p.ntx[m] + tx) + cls;
}

// Slot of key b in the workgroup's hash table (linear probing).  At most
// kVbChunk distinct keys go into kVbHash > kVbChunk slots, so a free or
// matching slot is always found within kVbHash probes.
__device__ inline int vbin_slot(int *hkey, int b) {
    int h = (int)(((uint32_t)b * 2654435761u) >> (32 - kVbHashBits));
    for (int probe = 0; probe < kVbHash; ++probe) {
        const int old = atomicCAS(&hkey[h], -1, b);
        if (old == -1 || old == b) return h;
        h = (h + 1) & (kVbHash - 1);
    }
    return -1;                                   // not reached
}

__global__ void __launch_bounds__(256) k_vbin_zero(const ViewsParams p) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < p.nbins; i += gridDim.x * 256) p.count[i] = 0u;
}

__global__ void __launch_bounds__(256) k_vbin_count(const ViewsParams p) {
    __shared__ int hkey[kVbHash];
    __shared__ uint32_t hcnt[kVbHash];
    for (int i = threadIdx.x; i < kVbHash; i += 256) {
        hkey[i] = -1;
        hcnt[i] = 0u;
    }
    __syncthreads();
    const int64_t cpv = (p.N + kVbChunk - 1) / kVbChunk;
    const int m = (int)(blockIdx.x / cpv);
    const int64_t q0 = ((int64_t)blockIdx.x - (int64_t)m * cpv) * kVbChunk;
#pragma unroll
    for (int k = 0; k < kVbKpt; ++k) {
        const int64_t q = q0 + k * 256 + threadIdx.x;
        if (q >= p.N) break;
        float fx, fy;
        int ix, iy, l;
        const int b = vbin_record(p, m, (int)q, fx, fy, ix, iy, l);
        if (b >= 0) {
            const int sl = vbin_slot(hkey, b);
            if (sl >= 0) atomicAdd(&hcnt[sl], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kVbHash; i += 256)
        if (hkey[i] >= 0) atomicAdd(&p.count[hkey[i]], hcnt[i]);
}

// One workgroup of 1024 threads: each thread sums a run of consecutive
// counts (read four at a time; nbins is a multiple of 4 and the arrays are
// 16-byte aligned), the 1024 run totals are scanned in LDS, and each thread
// writes its run's exclusive prefix sums (start and cursor); start[nbins] =
// total.
__global__ void __launch_bounds__(1024) k_vbin_scan(const ViewsParams p) {
    __shared__ uint32_t tot[1024];
    const int n4 = p.nbins / 4, t = threadIdx.x;
    const int per = (n4 + 1023) / 1024;
    const int b0 = min(t * per, n4), b1 = min(b0 + per, n4);
    const uint4 *c4 = reinterpret_cast<const uint4 *>(p.count);
    uint32_t s = 0u;
#pragma unroll 4
    for (int i = b0; i < b1; ++i) {
        const uint4 c = c4[i];
        s += c.x + c.y + c.z + c.w;
    }
    tot[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive scan (Hillis-Steele)
        const uint32_t v = t >= off ? tot[t - off] : 0u;
        __syncthreads();
        tot[t] += v;
        __syncthreads();
    }
    uint32_t run = tot[t] - s;                   // exclusive
    uint4 *s4 = reinterpret_cast<uint4 *>(p.start), *k4 = reinterpret_cast<uint4 *>(p.cursor);
#pragma unroll 4
    for (int i = b0; i < b1; ++i) {
        const uint4 c = c4[i];
        uint4 o;
        o.x = run;
        o.y = o.x + c.x;
        o.z = o.y + c.y;
        o.w = o.z + c.z;
        run = o.w + c.w;
        s4[i] = o;
        k4[i] = o;
    }
    if (t == 1023) p.start[p.nbins] = tot[1023];
}

__global__ void __launch_bounds__(256) k_vbin_write(const ViewsParams p) {
    __shared__ int hkey[kVbHash];
    __shared__ uint32_t hcnt[kVbHash];
    __shared__ uint32_t hbase[kVbHash];
    for (int i = threadIdx.x; i < kVbHash; i += 256) {
        hkey[i] = -1;
        hcnt[i] = 0u;
    }
    __syncthreads();
    const int64_t cpv = (p.N + kVbChunk - 1) / kVbChunk;
    const int m = (int)(blockIdx.x / cpv);
    const int64_t q0 = ((int64_t)blockIdx.x - (int64_t)m * cpv) * kVbChunk;
    int sl[kVbKpt], rb[kVbKpt];
    uint32_t rank[kVbKpt];
#pragma unroll
    for (int k = 0; k < kVbKpt; ++k) {
        sl[k] = -1;
        rb[k] = 0;
        rank[k] = 0u;
        const int64_t q = q0 + k * 256 + threadIdx.x;
        if (q >= p.N) continue;
        float fx, fy;
        int ix, iy, l;
        const int b = vbin_record(p, m, (int)q, fx, fy, ix, iy, l);
        if (b < 0) continue;
        rb[k] = b;
        sl[k] = vbin_slot(hkey, b);
        if (sl[k] >= 0) rank[k] = atomicAdd(&hcnt[sl[k]], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kVbHash; i += 256)
        if (hkey[i] >= 0) hbase[i] = atomicAdd(&p.cursor[hkey[i]], hcnt[i]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kVbKpt; ++k) {
        if (sl[k] < 0) continue;
        const uint32_t slot = hbase[sl[k]] + rank[k];
        if (slot >= p.start[rb[k] + 1]) continue;    // never taken: both passes bin alike
        p.rec[slot] = (int)(q0 + k * 256 + threadIdx.x);
    }
}

__global__ void __launch_bounds__(256) k_vbin_tile(const ViewsParams p) {
    extern __shared__ unsigned long long tacc[]; // [L][th][tw][4] (r, g, b, alpha) sums, 2^-32
    const int t = blockIdx.x;
    int m = 0;
    for (int i = 1; i < p.V; ++i) m = (t >= p.tbase[i]) ? i : m;
    const int ntx = p.ntx[m], nty = p.nty[m];
    const int lt = t - p.tbase[m];
    const int tx = lt % ntx, ty = lt / ntx;
    const int tw = p.tw, th = p.th, tpix = tw * th;
    const int x0 = tx * tw, y0 = ty * th;
    const int vw = p.vW[m], vh = p.vH[m];
    for (int i = threadIdx.x; i < 4 * p.L * tpix; i += 256) tacc[i] = 0ull;
    __syncthreads();
    // the record ranges: own bins, then the crossing bins of the tiles to the
    // right (left-crossing), below (top-crossing) and below right (both)
    uint32_t rs[5] = {0u, 0u, 0u, 0u, 0u}, re[5] = {0u, 0u, 0u, 0u, 0u};
    {
        const int b = 4 * (p.tbase[m] + ty * ntx + tx);
        rs[0] = p.start[b];
        re[0] = p.start[b + 4];
        if (tx + 1 < ntx) {
            rs[1] = p.start[b + 4 + 1];
            re[1] = p.start[b + 4 + 2];
            rs[2] = p.start[b + 4 + 3];
            re[2] = p.start[b + 4 + 4];
        }
        if (ty + 1 < nty) {
            const int bb = 4 * (p.tbase[m] + (ty + 1) * ntx + tx);
            rs[3] = p.start[bb + 2];
            re[3] = p.start[bb + 4];
            if (tx + 1 < ntx) {
                rs[4] = p.start[bb + 4 + 3];
                re[4] = p.start[bb + 4 + 4];
            }
        }
    }
    // the five ranges as one index space; a thread takes its records two
    // at a time so both records' loads are in flight together (each record
    // is a chain: its index, then the layer-pixel's depth and payload)
    uint32_t cum[6];
    cum[0] = 0u;
#pragma unroll
    for (int j = 0; j < 5; ++j) cum[j + 1] = cum[j] + (re[j] - rs[j]);
    const uint32_t total = cum[5];
    constexpr int U = 2;
    for (uint32_t k0 = threadIdx.x; k0 < total; k0 += 256u * U) {
        int q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t k = k0 + 256u * u;
            q[u] = -1;
            if (k < total) {
                int j = 0;
#pragma unroll
                for (int jj = 1; jj < 5; ++jj) j += (k >= cum[jj]) ? 1 : 0;
                q[u] = p.rec[rs[j] + (k - cum[j])];
            }
        }
        float fx[U], fy[U];
        int ix[U], iy[U], l[U];
        float4 v[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // the record is the layer-pixel's index: its footprint is
            // recomputed by the same function the binning passes ran (so it
            // is the one they binned) and its payload read from the LDM; an
            // index out of range is only a record never written
            ok[u] = (unsigned)q[u] < (unsigned)p.N;
            const int qq = ok[u] ? q[u] : 0;
            ok[u] = ok[u] && vbin_record(p, m, qq, fx[u], fy[u], ix[u], iy[u], l[u]) >= 0;
            v[u] = make_float4(p.color[(int64_t)qq * 3 + 0], p.color[(int64_t)qq * 3 + 1],
                               p.color[(int64_t)qq * 3 + 2], p.alpha[qq]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
            const float w[4] = {(1.0f - fx[u]) * (1.0f - fy[u]), fx[u] * (1.0f - fy[u]),
                                (1.0f - fx[u]) * fy[u], fx[u] * fy[u]};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int x = ix[u] + (k & 1), y = iy[u] + (k >> 1);
                const int lx = x - x0, ly = y - y0;
                if (lx < 0 || lx >= tw || ly < 0 || ly >= th || x >= vw || y >= vh) continue;
                unsigned long long *d = &tacc[4 * ((l[u] * th + ly) * tw + lx)];
                atomicAdd(d + 0, (unsigned long long)__float2ll_rn(w[k] * v[u].x * kVbFix));
                atomicAdd(d + 1, (unsigned long long)__float2ll_rn(w[k] * v[u].y * kVbFix));
                atomicAdd(d + 2, (unsigned long long)__float2ll_rn(w[k] * v[u].z * kVbFix));
                atomicAdd(d + 3, (unsigned long long)__float2ll_rn(w[k] * v[u].w * kVbFix));
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < tpix; i += 256) {
        const int lx = i % tw, ly = i / tw;
        const int x = x0 + lx, y = y0 + ly;
        if (x >= vw || y >= vh) continue;
        float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
        for (int l = 0; l < p.L; ++l) {
            const unsigned long long *e = &tacc[4 * ((l * th + ly) * tw + lx)];
            const float4 s = make_float4((float)(long long)e[0] * kVbUnfix, (float)(long long)e[1] * kVbUnfix,
                                         (float)(long long)e[2] * kVbUnfix, (float)(long long)e[3] * kVbUnfix);
            const float w = T * s.w;
            c0 = fmaf(w, s.x, c0);
            c1 = fmaf(w, s.y, c1);
            c2 = fmaf(w, s.z, c2);
            T *= 1.0f - s.w;
        }
        const int64_t o = (int64_t)y * vw + x;
        float *rgb = p.rgb[m];
        rgb[o * 3 + 0] = c0;
        rgb[o * 3 + 1] = c1;
        rgb[o * 3 + 2] = c2;
        if (p.acc[m] != nullptr) p.acc[m][o] = 1.0f - T;
    }
}

}  // namespace

hipError_t launch_render_to_views(const ViewsParams &p, hipStream_t s) {
    if (p.binned) {
        const int zb = (p.nbins + 255) / 256 < 1024 ? (p.nbins + 255) / 256 : 1024;
        hipLaunchKernelGGL(k_vbin_zero, dim3(zb > 0 ? zb : 1), dim3(256), 0, s, p);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int64_t cpv = (p.N + kVbChunk - 1) / kVbChunk;
        const unsigned g = (unsigned)(cpv * p.V);
        hipLaunchKernelGGL(k_vbin_count, dim3(g), dim3(256), 0, s, p);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_vbin_scan, dim3(1), dim3(1024), 0, s, p);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_vbin_write, dim3(g), dim3(256), 0, s, p);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const size_t lds = (size_t)p.L * p.th * p.tw * 32;
        hipLaunchKernelGGL(k_vbin_tile, dim3((unsigned)p.tbase[p.V]), dim3(256), lds, s, p);
        return hipGetLastError();
    }
    const int64_t n4 = p.ws_floats / 4;
    const int zb = (int)((n4 + 255) / 256 < 8192 ? (n4 + 255) / 256 : 8192);
    hipLaunchKernelGGL(k_views_zero, dim3(zb > 0 ? zb : 1), dim3(256), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_splat, dim3((unsigned)(((p.N + 255) / 256) * p.V)), dim3(256), 0, s, p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_views_composite, dim3((unsigned)((p.max_view_pixels + 255) / 256), p.V),
                       dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace qk
