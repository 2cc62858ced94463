// Direct stiffness summation (gather-scatter Q Q^T) on the periodic box,
// without atomics or index lists.
//
// A row is the lx nodes of one element that share (j, k).  The rows are split
// into tasks, one wave each, such that every row of the mesh belongs to
// exactly one task and a task holds every copy of the nodes in its rows: rows
// of different tasks are disjoint, so the in-place update is race free, and
// every row is read once and written once, whole (no partial-line writes reach
// memory).  Every copy of a node adds the same values in the same order (copy
// s takes the +d side in direction d when bit d of s is set, directions x, y,
// z in that order among the boundary ones) and so gets the same bits.
//
// A task walks one x-line of elements in segments; a lane holds V consecutive
// nodes of a row in one word of V * sizeof(T) bytes (16 where lx allows in the
// plane form, up to 8 in the row form).  The
// x copy of a node (i = N against the next element's i = 0) comes from the
// next element's lanes, or from the next segment's registers, or, across the
// periodic wrap, from values read before any row of the line is written.
// Two forms share this:
// - the plane form (dssum_planes_kernel), where an element's plane fits a
//   wave: one load moves rows 1..N of a plane of an element;
// - the row form (dssum_rows_kernel) for the other orders: one load moves one
//   row from each of 64 / (lx / V) elements.
#include "k_common.h"

namespace semk {

// segments in flight per task: with three, the rows of a wave cover the HBM
// latency (measured at 64^3 elements, N = 7: 0.50 against 0.51 ms for two at
// fp64, 0.30 against 0.31 ms at fp32)
constexpr int GS_DEPTH = 3;

template <int B> struct GsWord;
template <> struct GsWord<2> { using type = unsigned short; };
template <> struct GsWord<4> { using type = unsigned int; };
template <> struct GsWord<8> { using type = unsigned long long; };
typedef unsigned long long GsW16 __attribute__((ext_vector_type(2)));
template <> struct GsWord<16> { using type = GsW16; };

template <typename U> __device__ __forceinline__ U lane_get(U v, int src)
{
    if constexpr (sizeof(U) == 16) {
        U r;
        r.x = lane_get(v.x, src);
        r.y = lane_get(v.y, src);
        return r;
    } else if constexpr (sizeof(U) == 8) {
        const int lo = __shfl((int)(unsigned)v, src, 64), hi = __shfl((int)(unsigned)(v >> 32), src, 64);
        return (U)(unsigned)lo | ((U)(unsigned)hi << 32);
    } else {
        return (U)(unsigned)__shfl((int)(unsigned)v, src, 64);
    }
}

template <typename U> __device__ __forceinline__ U lane_bcast(U v, int src)
{
    if constexpr (sizeof(U) == 16) {
        U r;
        r.x = lane_bcast(v.x, src);
        r.y = lane_bcast(v.y, src);
        return r;
    } else if constexpr (sizeof(U) == 8) {
        const int lo = __builtin_amdgcn_readlane((int)(unsigned)v, src);
        const int hi = __builtin_amdgcn_readlane((int)(unsigned)(v >> 32), src);
        return (U)(unsigned)lo | ((U)(unsigned)hi << 32);
    } else {
        return (U)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, src);
    }
}

template <typename T, int V, typename U> __device__ __forceinline__ T word_get(U w, int q)
{
    T v[V];
    __builtin_memcpy(v, &w, sizeof(U));
    return v[q];
}

// Row form.  Task (x-line of elements (ey, ez), j, k), j and k in [1, N],
// owns the rows (e, j, k) of every element e of the line and, where they hold
// the same nodes, the rows (e+y, 0, k) when j = N, (e+z, j, 0) when k = N and
// (e+y+z, 0, 0) when both.  Lane el * (lx / V) + p holds word p of the rows of
// element el of the segment.
//
// one task: NC = 1, 2 or 4 copy rows; row t of the line's element ex starts
// at byte rr[t] + ex * eb (eb = bytes per element, ib = the lane's byte
// offset in a row; the setup keeps a line of elements below 4 GB).  Segment
// s + GS_DEPTH is loaded while segment s is summed, so the x-neighbour of its
// last element (segment s + 1) is already in registers; the GS_DEPTH + 1
// segment buffers rotate by name (the loop is unrolled), so no register copy
// waits for a load in flight.
template <int NC, int V, typename T, typename A>
__device__ __forceinline__ void gs_row_task(const SEM_GLOBAL char* const* rr, SEM_GLOBAL char* const* rw,
                                            unsigned eb, unsigned ib, int nx, int W, int LP, int el, int p,
                                            int lane, bool nrm, double& acc)
{
    using U = typename GsWord<V * sizeof(T)>::type;
    const int nseg = (nx + W - 1) / W;
    U buf[GS_DEPTH + 1][NC], first[NC], carry[NC];
    // segment s, lane (el, p); lanes past the line read its last element
    // (their values are never used)
    auto load = [&](U (&v)[NC], int s) {
        const unsigned off = (unsigned)min(s * W + el, nx - 1) * eb + ib;
#pragma unroll
        for (int t = 0; t < NC; ++t) v[t] = *(const SEM_GLOBAL U*)(rr[t] + off);
    };
    // lane p = 0 holds node i = 0 in its first slot, lane p = LP - 1 node i = N in its last
    const bool lo = p == 0, hi = p == LP - 1;
    // sum and store segment s (cur), load segment s + GS_DEPTH into nn
    auto step = [&](U (&cur)[NC], const U (&nxt)[NC], U (&nn)[NC], int s) {
        load(nn, s + GS_DEPTH);
        const int ws = min(W, nx - s * W);
        const bool more = s + 1 < nseg;
        T lp[NC], rp[NC];
#pragma unroll
        for (int t = 0; t < NC; ++t) {
            if (s == 0) first[t] = lane_bcast(cur[t], 0);
            const U r = lane_get(cur[t], min(lane + 1, 63));
            const U l = lane_get(cur[t], max(lane - 1, 0));
            const U nb0 = more ? lane_bcast(nxt[t], 0) : first[t];
            rp[t] = word_get<T, V>(el + 1 < ws ? r : nb0, 0);          // i = 0 of element e+x
            lp[t] = word_get<T, V>(el > 0 ? l : carry[t], V - 1);      // i = N of element e-x
        }
        T out[V];
#pragma unroll
        for (int q = 0; q < V; ++q) {
            const bool xl = lo && q == 0, xh = hi && q == V - 1;
            const T o0 = word_get<T, V>(cur[0], q);
            A sum = to<A>(xl ? lp[0] : o0);
            if (xl || xh) sum += to<A>(xl ? o0 : rp[0]);
#pragma unroll
            for (int t = 1; t < NC; ++t) {
                const T ot = word_get<T, V>(cur[t], q);
                sum += to<A>(xl ? lp[t] : ot);
                if (xl || xh) sum += to<A>(xl ? ot : rp[t]);
            }
            out[q] = to<T>(sum);
        }
        U w;
        __builtin_memcpy(&w, out, sizeof(U));
        if (el < ws) {
            const unsigned off = (unsigned)(s * W + el) * eb + ib;
#pragma unroll
            for (int t = 0; t < NC; ++t) *(SEM_GLOBAL U*)(rw[t] + off) = w;
            // NC copies of each node written here, each 1 / (NC * 2^x) of it
            if (nrm) {
#pragma unroll
                for (int q = 0; q < V; ++q) {
                    const double v = to<double>(out[q]);
                    const bool xb = (lo && q == 0) || (hi && q == V - 1);
                    acc += xb ? 0.5 * v * v : v * v;
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NC; ++t) carry[t] = lane_bcast(cur[t], W * LP - 1);
    };
    {
        // the word holding i = N of the line's last element
        const unsigned off = (unsigned)(nx - 1) * eb + (unsigned)((LP - 1) * V * sizeof(T));
#pragma unroll
        for (int t = 0; t < NC; ++t) carry[t] = *(const SEM_GLOBAL U*)(rr[t] + off);
    }
#pragma unroll
    for (int r = 0; r < GS_DEPTH; ++r) load(buf[r], r);
    for (int s = 0;;) {
#pragma unroll
        for (int r = 0; r <= GS_DEPTH; ++r) {
            step(buf[r], buf[(r + 1) % (GS_DEPTH + 1)], buf[(r + GS_DEPTH) % (GS_DEPTH + 1)], s);
            if (++s >= nseg) return;
        }
    }
}

// Squared norm over unique nodes, fused into the sum: every local point is
// written by exactly one lane, which adds w^2 / (its node's copy count), so a
// workgroup's lanes add up to sum_nodes w^2 over the nodes they wrote.  The
// workgroup's fixed-order sum is its partial (slot pslot, one per workgroup of
// the request; workgroup 0 records their number).
__device__ __forceinline__ void gs_put_norm(const ReqDesc* R, int pslot, int blk, double acc, int nblk)
{
    __shared__ double red[SEM_GS_THREADS / 64];
    double v[1] = {acc};
    block_sum<double, 1>(v, red);
    if (threadIdx.x == 0) {
        gp(R->part)[(long long)pslot * R->pstride + blk] = v[0];
        if (blk == 0) gp(R->I)[I_PCNT + pslot] = nblk;
    }
}

// Workgroup p runs task block (p % 8) * per + p / 8, so each XCD walks one
// contiguous range; within a request the blocks go (ez, k, ey), so the two
// blocks that share the lines of a row j = 0 are neighbours on one XCD.
template <typename T, typename A, int V>
__global__ void __launch_bounds__(SEM_GS_THREADS)
dssum_rows_kernel(Batch bt, int field, int gate, void* raw, int per, int pslot)
{
    const int pb = blockIdx.x;
    const int g = (pb & 7) * per + (pb >> 3);
    if (g >= bt.gl[bt.n]) return;
    const int ri = find_req(bt.gl, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    if (!gate_ok(R, gate)) return;
    const int lx = R->lx, N = lx - 1, nx = R->nel[0], ny = R->nel[1], nz = R->nel[2];
    const int blk = g - bt.gl[ri];
    const int ey = blk % ny, k = 1 + (blk / ny) % N, ez = blk / (ny * N);
    const int eyp = ey + 1 == ny ? 0 : ey + 1, ezp = ez + 1 == nz ? 0 : ez + 1;
    const long long L3 = (long long)lx * lx * lx;
    const int lane = threadIdx.x & 63;
    const int LP = lx / V, W = 64 / LP, el = lane / LP, p = lane - el * LP;
    const SEM_GLOBAL T* ur = field >= 0 ? gfield<T>(R, field) : gp((const T*)raw);
    SEM_GLOBAL T* uw = field >= 0 ? gfieldw<T>(R, field) : gp((T*)raw);
    const unsigned eb = (unsigned)(L3 * sizeof(T)), ib = (unsigned)(p * V * sizeof(T));
    // the wave index is uniform; say so, so that the row bases stay scalar
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double acc = 0.0;
    for (int j = 1 + wv; j <= N; j += SEM_GS_THREADS / 64) {
        const int by = j == N, bz = k == N;
        const SEM_GLOBAL char* rr[4];
        SEM_GLOBAL char* rw[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            int yy = ey, jj = j, zz = ez, kk = k, bit = 0;
            if (by && ((t >> bit++) & 1)) { yy = eyp; jj = 0; }
            if (bz && ((t >> bit++) & 1)) { zz = ezp; kk = 0; }
            const long long o = (long long)nx * (yy + (long long)ny * zz) * L3 + lx * (jj + lx * kk);
            rr[t] = (const SEM_GLOBAL char*)(ur + o);
            rw[t] = (SEM_GLOBAL char*)(uw + o);
        }
        if (by && bz) gs_row_task<4, V, T, A>(rr, rw, eb, ib, nx, W, LP, el, p, lane, pslot >= 0, acc);
        else if (by || bz) gs_row_task<2, V, T, A>(rr, rw, eb, ib, nx, W, LP, el, p, lane, pslot >= 0, acc);
        else gs_row_task<1, V, T, A>(rr, rw, eb, ib, nx, W, LP, el, p, lane, pslot >= 0, acc);
    }
    if (pslot >= 0) gs_put_norm(R, pslot, blk, acc, bt.gl[ri + 1] - bt.gl[ri]);
}

// Plane form, where an element's plane fits a wave (lx * lx / V <= 64 lanes).
// Task (x-line of elements, k), k in [1, N], owns for every element e of the
// line the rows (e, j, k), j in [1, N], and the row (e+y, 0, k), which holds
// the other copies of the plane's j = N nodes; when k = N it also owns the
// same rows of the planes k = 0 of e+z and e+y+z.  Lane el * SL + r * LP + p
// (SL = lx * LP lanes an element) holds word p of slot r: slot 0 the row
// (e+y, 0, k), slots 1..N the rows (e, r, k); a load thus moves rows 1..N of
// an element's plane, which are contiguous, and the neighbour's row 0.  The y
// copy of a node sits N slots away in the same register, the z copy in the
// z-plane register of the same lane, and the x copies come from the next or
// previous element's lanes.
template <typename U> struct GsSeg {
    U m[2];   // [0] plane k, [1] plane 0 of e+z
};

template <int ZC, int V, typename T, typename A>
__device__ __forceinline__ void gs_plane_task(SEM_GLOBAL char* const* lp, unsigned eb, int nx, int EW, int SL,
                                              int LP, int N, int el, int r, int p, int lane, bool nrm, double& acc)
{
    using U = typename GsWord<V * sizeof(T)>::type;
    constexpr int NZ = ZC + 1;
    const int nseg = (nx + EW - 1) / EW;
    // source lanes: the same slot of the next and previous element (in this
    // segment, or element 0 of the next and the last of the previous one), and
    // for each the y copy, dy lanes away (lanes past the last element of a
    // segment clamp; their values are never used)
    const int dy = r == 0 ? N * LP : r == N ? -N * LP : 0;
    auto cl = [](int l) { return min(max(l, 0), 63); };
    const int rsrc = cl(lane + SL - LP + 1), lsrc = cl(lane - SL + LP - 1);
    const int rnext = r * LP, lprev = (EW - 1) * SL + r * LP + LP - 1;
    const int ysrc = cl(lane + dy), rsrc_y = cl(rsrc + dy), lsrc_y = cl(lsrc + dy);
    const int rnext_y = cl(rnext + dy), lprev_y = cl(lprev + dy);
    GsSeg<U> buf[GS_DEPTH + 1], first, prev;
    auto load = [&](GsSeg<U>& b, int s) {
        const unsigned off = (unsigned)min(s * EW + el, nx - 1) * eb;
#pragma unroll
        for (int z = 0; z < NZ; ++z) b.m[z] = *(const SEM_GLOBAL U*)(lp[z] + off);
    };
    const bool own_y = r == 0, yb = r == 0 || r == N;
    // sum and store segment s (cur), load segment s + GS_DEPTH into nn
    auto step = [&](GsSeg<U>& cur, GsSeg<U>& nxt, GsSeg<U>& nn, int s) {
        load(nn, s + GS_DEPTH);
        const int ws = min(EW, nx - s * EW);
        const bool more = s + 1 < nseg;
        if (s == 0) first = cur;
        // per z plane, the words of this lane's node and of its x neighbours on
        // the -y side (..m) and the +y side (..p) of the node: own element (c),
        // previous element (l), next element (r)
        U cm[2], cp[2], lm[2], lpl[2], rm[2], rp[2];
#pragma unroll
        for (int z = 0; z < NZ; ++z) {
            const U an = more ? nxt.m[z] : first.m[z];
            const U cy = lane_get(cur.m[z], ysrc);
            U rw0 = lane_get(an, rnext), rw1 = lane_get(an, rnext_y);
            U lw0 = lane_get(prev.m[z], lprev), lw1 = lane_get(prev.m[z], lprev_y);
            if (EW > 1) {
                const U c0 = lane_get(cur.m[z], rsrc), c1 = lane_get(cur.m[z], rsrc_y);
                const U d0 = lane_get(cur.m[z], lsrc), d1 = lane_get(cur.m[z], lsrc_y);
                if (el + 1 < ws) { rw0 = c0; rw1 = c1; }
                if (el > 0) { lw0 = d0; lw1 = d1; }
            }
            cm[z] = own_y ? cy : cur.m[z];
            cp[z] = own_y ? cur.m[z] : cy;
            lm[z] = own_y ? lw1 : lw0;
            lpl[z] = own_y ? lw0 : lw1;
            rm[z] = own_y ? rw1 : rw0;
            rp[z] = own_y ? rw0 : rw1;
        }
        T out[V];
#pragma unroll
        for (int q = 0; q < V; ++q) {
            // lo: node i = 0, the +x copy (its -x copy is the previous element's
            // i = N); hi: node i = N, the -x copy
            const bool lo = p == 0 && q == 0, hi = p == LP - 1 && q == V - 1, xb = lo || hi;
            // copy (xs, ys, zs) of the node, xs / ys = 1 on the +x / +y side
            auto term = [&](int zs, int ys, int xs) -> A {
                const T own = word_get<T, V>(ys ? cp[zs] : cm[zs], q);
                const T left = word_get<T, V>(ys ? lpl[zs] : lm[zs], V - 1);
                const T right = word_get<T, V>(ys ? rp[zs] : rm[zs], 0);
                return to<A>(xs ? (lo ? own : right) : (lo ? left : own));
            };
            A sum = term(0, 0, 0);
            if (xb) sum += term(0, 0, 1);
            if (yb) {
                sum += term(0, 1, 0);
                if (xb) sum += term(0, 1, 1);
            }
            if constexpr (ZC) {
                sum += term(1, 0, 0);
                if (xb) sum += term(1, 0, 1);
                if (yb) {
                    sum += term(1, 1, 0);
                    if (xb) sum += term(1, 1, 1);
                }
            }
            out[q] = to<T>(sum);
        }
        U w;
        __builtin_memcpy(&w, out, sizeof(U));
        if (el < ws) {
            const unsigned off = (unsigned)(s * EW + el) * eb;
#pragma unroll
            for (int z = 0; z < NZ; ++z) *(SEM_GLOBAL U*)(lp[z] + off) = w;
            // NZ copies of each node written here, each 1 / (NZ * 2^(x + y)) of it
            if (nrm) {
#pragma unroll
                for (int q = 0; q < V; ++q) {
                    const double v = to<double>(out[q]);
                    const bool xb = (p == 0 && q == 0) || (p == LP - 1 && q == V - 1);
                    const double f = (xb ? 0.5 : 1.0) * (yb ? 0.5 : 1.0);
                    acc += f * v * v;
                }
            }
        }
        prev = cur;
    };
    {
        // the line's last element, for the left neighbour of the first
        const unsigned off = (unsigned)(nx - 1) * eb;
#pragma unroll
        for (int z = 0; z < NZ; ++z) prev.m[z] = *(const SEM_GLOBAL U*)(lp[z] + off);
    }
#pragma unroll
    for (int b = 0; b < GS_DEPTH; ++b) load(buf[b], b);
    for (int s = 0;;) {
#pragma unroll
        for (int b = 0; b <= GS_DEPTH; ++b) {
            step(buf[b], buf[(b + 1) % (GS_DEPTH + 1)], buf[(b + GS_DEPTH) % (GS_DEPTH + 1)], s);
            if (++s >= nseg) return;
        }
    }
}

// Workgroup p runs task block (p % 8) * per + p / 8 (one x-line and four
// planes k, a wave each); within a request the blocks go (ez, k / 4, ey).
template <typename T, typename A, int V>
__global__ void __launch_bounds__(SEM_GS_THREADS)
dssum_planes_kernel(Batch bt, int field, int gate, void* raw, int per, int pslot)
{
    const int pb = blockIdx.x;
    const int g = (pb & 7) * per + (pb >> 3);
    if (g >= bt.gq[bt.n]) return;
    const int ri = find_req(bt.gq, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    if (!gate_ok(R, gate)) return;
    const int lx = R->lx, N = lx - 1, nx = R->nel[0], ny = R->nel[1], nz = R->nel[2];
    const int nkq = (N + 3) / 4;
    const int blk = g - bt.gq[ri];
    const int ey = blk % ny, kq = (blk / ny) % nkq, ez = blk / (ny * nkq);
    // the wave index is uniform; say so, so that k and its branches stay scalar
    const int k = 4 * kq + 1 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int eyp = ey + 1 == ny ? 0 : ey + 1, ezp = ez + 1 == nz ? 0 : ez + 1;
    const long long L3 = (long long)lx * lx * lx;
    const int lane = threadIdx.x & 63;
    const int LP = lx / V, SL = lx * LP, EW = 64 / SL;
    const int el = lane / SL, r = (lane - el * SL) / LP, p = lane - el * SL - r * LP;
    SEM_GLOBAL T* u = field >= 0 ? gfieldw<T>(R, field) : gp((T*)raw);
    // this lane's word in element 0 of the line: slot 0 from the +y line
    const long long lin = (long long)nx * (ey + (long long)ny * ez), liny = (long long)nx * (eyp + (long long)ny * ez);
    const long long linz = (long long)nx * (ey + (long long)ny * ezp), linyz = (long long)nx * (eyp + (long long)ny * ezp);
    SEM_GLOBAL char* lp[2];
    lp[0] = (SEM_GLOBAL char*)(u + (r == 0 ? liny : lin) * L3 + lx * (r + lx * k) + p * V);
    lp[1] = (SEM_GLOBAL char*)(u + (r == 0 ? linyz : linz) * L3 + lx * r + p * V);
    const unsigned eb = (unsigned)(L3 * sizeof(T));
    double acc = 0.0;
    if (k == N) gs_plane_task<1, V, T, A>(lp, eb, nx, EW, SL, LP, N, el, r, p, lane, pslot >= 0, acc);
    else if (k < N) gs_plane_task<0, V, T, A>(lp, eb, nx, EW, SL, LP, N, el, r, p, lane, pslot >= 0, acc);
    if (pslot >= 0) gs_put_norm(R, pslot, blk, acc, bt.gq[ri + 1] - bt.gq[ri]);
}

// The plane form asks for LDS it does not use, so that at most five of its
// workgroups share a CU (160 KB): fewer line walks at once run faster (64^3
// elements, N = 7: fp64 0.461 against 0.487 ms at seven waves per SIMD, fp32
// 0.237 against 0.242 ms; three workgroups: 0.658 ms).
constexpr unsigned GS_PLANES_LDS = 32000;

// one launch per component
template <typename T, typename A, int V>
static void dssum_go(const Batch& b, int field, int ncomp, int gate, void* raw, hipStream_t s, int pslot,
                     bool planes)
{
    const int nblk = planes ? b.gq[b.n] : b.gl[b.n];
    const int per = (nblk + 7) / 8;
    dim3 grid(8 * per);
    for (int c = 0; c < ncomp; ++c) {
        const int f = field >= 0 ? field + c : field, gt = gate < 0 ? gate : gate + c;
        const int ps = pslot >= 0 ? pslot + c : -1;
        if (planes)
            hipLaunchKernelGGL((dssum_planes_kernel<T, A, V>), grid, dim3(SEM_GS_THREADS), GS_PLANES_LDS, s, b, f, gt,
                               raw, per, ps);
        else
            hipLaunchKernelGGL((dssum_rows_kernel<T, A, V>), grid, dim3(SEM_GS_THREADS), 0, s, b, f, gt, raw, per, ps);
    }
}

// Word size and form, as measured (a batch shares one lx):
// - 16-byte words where they divide a row: the plane form when its segments
//   fill at least 48 of the 64 lanes, else the row form (64^3 elements, N = 7:
//   fp64 planes 0.442 ms against 0.467 with 8-byte words; 16^3, N = 11: fp64
//   rows 24.5 against 27.7 us with 8-byte rows, fp32 rows 19.5 against 22.5 us
//   in planes of 36 lanes);
// - else as many nodes as fit 8 bytes and divide lx, in the plane form where
//   the plane fits a wave (16^3, N = 11, fp16: 13.8 us against 18.2 in rows).
static int gs_plane_lanes(int lx, int V) { return (64 / (lx * (lx / V))) * lx * (lx / V); }

template <typename T, typename A>
static void dssum_pick(const Batch& b, int field, int ncomp, int gate, void* raw, hipStream_t s, int pslot)
{
    const int lx = b.lx;
    constexpr int V16 = 16 / (int)sizeof(T);
    if (lx % V16 == 0) {
        const bool planes = gs_planes(lx, V16) && gs_plane_lanes(lx, V16) >= 48;
        return dssum_go<T, A, V16>(b, field, ncomp, gate, raw, s, pslot, planes);
    }
    if constexpr (sizeof(T) <= 2)
        if (lx % 4 == 0) return dssum_go<T, A, 4>(b, field, ncomp, gate, raw, s, pslot, gs_planes(lx, 4));
    if constexpr (sizeof(T) <= 4)
        if (lx % 2 == 0) return dssum_go<T, A, 2>(b, field, ncomp, gate, raw, s, pslot, gs_planes(lx, 2));
    dssum_go<T, A, 1>(b, field, ncomp, gate, raw, s, pslot, gs_planes(lx, 1));
}

void launch_dssum(const Batch& b, int field, int ncomp, int tprec, int gate, void* raw, hipStream_t s, int pslot)
{
    if (b.gl[b.n] == 0) return;
    switch (tprec) {
    case P64: dssum_pick<double, double>(b, field, ncomp, gate, raw, s, pslot); break;
    case P32: dssum_pick<float, float>(b, field, ncomp, gate, raw, s, pslot); break;
    case P16: dssum_pick<__half, float>(b, field, ncomp, gate, raw, s, pslot); break;
    case PBF: dssum_pick<__hip_bfloat16, float>(b, field, ncomp, gate, raw, s, pslot); break;
    default: break;
    }
}

}  // namespace semk
