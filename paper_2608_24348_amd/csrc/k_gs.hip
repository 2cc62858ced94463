// Direct stiffness summation (gather-scatter Q Q^T) on the periodic box,
// without atomics or index lists.
//
// Every shared node has one owner copy: the one whose local coordinates are
// all in [1, N] (a node on the face i = 0 is the i = N node of the element
// before it in x, and so on).  Element e owns N^3 - (N-1)^3 nodes -- its faces
// k = N, j = N (k < N) and i = N (j, k < N) -- and for each one a thread reads
// all 2, 4 or 8 copies, adds them in a fixed order (copy s takes the +d
// neighbour's side in direction d when bit d of s is set, directions x, y, z
// in that order among the boundary ones) and writes the sum to every copy.
// Each node's copies are touched by its owner thread only, so the in-place
// update is race free and every copy gets the same bits.  Workgroup p runs
// element block (p % 8) * per + p / 8: workgroups go round-robin over the 8
// XCDs, so each XCD walks one contiguous range of blocks and the x and y
// neighbours' lines an owner touches were brought into that XCD's L2 by the
// blocks just before it.
#include "k_common.h"

namespace semk {

template <typename T, typename A>
__global__ void __launch_bounds__(SEM_GS_THREADS)
dssum_box_kernel(Batch bt, int field, int gate, void* raw, int per)
{
    const int p = blockIdx.x;
    const int g = (p & 7) * per + (p >> 3);
    if (g >= bt.eb[bt.n]) return;
    const int ri = find_req(bt.eb, bt.n, g);
    const ReqDesc* R = bt.r[ri];
    if (!gate_ok(R, gate)) return;
    const int blk = g - bt.eb[ri];
    const int lx = R->lx, N = lx - 1, nx = R->nel[0], ny = R->nel[1], nz = R->nel[2];
    const long long L3 = (long long)lx * lx * lx;
    const int nown = N * N + N * (N - 1) + (N - 1) * (N - 1);
    const int e0 = blk * R->epb;
    const int ne = min(R->epb, R->E - e0);
    const SEM_GLOBAL T* ur = field >= 0 ? gfield<T>(R, field) : gp((const T*)raw);
    SEM_GLOBAL T* uw = field >= 0 ? gfieldw<T>(R, field) : gp((T*)raw);

    for (int q = threadIdx.x; q < ne * nown; q += SEM_GS_THREADS) {
        const int el = q / nown;
        int r = q - el * nown;
        int i, j, k;
        if (r < N * N) { k = N; i = 1 + r % N; j = 1 + r / N; }
        else if ((r -= N * N) < N * (N - 1)) { j = N; i = 1 + r % N; k = 1 + r / N; }
        else { r -= N * (N - 1); i = N; j = 1 + r % (N - 1); k = 1 + r / (N - 1); }
        const int e = e0 + el;
        const int ex = e % nx, ey = (e / nx) % ny, ez = e / (nx * ny);
        // per direction: the two (element coordinate, local coordinate) sides
        const int cx[2] = {ex, ex + 1 == nx ? 0 : ex + 1}, lxi[2] = {i, 0};
        const int cy[2] = {ey, ey + 1 == ny ? 0 : ey + 1}, lyj[2] = {j, 0};
        const int cz[2] = {ez, ez + 1 == nz ? 0 : ez + 1}, lzk[2] = {k, 0};
        const int bx = i == N, by = j == N, bz = k == N;
        const int nb = bx + by + bz;
        long long idx[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            if (s >> nb) break;
            // bit b of s goes to the b-th boundary direction (x, y, z order)
            int b = 0, sx = 0, sy = 0, sz = 0;
            if (bx) sx = (s >> b++) & 1;
            if (by) sy = (s >> b++) & 1;
            if (bz) sz = (s >> b++) & 1;
            const long long ee = cx[sx] + (long long)nx * (cy[sy] + (long long)ny * cz[sz]);
            idx[s] = ee * L3 + lxi[sx] + lx * (lyj[sy] + lx * lzk[sz]);
        }
        const int ncopy = 1 << nb;
        T v[8];
#pragma unroll
        for (int s = 0; s < 8; ++s)
            if (s < ncopy) v[s] = ldg(ur + idx[s]);
        A sum = (A)0;
#pragma unroll
        for (int s = 0; s < 8; ++s)
            if (s < ncopy) sum += to<A>(v[s]);
        const T w = to<T>(sum);
#pragma unroll
        for (int s = 0; s < 8; ++s)
            if (s < ncopy) stg(uw + idx[s], w);
    }
}

// one launch per component: with three fields at once the lines a block's
// neighbours touch no longer fit an XCD's L2 across the blocks in flight
// (measured at 32^3, N = 7: 1.04 against 0.93 ms of fp64 dssum per step)
template <typename T, typename A>
static void dssum_box_go(const Batch& b, int field, int ncomp, int gate, void* raw, hipStream_t s)
{
    const int nblk = b.eb[b.n];
    const int per = (nblk + 7) / 8;
    dim3 grid(8 * per);
    for (int c = 0; c < ncomp; ++c)
        hipLaunchKernelGGL((dssum_box_kernel<T, A>), grid, dim3(SEM_GS_THREADS), 0, s, b,
                           field >= 0 ? field + c : field, gate < 0 ? gate : gate + c, raw, per);
}

void launch_dssum(const Batch& b, int field, int ncomp, int tprec, int gate, void* raw, hipStream_t s)
{
    if (b.eb[b.n] == 0) return;
    switch (tprec) {
    case P64: dssum_box_go<double, double>(b, field, ncomp, gate, raw, s); break;
    case P32: dssum_box_go<float, float>(b, field, ncomp, gate, raw, s); break;
    case P16: dssum_box_go<__half, float>(b, field, ncomp, gate, raw, s); break;
    case PBF: dssum_box_go<__hip_bfloat16, float>(b, field, ncomp, gate, raw, s); break;
    default: break;
    }
}

}  // namespace semk
