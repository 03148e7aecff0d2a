// laystats.hpp -- pieces shared by the two forms of the sub-cluster pass over
// the cluster-sorted copy (laysub.hip, and the pass fused into the
// matrix-core cluster draw in assign_mfma.hip): the 8-bit integer operands of
// v_mfma_i32_16x16x32_i8 built from the dense count fragments, and the exact
// statistics of a wavefront's 32 cells.
#pragma once
#include "dpmm_common.hpp"

namespace dpmm {

typedef __attribute__((__vector_size__(4 * sizeof(int)))) int intx4_t;

constexpr int kPlaces = kLayDmax * kBlkGenes;  // places of a cluster's gene order in the dense chunks
constexpr int kPartRows = 4;                   // histogram rows: sub-cluster 0, 1, coin 0, 1

// byte 0 of each of four words -> one word
__device__ inline uint32_t low_bytes(const intx4_t& c)
{
    const uint32_t lo = __builtin_amdgcn_perm((uint32_t)c[1], (uint32_t)c[0], 0x0c0c0400u);
    const uint32_t hi = __builtin_amdgcn_perm((uint32_t)c[3], (uint32_t)c[2], 0x0c0c0400u);
    return __builtin_amdgcn_perm(hi, lo, 0x05040100u);
}

// x -> x - 128 on eight count bytes taken as signed 8-bit values
constexpr long kOffset8 = (long)0x8080808080808080ull;

// k-step s (0, 1) of a fragment: 8 bytes, places 32 s + 8 (l / 16) .. + 7
__device__ inline long kstep(const uint4& v, int s)
{
    return s ? (long)((uint64_t)v.z | ((uint64_t)v.w << 32)) : (long)((uint64_t)v.x | ((uint64_t)v.y << 32));
}

// A lane's fragment of row tile 2 w + m of chunk j (16 bytes)
__device__ inline uint4 frag(const uint8_t* dense, uint32_t doff, int j, int m)
{
    return *reinterpret_cast<const uint4*>(dense + (doff + (uint32_t)(j * kDenseChunkBytes + m * 1024)));
}

// The statistics of a wavefront's 32 cells over the block's dense chunks
// (step 3 of the sub-cluster pass), chunk by chunk with the next chunk's fragments in
// flight: eight selection products bring the counts of each place to the
// lanes of its column, four products with the 0/1 rows sum them over the
// cells, and lane group 0 adds rows 0 .. ROWS - 1 to the block's LDS
// histogram over (row, place).
template <int ROWS>
__device__ inline void chunk_stats(const uint8_t* dense, uint32_t doff, int D, long amask, const long (&sel)[2],
                                   const int (&rc128)[4], uint32_t (*phist)[kPlaces], int g, int r)
{
    if (D <= 0) return;
    const intx4_t zero = {0, 0, 0, 0};
    uint4 f0 = frag(dense, doff, 0, 0), f1 = frag(dense, doff, 0, 1);
#pragma unroll 1
    for (int j = 0; j < D; ++j) {
        uint4 n0 = f0, n1 = f1;
        if (j + 1 < D) {
            n0 = frag(dense, doff, j + 1, 0);
            n1 = frag(dense, doff, j + 1, 1);
        }
        // lane (r, g) gets the counts of place 16 nt + r for cells 16 m + 4 g + i in word i
        intx4_t o[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const intx4_t c0 = __builtin_amdgcn_mfma_i32_16x16x32_i8(kstep(f0, nt >> 1), sel[nt & 1], zero, 0, 0, 0);
            const intx4_t c1 = __builtin_amdgcn_mfma_i32_16x16x32_i8(kstep(f1, nt >> 1), sel[nt & 1], zero, 0, 0, 0);
            const uint64_t xb = ((uint64_t)low_bytes(c0) | ((uint64_t)low_bytes(c1) << 32)) ^ (uint64_t)kOffset8;
            o[nt] = __builtin_amdgcn_mfma_i32_16x16x32_i8(amask, (long)xb, zero, 0, 0, 0);
        }
        // rows 0 .. 3 of the products are in lane group 0, row i in word i
        if (g == 0) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int i = 0; i < ROWS; ++i) atomicAdd(&phist[i][j * kBlkGenes + 16 * nt + r], (uint32_t)(o[nt][i] + rc128[i]));
        }
        f0 = n0;
        f1 = n1;
    }
}

}  // namespace dpmm
