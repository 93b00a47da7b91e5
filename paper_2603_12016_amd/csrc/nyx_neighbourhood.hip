// nyx_neighbourhood.hip -- neighbourhood texture matrices of every ROI.
//
// Three texture families of the paper's feature list (Supplementary Table S3,
// rows with the NY mark) come from one scan of each ROI voxel's
// neighbourhood: the neighbouring grey level dependence matrix (NGLDM, rows
// 175-192), the neighbourhood grey tone difference matrix (NGTDM, rows
// 246-250) and the grey level dependence matrix (GLDM, rows 251-264; the same
// dependence matrix under other names).  The paper names the features; the
// definitions are the usual ones:
//   * levels are the fixed-bin-number levels of the texture features, the
//     neighbourhood is Chebyshev distance 1 (8 neighbours in a plane, 26 in a
//     volume), and only neighbours inside the image and the ROI take part;
//   * dependence k = 1 + the neighbours whose level differs by at most alpha;
//     S(i, k) counts the ROI voxels of level i and dependence k;
//   * NGTDM: n_i counts the voxels of level i with at least one neighbour,
//     s_i sums |i - mean level of their neighbours| over them; the five
//     features use p_i = n_i / sum n over the levels present, with
//     COARSENESS = 1e6, and CONTRAST, BUSYNESS, STRENGTH = 0, where their
//     denominators vanish (a flat texture), and NaN when no voxel has a
//     neighbour.
//
// One work-group per ROI.  The scan gathers each ROI voxel's neighbours
// (label and level) and counts, with LDS atomics, S(i, k), n_i and the exact
// integers A(i, W) = sum |i W - sum of the W neighbour levels| per level i
// and neighbour count W, so s_i = sum_W A(i, W) / W needs no floating sum
// during the scan.  The features then come from exact integer moments of S
// (GLM, GLV, DCM, DCV, the non-uniformities, energy) and double sums (the
// weighted emphases, entropy, and the NGTDM pair sums over the levels
// present).
#include <hip/hip_runtime.h>
#include <math.h>

#include "nyx_device.h"
#include "nyx_features.h"
#include "nyx_launch.h"

namespace nyx {

namespace {

constexpr int kNbBlock = 256;
constexpr int kNbWaves = kNbBlock / kWave;

enum NbFeat : int {
    // NGLDM
    NB_DCENRG, NB_DCENT, NB_DCNU, NB_DCNUN, NB_DCM, NB_DCV, NB_GLNU, NB_GLNUN, NB_GLM, NB_GLV, NB_HDE, NB_HDHGLE,
    NB_HDLGLE, NB_HGLCE, NB_LDE, NB_LDHGLE, NB_LDLGLE, NB_LGLCE,
    // NGTDM
    NB_BUSYNESS, NB_COARSENESS, NB_COMPLEXITY, NB_CONTRAST, NB_STRENGTH,
    // GLDM
    NB_G_SDE, NB_G_LDE, NB_G_GLN, NB_G_DN, NB_G_DNN, NB_G_GLV, NB_G_DV, NB_G_DE, NB_G_LGLE, NB_G_HGLE, NB_G_SDLGLE,
    NB_G_SDHGLE, NB_G_LDLGLE, NB_G_LDHGLE, NB_COUNT
};
static_assert(NB_COUNT == kNumNeighbourFeat, "column count");

struct NbShared {
    uint64_t red[kNbWaves];
    uint32_t n_occ;          // levels present in the NGTDM
};

}  // namespace

// LDS bytes of the per-ROI tables for ng levels and nn neighbours.
__host__ __device__ inline uint32_t nb_lds_bytes(uint32_t ng, uint32_t nn) {
    // A (u64, ng * nn) | S (u32, ng * (nn + 1)) | n (u32, ng) | occupied levels (u32, ng) | s (double, ng)
    return ng * nn * 8u + ng * (nn + 1u) * 4u + ng * 4u + ng * 4u + ng * 8u + 16u;
}

// One work-group per ROI: the kNumNeighbourFeat features of ROI blockIdx.x.
// nn_max: neighbours per voxel the LDS tables are laid out for (8 or 26).
template <class OutT>
__global__ __launch_bounds__(kNbBlock) void k_neighbourhood(const ImgDesc *imgs, int n_images, const RoiDesc *rois,
                                                            const uint32_t *n_rois_ptr, uint32_t roi_cap,
                                                            uint32_t ng, uint32_t alpha, uint32_t nn_max,
                                                            OutT *table, uint32_t table_rows, uint32_t *err) {
    __shared__ NbShared S;
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t r = blockIdx.x;
    const uint32_t n_rois = min(*n_rois_ptr, roi_cap);
    if (r >= n_rois) return;
    if (r >= table_rows) {
        if (threadIdx.x == 0) atomicOr(err, (uint32_t)E_TABLE_CAP);
        return;
    }
    const RoiDesc rd = rois[r];
    if (rd.image >= (uint32_t)n_images) return;
    const ImgDesc im = imgs[rd.image];
    if (rd.x0 < 0 || rd.y0 < 0 || rd.z0 < 0 || rd.x1 >= im.nx || rd.y1 >= im.ny || rd.z1 >= im.nz ||
        rd.x0 > rd.x1 || rd.y0 > rd.y1 || rd.z0 > rd.z1)
        return;
    OutT *out = table + (uint64_t)r * kNumNeighbourFeat;
    const bool vol = im.nz > 1;
    const uint32_t nn = vol ? 26u : 8u, nk = nn + 1u;
    if (nn > nn_max) {
        if (threadIdx.x == 0) atomicOr(err, (uint32_t)E_LIST_CAP);
        return;
    }
    uint64_t *A = reinterpret_cast<uint64_t *>(smem);              // ng * nn
    uint32_t *Sd = reinterpret_cast<uint32_t *>(A + ng * nn);       // ng * nk dependence matrix
    uint32_t *cnt = Sd + ng * nk;                                   // ng: voxels with a neighbour
    uint32_t *occ = cnt + ng;                                       // ng: levels present (compacted)
    double *sl = reinterpret_cast<double *>(occ + ng + ((ng & 1u) ? 1u : 0u));   // ng: s_i
    for (uint32_t i = threadIdx.x; i < ng * nn; i += kNbBlock) A[i] = 0ull;
    for (uint32_t i = threadIdx.x; i < ng * nk; i += kNbBlock) Sd[i] = 0u;
    for (uint32_t i = threadIdx.x; i < ng; i += kNbBlock) cnt[i] = 0u;
    if (threadIdx.x == 0) S.n_occ = 0u;
    __syncthreads();

    const uint32_t W = (uint32_t)(rd.x1 - rd.x0 + 1), H = (uint32_t)(rd.y1 - rd.y0 + 1),
                   Dz = (uint32_t)(rd.z1 - rd.z0 + 1);
    const uint32_t nx = (uint32_t)im.nx, plane = (uint32_t)im.ny * nx;
    const uint32_t label = rd.label, vmin = rd.vmin, D = rd.vmax - rd.vmin;
    const float rcpD = D ? 1.0f / (float)D : 0.0f;
    const int zlo = vol ? -1 : 0, zhi = vol ? 1 : 0;
    for (BoxWalk<kNbBlock> b(W, H, Dz); b.ok(); b.next()) {
        const int32_t X = rd.x0 + (int32_t)b.x, Y = rd.y0 + (int32_t)b.y, Z = rd.z0 + (int32_t)b.z;
        const uint32_t v = (uint32_t)Z * plane + (uint32_t)Y * nx + (uint32_t)X;
        if (ldg(im.L, v) != label) continue;
        const uint32_t bv = fbn_level(ldg(im.I, v), vmin, D, rcpD, ng);
        uint32_t wn = 0, tot = 0, dep = 1;
        for (int dz = zlo; dz <= zhi; ++dz) {
            const int32_t wz = Z + dz;
            if (wz < 0 || wz >= im.nz) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int32_t wy = Y + dy;
                if (wy < 0 || wy >= im.ny) continue;
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int32_t wx = X + dx;
                    if ((dz | dy | dx) == 0 || wx < 0 || wx >= im.nx) continue;
                    const uint32_t w = (uint32_t)wz * plane + (uint32_t)wy * nx + (uint32_t)wx;
                    if (ldg(im.L, w) != label) continue;
                    const uint32_t bw = fbn_level(ldg(im.I, w), vmin, D, rcpD, ng);
                    ++wn;
                    tot += bw;
                    dep += (bw > bv ? bw - bv : bv - bw) <= alpha;
                }
            }
        }
        atomicAdd(&Sd[(bv - 1u) * nk + dep - 1u], 1u);
        if (wn) {
            atomicAdd(&cnt[bv - 1u], 1u);
            const uint32_t iw = bv * wn;
            atomicAdd(reinterpret_cast<unsigned long long *>(&A[(bv - 1u) * nn + wn - 1u]),
                      (unsigned long long)(iw > tot ? iw - tot : tot - iw));
        }
    }
    __syncthreads();

    // ---- dependence matrix: exact integer moments and double emphases
    uint64_t Ns = 0, e2 = 0, si = 0, si2 = 0, sk = 0, sk2 = 0, sik2 = 0, rows2 = 0;
    double ent = 0.0, hdl = 0.0, lde = 0.0, ldh = 0.0, ldl = 0.0, lgl = 0.0;
    for (uint32_t c = threadIdx.x; c < ng * nk; c += kNbBlock) {
        const uint32_t q = Sd[c];
        if (!q) continue;
        const uint32_t i0 = c / nk, k = c - i0 * nk + 1u, i = i0 + 1u;
        const uint64_t ii = (uint64_t)i * i, kk = (uint64_t)k * k;
        Ns += q;
        e2 += (uint64_t)q * q;
        si += (uint64_t)i * q;
        si2 += ii * q;
        sk += (uint64_t)k * q;
        sk2 += kk * q;
        sik2 += ii * kk * q;
        const double qd = (double)q, id = (double)ii, kd = (double)kk;
        ent += qd * log2(qd);
        hdl += qd * kd / id;
        lde += qd / kd;
        ldh += qd * id / kd;
        ldl += qd / (id * kd);
        lgl += qd / id;
    }
    for (uint32_t i = threadIdx.x; i < ng; i += kNbBlock) {
        uint64_t row = 0;
        for (uint32_t k = 0; k < nk; ++k) row += Sd[i * nk + k];
        rows2 += row * row;
    }
    uint64_t cols2 = 0;
    for (uint32_t k = threadIdx.x; k < nk; k += kNbBlock) {
        uint64_t col = 0;
        for (uint32_t i = 0; i < ng; ++i) col += Sd[i * nk + k];
        cols2 += col * col;
    }
    Ns = block_sum<kNbWaves>(Ns, S.red);
    e2 = block_sum<kNbWaves>(e2, S.red);
    si = block_sum<kNbWaves>(si, S.red);
    si2 = block_sum<kNbWaves>(si2, S.red);
    sk = block_sum<kNbWaves>(sk, S.red);
    sk2 = block_sum<kNbWaves>(sk2, S.red);
    sik2 = block_sum<kNbWaves>(sik2, S.red);
    rows2 = block_sum<kNbWaves>(rows2, S.red);
    cols2 = block_sum<kNbWaves>(cols2, S.red);
    ent = block_sum<kNbWaves>(ent, S.red);
    hdl = block_sum<kNbWaves>(hdl, S.red);
    lde = block_sum<kNbWaves>(lde, S.red);
    ldh = block_sum<kNbWaves>(ldh, S.red);
    ldl = block_sum<kNbWaves>(ldl, S.red);
    lgl = block_sum<kNbWaves>(lgl, S.red);

    // ---- NGTDM: s_i and the list of levels present
    for (uint32_t i = threadIdx.x; i < ng; i += kNbBlock) {
        double s = 0.0;
        for (uint32_t w = 0; w < nn; ++w) {
            const uint64_t a = A[i * nn + w];
            if (a) s += (double)a / (double)(w + 1u);
        }
        sl[i] = s;
        if (cnt[i]) occ[atomicAdd(&S.n_occ, 1u)] = i;
    }
    __syncthreads();
    const uint32_t ngp = S.n_occ;
    uint64_t nvp = 0;
    double ps = 0.0, ssum = 0.0;
    for (uint32_t q = threadIdx.x; q < ngp; q += kNbBlock) {
        const uint32_t i = occ[q];
        nvp += cnt[i];
        ssum += sl[i];
    }
    nvp = block_sum<kNbWaves>(nvp, S.red);
    ssum = block_sum<kNbWaves>(ssum, S.red);
    const double nvpd = (double)nvp, inv_nvp = nvp ? 1.0 / nvpd : 0.0;
    for (uint32_t q = threadIdx.x; q < ngp; q += kNbBlock) {
        const uint32_t i = occ[q];
        ps += (double)cnt[i] * inv_nvp * sl[i];
    }
    ps = block_sum<kNbWaves>(ps, S.red);
    // pair sums over the levels present (both orders, as the definitions run)
    double con = 0.0, bden = 0.0, cpx = 0.0, str = 0.0;
    for (uint32_t q = threadIdx.x; q < ngp * ngp; q += kNbBlock) {
        const uint32_t a = q / ngp, c = q - a * ngp;
        const uint32_t i = occ[a], j = occ[c];
        const double pi = (double)cnt[i] * inv_nvp, pj = (double)cnt[j] * inv_nvp;
        const double li = (double)(i + 1u), lj = (double)(j + 1u), d = li - lj;
        con += pi * pj * d * d;
        bden += fabs(li * pi - lj * pj);
        cpx += fabs(d) * (pi * sl[i] + pj * sl[j]) / (pi + pj);
        str += (pi + pj) * d * d;
    }
    con = block_sum<kNbWaves>(con, S.red);
    bden = block_sum<kNbWaves>(bden, S.red);
    cpx = block_sum<kNbWaves>(cpx, S.red);
    str = block_sum<kNbWaves>(str, S.red);

    if (threadIdx.x != 0) return;
    double f[NB_COUNT];
    const double nsd = (double)Ns, inv = 1.0 / nsd, ns2 = nsd * nsd;
    f[NB_DCENRG] = (double)e2 / ns2;
    f[NB_DCENT] = log2(nsd) - ent * inv;
    f[NB_DCNU] = (double)cols2 * inv;
    f[NB_DCNUN] = (double)cols2 / ns2;
    f[NB_DCM] = (double)sk * inv;
    f[NB_DCV] = u128_to_double((u128)Ns * sk2 - (u128)sk * sk) / ns2;
    f[NB_GLNU] = (double)rows2 * inv;
    f[NB_GLNUN] = (double)rows2 / ns2;
    f[NB_GLM] = (double)si * inv;
    f[NB_GLV] = u128_to_double((u128)Ns * si2 - (u128)si * si) / ns2;
    f[NB_HDE] = (double)sk2 * inv;
    f[NB_HDHGLE] = (double)sik2 * inv;
    f[NB_HDLGLE] = hdl * inv;
    f[NB_HGLCE] = (double)si2 * inv;
    f[NB_LDE] = lde * inv;
    f[NB_LDHGLE] = ldh * inv;
    f[NB_LDLGLE] = ldl * inv;
    f[NB_LGLCE] = lgl * inv;
    if (nvp == 0) {
        f[NB_BUSYNESS] = f[NB_COARSENESS] = f[NB_COMPLEXITY] = f[NB_CONTRAST] = f[NB_STRENGTH] = __builtin_nan("");
    } else {
        f[NB_COARSENESS] = ps > 0.0 ? 1.0 / ps : 1.0e6;
        f[NB_CONTRAST] = ngp > 1u ? con / ((double)ngp * (double)(ngp - 1u)) * ssum * inv_nvp : 0.0;
        f[NB_BUSYNESS] = bden > 0.0 ? ps / bden : 0.0;
        f[NB_COMPLEXITY] = cpx * inv_nvp;
        f[NB_STRENGTH] = ssum > 0.0 ? str / ssum : 0.0;
    }
    f[NB_G_SDE] = f[NB_LDE];
    f[NB_G_LDE] = f[NB_HDE];
    f[NB_G_GLN] = f[NB_GLNU];
    f[NB_G_DN] = f[NB_DCNU];
    f[NB_G_DNN] = f[NB_DCNUN];
    f[NB_G_GLV] = f[NB_GLV];
    f[NB_G_DV] = f[NB_DCV];
    f[NB_G_DE] = f[NB_DCENT];
    f[NB_G_LGLE] = f[NB_LGLCE];
    f[NB_G_HGLE] = f[NB_HGLCE];
    f[NB_G_SDLGLE] = f[NB_LDLGLE];
    f[NB_G_SDHGLE] = f[NB_LDHGLE];
    f[NB_G_LDLGLE] = f[NB_HDLGLE];
    f[NB_G_LDHGLE] = f[NB_HDHGLE];
    for (int k = 0; k < NB_COUNT; ++k) out[k] = (OutT)f[k];
}

uint32_t neighbourhood_lds_bytes(uint32_t ng, int any_volume) { return nb_lds_bytes(ng, any_volume ? 26u : 8u); }

hipError_t launch_neighbourhood(const StepArgs &a, uint32_t grid, int fp64, uint32_t alpha, int any_volume,
                                void *table, uint32_t table_rows, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    const uint32_t nn = any_volume ? 26u : 8u;
    const uint32_t lds = nb_lds_bytes((uint32_t)a.ng, nn);
    const void *f = fp64 ? reinterpret_cast<const void *>(&k_neighbourhood<double>)
                         : reinterpret_cast<const void *>(&k_neighbourhood<float>);
    // the dynamic tables plus the static NbShared stay within the CU's 160 KB
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (fp64)
        hipLaunchKernelGGL(k_neighbourhood<double>, dim3(grid), dim3(kNbBlock), lds, st, a.imgs, a.n_images, a.rois,
                           a.counters + C_NROIS, a.roi_cap, (uint32_t)a.ng, alpha, nn,
                           reinterpret_cast<double *>(table), table_rows, a.counters + C_ERR);
    else
        hipLaunchKernelGGL(k_neighbourhood<float>, dim3(grid), dim3(kNbBlock), lds, st, a.imgs, a.n_images, a.rois,
                           a.counters + C_NROIS, a.roi_cap, (uint32_t)a.ng, alpha, nn,
                           reinterpret_cast<float *>(table), table_rows, a.counters + C_ERR);
    return hipGetLastError();
}

}  // namespace nyx
