// ss_mlp.hip -- the learned footprint f_theta (Sec. 2.2) on gfx950 matrix cores.
//
// Network: 5 -> 64 -> 64 -> 64 -> 64 -> 1, SiLU after each hidden layer.
// Precision split: fold, frame and layer 1 in FP32 (layer 1 on the FP32
// matrix core, v_mfma_f32_32x32x2_f32); the three 64x64 layers on the BF16
// matrix core with FP32 accumulation (v_mfma_f32_32x32x16_bf16); SiLU in
// FP32, its result rounded to BF16 (nearest even) when it feeds a BF16 layer;
// output layer in FP32.  The network value is multiplied by the indicator
// that the line meets the basis support (exact slab test), so the pair set
// equals the quadrature form's.
//
// Tile layout.  A wave evaluates 32 (line, basis) pairs at a time, pairs
// along the N (column) dimension of the MFMA.  The 32x32 accumulator of an
// MFMA puts column j in lanes j and j + 32; lane l, register r holds row
// 8 (r / 4) + 4 (l / 32) + (r % 4).  The next layer's B operand needs, in
// lane l, the K slots 8 (l / 32) + e (e < 8) of each 16-wide K step.  The
// hidden units are therefore renumbered so that K step kk of a layer reads
// accumulator block kk / 2, registers 8 (kk % 2) + e of the *same* lane: the
// K slot 16 kk + 8 h + e holds unit 16 kk + 8 (e / 4) + 4 h + (e % 4).  The
// weight image (built on the host from the blob) bakes this permutation
// into the A operands, so activations never leave their lane.
#include "ss_kernels.hpp"

#include <cstring>

namespace ss {

constexpr int HID = 64;

// Weight image, kept in LDS by the kernels (27.4 KB).
struct MlpImage {
    float w1a[2][3][64];       // layer-1 A operand: [row block][K step][lane]
    float bias[4][2][32];      // [layer][lane half][block * 16 + reg]
    uint32_t wh[3][2][4][64][4];  // hidden A operands: 8 bf16 per lane
    float wout[2][32];         // [lane half][block * 16 + reg]
    float bout;
    float pad[3];
};

// accumulator (block b, register r) of lane half hf -> hidden unit
__host__ __device__ constexpr int acc_unit(int b, int r, int hf) { return 32 * b + 8 * (r / 4) + 4 * hf + (r % 4); }
// K slot of a hidden layer's input -> hidden unit
__host__ __device__ constexpr int kslot_unit(int ks) {
    return 16 * (ks / 16) + 8 * ((ks % 8) / 4) + 4 * ((ks % 16) / 8) + (ks % 4);
}

namespace {

struct BlobHeader {
    char magic[8];
    uint32_t version, degree, in, hidden, depth, act, fold, seed;
    float rel_fp32, rel_bf16;
};
static_assert(sizeof(BlobHeader) == 48, "blob header layout");

constexpr size_t BLOB_BODY = 4 * (HID * 5 + HID) + 3 * (2 * HID * HID + 4 * HID) + 4 * (HID + 1);

}  // namespace

ss_status mlp_blob_to_image(const void *blob, size_t bytes, int degree, std::vector<unsigned char> &image) {
    if (bytes != sizeof(BlobHeader) + BLOB_BODY)
        return fail(SS_EBLOB, "weight blob has %zu bytes, expected %zu", bytes, sizeof(BlobHeader) + BLOB_BODY);
    BlobHeader hd;
    std::memcpy(&hd, blob, sizeof hd);
    static const char MAGIC[8] = {'S', 'S', 'M', 'L', 'P', 0, 0, 1};
    if (std::memcmp(hd.magic, MAGIC, 8) != 0) return fail(SS_EBLOB, "weight blob: bad magic");
    if (hd.version != 1) return fail(SS_EBLOB, "weight blob: version %u, expected 1", hd.version);
    if ((int)hd.degree != degree)
        return fail(SS_EBLOB, "weight blob trained for degree %u, context has degree %d", hd.degree, degree);
    if (hd.in != 5 || hd.hidden != HID || hd.depth != 4 || hd.act != 1 || hd.fold != 1)
        return fail(SS_EBLOB, "weight blob: unsupported architecture (in %u hidden %u depth %u act %u fold %u)",
                    hd.in, hd.hidden, hd.depth, hd.act, hd.fold);
    const unsigned char *p = (const unsigned char *)blob + sizeof(BlobHeader);
    float W1[HID][5], b1[HID], bh[3][HID], wo[HID], bo;
    uint16_t Wh[3][HID][HID];
    std::memcpy(W1, p, sizeof W1); p += sizeof W1;
    std::memcpy(b1, p, sizeof b1); p += sizeof b1;
    for (int l = 0; l < 3; ++l) {
        std::memcpy(Wh[l], p, sizeof Wh[l]); p += sizeof Wh[l];
        std::memcpy(bh[l], p, sizeof bh[l]); p += sizeof bh[l];
    }
    std::memcpy(wo, p, sizeof wo); p += sizeof wo;
    std::memcpy(&bo, p, sizeof bo);
    for (int u = 0; u < HID; ++u) {
        for (int k = 0; k < 5; ++k)
            if (!std::isfinite(W1[u][k])) return fail(SS_EBLOB, "weight blob: non-finite layer-1 weight");
        if (!std::isfinite(b1[u]) || !std::isfinite(wo[u])) return fail(SS_EBLOB, "weight blob: non-finite value");
    }
    if (!std::isfinite(bo)) return fail(SS_EBLOB, "weight blob: non-finite output bias");
    MlpImage im;
    std::memset(&im, 0, sizeof im);
    for (int b = 0; b < 2; ++b)
        for (int kk = 0; kk < 3; ++kk)
            for (int l = 0; l < 64; ++l) {
                const int unit = 32 * b + (l % 32), feat = 2 * kk + l / 32;
                im.w1a[b][kk][l] = feat < 5 ? W1[unit][feat] : 0.0f;
            }
    for (int hf = 0; hf < 2; ++hf)
        for (int b = 0; b < 2; ++b)
            for (int r = 0; r < 16; ++r) {
                const int u = acc_unit(b, r, hf);
                im.bias[0][hf][b * 16 + r] = b1[u];
                for (int l = 0; l < 3; ++l) im.bias[l + 1][hf][b * 16 + r] = bh[l][u];
                im.wout[hf][b * 16 + r] = wo[u];
            }
    for (int l = 0; l < 3; ++l)
        for (int b = 0; b < 2; ++b)
            for (int kk = 0; kk < 4; ++kk)
                for (int ln = 0; ln < 64; ++ln) {
                    const int out = 32 * b + (ln % 32);
                    uint16_t v[8];
                    for (int e = 0; e < 8; ++e) v[e] = Wh[l][out][kslot_unit(16 * kk + 8 * (ln / 32) + e)];
                    std::memcpy(im.wh[l][b][kk][ln], v, sizeof v);
                }
    im.bout = bo;
    image.resize(sizeof im);
    std::memcpy(image.data(), &im, sizeof im);
    return SS_OK;
}

hipError_t launch_project_mlp(int, const LaunchArgs &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_backproject_mlp(int, const LaunchArgs &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_footprint_mlp(int, const void *, const float *, const float *, int, float *, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace ss
