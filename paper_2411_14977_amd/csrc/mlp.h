// Element-local MLP (learned smoothing stage): BF16 MFMA kernels with FP32 accumulation,
// training driver (forward, backward, Adam) and the fused inference kernels of the V-cycle.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace semm {

constexpr int NH = 128;  // hidden width

inline int pad16(int n) { return (n + 15) / 16 * 16; }

// Host copy of the network in FP32 (unpadded, row-major): W1 [nin x NH], b1, W2 [NH x NH], b2,
// W3 [NH x nout], b3.
struct Net {
  int nin = 0, nout = 0;
  uint64_t seed = 0;
  float train_loss = 0.f, val_loss = 0.f;
  int epochs = 0, steps = 0;
  std::vector<float> W1, b1, W2, b2, W3, b3;
  size_t nparams() const { return W1.size() + b1.size() + W2.size() + b2.size() + W3.size() + b3.size(); }
};

// blob = 64-byte header + parameters in the order above
size_t blob_size(int nin, int nout);
bool net_from_blob(const void* blob, size_t nbytes, Net& net, std::string& err);
void net_to_blob(const Net& net, void* blob);
void net_init(Net& net, int nin, int nout, uint64_t seed);   // U(+-1/sqrt(fan_in)), b = 0

// ---- generic BF16 GEMM: C[m][n] (+)= sum_k A(m,k) B(k,n), A(m,k) = A[m*sam + k*sak],
// B(k,n) = B[k*sbk + n*sbn] (bf16 bits), C fp32 row-major with ldc.  M, N, K multiples of 16.
// Optional epilogue of a product with ldc columns of hidden units (row r, column n, sum s):
//   BIAS_GELU:  z = s + bias[n];        C = z, Hb = bf16(GELU(z))
//   GELU_BACK:  g = s GELU'(Zin[r][n]);  C = g, Hb = bf16(g)
// each also writing the bf16 value batch-major into HT[n * ldT + r] when HT is given.
struct GemmEpi {
  enum Kind { BIAS_GELU = 1, GELU_BACK = 2 } kind;
  const float* bias;
  const float* Zin;
  uint16_t* Hb;
  uint16_t* HT;
  int ldT;
};
hipError_t gemm_bf16(const uint16_t* A, long sam, long sak, const uint16_t* B, long sbk, long sbn,
                     float* C, int ldc, int M, int N, int K, int accumulate, hipStream_t st,
                     const GemmEpi* epi = nullptr);
hipError_t to_bf16_padded(const float* src, int rows, int cols, int lds, uint16_t* dst, int ldd,
                          int dcols, const int* rowidx, hipStream_t st, uint16_t* dstT = nullptr,
                          int ldT = 0);

hipError_t add_bias(float* Z, const float* b, int rows, int cols, hipStream_t st);
constexpr int MAX_STAGE_OUT = 96;  // the fused inference kernel handles (P+1)^2 <= 96 (P <= 8)
constexpr int MAX_STAGE_P3 = 6;    // hexahedra: (P+1)^3 <= 343

struct TrainCfg {
  int epochs = 30, batch = 1024;
  float lr = 1e-3f;
  uint64_t seed = 1234;
  float val_frac = 0.1f;
};

// Train on device samples X [n x nin] and T [n x nout] (fp32, row-major).  On return net holds
// the trained FP32 weights; losses (optional) gets 2 floats per epoch (train, validation).
// init (optional): start from these weights instead of the seeded draw.
bool train(const float* X, const float* T, int n, int nin, int nout, const TrainCfg& cfg, Net& net,
           std::vector<float>* losses, hipStream_t st, std::string& err,
           const Net* init = nullptr);

// Batched forward with the training kernels (test hook): Y [n x nout] fp32.
bool forward(const Net& net, const float* X, int n, float* Y, hipStream_t st, std::string& err);
// Loss and parameter gradients for one batch (test hook); grads packed like the blob.
bool gradients(const Net& net, const float* X, const float* T, int n, float* grads, float* loss,
               hipStream_t st, std::string& err);

// The same forward with no device allocation: the network and the activations of one chunk of
// 256 rows sit in a file-scope device array of forward_noalloc_bytes() bytes (one per GPU, kept
// until the process ends).  nin <= 416, nout <= 96.  Runs on the null stream and synchronises
// it; two calls that overlap on one GPU use the same array and race.
bool forward_noalloc(const void* blob, size_t nbytes, const float* X, int n, float* Y,
                     std::string& err);
size_t forward_noalloc_bytes();

// ---- inference state of one solver context (2D element columns) ----------------------------
struct Stage {
  bool enabled = false;
  int dim = 2;
  int nin = 0, nout = 0, P = 0, Nx = 0, Ny = 1, Nz = 0, nyn = 1, nzn = 0;
  size_t E = 0;
  // bf16, padded, transposed (output-major) and stored in MFMA A-operand fragment order:
  // fragment (t, k) of an [M][K] matrix holds rows 16t.., columns 16k.. as 64 lanes x 4 values
  // (lane l: row 16t + l%16, columns 16k + 4(l/16) + 0..3); W1r [NH][KR], W2 [NH][NH], W3 [N3][NH]
  uint16_t *W1r = nullptr, *W2 = nullptr, *W3 = nullptr;
  float *b2 = nullptr, *b3 = nullptr;
  float* Z1geo = nullptr;   // [E x NH] = geometric part of layer 1 + b1
  float* abar = nullptr;    // [E] mean of the element-matrix diagonal
  float* CE = nullptr;      // [E x nout] element-local corrections (layout semk::ce_index)
  int* skips = nullptr;     // device counter of rejected stages
  std::vector<void*> allocs;
};

// One learned stage on the fine level (precision dbl ? double : float), driven by the caller:
//   the residual r = b - A x (semk::resid2d), stage_mlp (c_e, c.r), stage_assemble (c), the
//   caller's apply of c with c.q partials, stage_update (alpha, x, R).
// c_e for every element from the complete residual vector r, and each block's part of c . r
// (c the assembled correction, zero on the Dirichlet surface when masked) in
// pcr[0 .. stage_mlp_blocks)
hipError_t stage_mlp(const Stage& s, bool dbl, const void* r, int masked, double* pcr,
                     hipStream_t st);
int stage_mlp_blocks(size_t E);  // workgroups of stage_mlp (entries of its c . r partials)
// c = W sum_e R_e^T c_e, zero on the Dirichlet surface when masked
hipError_t stage_assemble(const Stage& s, bool dbl, void* c, int masked, hipStream_t st);
// alpha = c.r / c.q from the partials (ncr of c.r, ncq of c.q); R holds r on entry; if accepted
// x += alpha c and R = r - alpha q (q = yq + Sq, the side-buffer form of A c; Sq null: q = yq
// complete), else R = r and skips[0] += 1.  With dinv (post-smoothing follows): also the first
// smoothing step from the stage's residual, dn = sr dinv R, d = dn (store_d), x += dn.
hipError_t stage_update(bool dbl, void* x, void* R, const void* c, const void* yq, const void* Sq,
                        const double* pcr, int ncr, const double* pcq, int ncq, int* skips,
                        unsigned N, unsigned nzn, unsigned P, const void* dinv, void* d,
                        double sr, int store_d, hipStream_t st);
// Training features of an assembled residual r on a 2D mesh: X [E x 5n] fp32; targets T [E x n]
// fp32 from the error e ((a_e/s_e) R_e e) or, if e is null, from the element-block inverses
// Ainv [E x n x n] ((a_e/s_e) Ainv_e R_e r).  elist (device, nrows entries): write row k for
// element elist[k] only; null: row e for every element e.
hipError_t features(const double* r, const double* e, const double* Ainv, const float* geo,
                    const float* abar, float* X, float* T, size_t E, int P, int Nz, int nzn,
                    hipStream_t st, const int* elist = nullptr, size_t nrows = 0);
// The same for hexahedra (3D, X [rows x 7n]; geo [E x 6n]).
hipError_t features3d(const double* r, const double* e, const double* Ainv, const float* geo,
                      const float* abar, float* X, float* T, size_t E, int P, int Ny, int Nz,
                      int nyn, int nzn, hipStream_t st, const int* elist = nullptr,
                      size_t nrows = 0);

}  // namespace semm
