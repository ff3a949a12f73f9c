/* Device formation of the log-derivative matrix O on MI355X (gfx950).
 *
 * O_k(x) = d log psi_theta(x) / d theta_k, one row per sample x and one
 * column per parameter (paper, Sec. 2: the definition that follows Eq. 2; the
 * columns are grouped into the layer blocks of Eq. 3).  These calls produce
 * the input of qgt_block_form directly in device memory, for the network
 * families that stand in for the paper's Vision Transformer: an RBM, dense
 * feed-forward networks and periodic convolutional networks.  The networks are
 * holomorphic in their complex parameters: O is the plain complex derivative.
 *
 * Common conventions
 *   theta      device, complex128 (interleaved re/im), n_p entries in the flat
 *              parameter order given per network below.
 *   x          device, int8, n_s rows of N spin values (+1/-1; any int8 value
 *              is taken as the number it is), row stride ldx >= N elements.
 *   O          device, row-major n_s x n_p, row stride ldo >= n_p elements,
 *              complex64 or complex128 (qgt_dtype).  Every entry is computed
 *              in FP64 and rounded once to the output type.
 *   workspace  device, at least the queried number of bytes, 256-byte
 *              aligned: per-sample activations and derivatives, overwritten.
 *   stream     every kernel runs on this stream; nothing is allocated and no
 *              synchronisation is made, so the calls can be captured in a HIP
 *              graph.
 * The caller owns every buffer.  Argument errors return synchronously
 * (QGT_ERR_INVALID_ARGUMENT, QGT_ERR_UNSUPPORTED for sizes beyond the limits
 * below, QGT_ERR_WORKSPACE_TOO_SMALL); a failed launch returns QGT_ERR_HIP.
 * Detail: qgt_last_error().
 *
 * logcosh(z) = s z + log1p(exp(-2 s z)) - log 2 with s = +1 if Re z >= 0 else
 * -1 (one fixed branch of log cosh; its derivative is tanh z on either branch).
 */
#ifndef QGT_JACOBIAN_H
#define QGT_JACOBIAN_H

#include "qgt_block.h"

#ifdef __cplusplus
extern "C" {
#endif

/* RBM with N visible and M hidden units:
 *   log psi(x) = sum_i a_i x_i + sum_j logcosh(b_j + sum_i W_ji x_i).
 * theta = [W (M x N, row-major) | b (M) | a (N)], n_p = M N + M + N; the
 * three blocks are W, b and a.  O rows: [tanh(t_j) x_i | tanh(t_j) | x_i] with
 * t = W x + b.  Limits: N, M in [1, 65535], n_s in [1, 2^24], the number
 * of workgroups (n_s times the row tasks, about n_p / 4096 + 2) below 2^31. */
size_t qgt_rbm_jacobian_workspace_bytes(int32_t n_visible, int32_t n_hidden, int64_t n_s);
qgt_status qgt_rbm_jacobian(int32_t n_visible, int32_t n_hidden, const void* theta, const int8_t* x,
                            int64_t ldx, int64_t n_s, qgt_dtype o_dtype, void* O, int64_t ldo,
                            void* workspace, size_t ws_bytes, hipStream_t stream);

/* Feed-forward network of L dense logcosh layers:
 *   h^0 = x,  z^l = W^l h^{l-1} + b^l,  h^l = logcosh(z^l)  (l = 1..L),
 *   log psi = sum_k h^L_k, or v . h^L + c with a dense readout.
 * widths (host) holds the L + 1 widths [N, w_1, ..., w_L].  theta =
 * [W^1 (w_1 x N, row-major) | b^1 | W^2 | b^2 | ... | W^L | b^L (| v | c)];
 * each layer (and the readout) is one block.  O rows, layer l:
 * g^l_j h^{l-1}_i then g^l_j, with g^l = d log psi / d z^l from the chain rule
 * (g^L = tanh(z^L) times v or 1; g^{l-1} = tanh(z^{l-1}) * (W^l)^T g^l); the
 * readout block is h^L then 1.  Limits: 1 <= L <= 8, widths in [1, 65535],
 * n_p below 2^31, n_s in [1, 2^24], the number of workgroups (n_s times the
 * row tasks, about n_p / 4096 + L + 1) below 2^31. */
typedef struct {
  int32_t n_layers;        /* L */
  const int32_t* widths;   /* host, L + 1 entries */
  int32_t readout;         /* 0: sum of the last layer; 1: dense readout v . h^L + c */
} qgt_ffnn;

int64_t qgt_ffnn_n_params(const qgt_ffnn* net);  /* -1 on invalid arguments */
size_t qgt_ffnn_jacobian_workspace_bytes(const qgt_ffnn* net, int64_t n_s);  /* 0 on invalid arguments */
qgt_status qgt_ffnn_jacobian(const qgt_ffnn* net, const void* theta, const int8_t* x, int64_t ldx,
                             int64_t n_s, qgt_dtype o_dtype, void* O, int64_t ldo, void* workspace,
                             size_t ws_bytes, hipStream_t stream);

/* Convolutional network on a periodic side x side lattice (sites row-major):
 *   h^0 = the spins as one channel,
 *   z^l[c, y, x] = b^l[c] + sum_{c', dy, dx} K^l[c, c', dy, dx]
 *                  h^{l-1}[c', (y + dy - 1) mod side, (x + dx - 1) mod side],
 *   h^l = logcosh(z^l)  (l = 1..L),   log psi = sum_{c, y, x} h^L[c, y, x].
 * theta = [K^1 (channels x 1 x 3 x 3) | b^1 | K^2 (channels x channels x 3 x 3)
 * | b^2 | ...]; each layer is one block.  O rows, layer l: the kernel
 * derivatives sum_sites g^l[c, y, x] h^{l-1}[c', y + dy - 1, x + dx - 1] in
 * the kernel's index order, then the bias derivatives sum_sites g^l[c, .],
 * with g^l = d log psi / d z^l from the chain rule (g^L = tanh(z^L); the
 * derivative reaching h^{l-1} is the correlation of g^l with the kernel taken
 * the other way, times tanh(z^{l-1})).  x holds side^2 spins per sample.
 * Limits: 1 <= L <= 8, channels in [1, 16], side >= 2 with
 * (32 channels + 18) side^2 <= 65536 (e.g. 16 channels up to 11 x 11;
 * (16 + 18) side^2 with one layer), n_s in [1, 2^24]. */
typedef struct {
  int32_t side;            /* lattice side */
  int32_t channels;        /* channels of every layer (the input has one) */
  int32_t n_layers;        /* L */
} qgt_cnn;

int64_t qgt_cnn_n_params(const qgt_cnn* net);  /* -1 on invalid arguments */
size_t qgt_cnn_jacobian_workspace_bytes(const qgt_cnn* net, int64_t n_s);  /* 0 on invalid arguments */
qgt_status qgt_cnn_jacobian(const qgt_cnn* net, const void* theta, const int8_t* x, int64_t ldx,
                            int64_t n_s, qgt_dtype o_dtype, void* O, int64_t ldo, void* workspace,
                            size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* QGT_JACOBIAN_H */
