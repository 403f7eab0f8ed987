"""GPU parity of the float-float GEMM.

* FMA loop: bit-exact against the oracle's plain float-float GEMM (Add22
  accumulation of Mul22 terms, k ascending).
* Sliced (int8 and BF16 digits on matrix cores): against the exact product
  (long accumulator) entry by entry, normwise |C - exact| <= 2^-44 (|A||B|);
  exactly equal to each other (both sum the same digit products exactly);
  exact on integer data and on A times the identity when every row of A sits
  in one binade; on rows and columns spanning 40 binades, within the bound
  the algorithm documents for that case.
"""
import math
import sys
from fractions import Fraction

import numpy as np
import pytest
import torch

import ff_inputs as fi
import oracle
from fpexact import frac, same_bits

pytestmark = pytest.mark.gpu

TWO_M44 = Fraction(1, 1 << 44)


def _ff():
    import paper_cs_0603115_amd as ff
    return ff


def _announce(msg):
    print(msg, file=sys.stderr, flush=True)


def check_entries(A, B, C, rows, cols, label, target=TWO_M44):
    """C at (rows x cols) against the exact product, normwise."""
    An, Bn, Cn = A.cpu().numpy(), B.cpu().numpy(), C.cpu().numpy()
    ri, ci = np.meshgrid(np.asarray(rows), np.asarray(cols), indexing="ij")
    ri, ci = ri.ravel(), ci.ravel()
    exact = oracle.exact_gemm_entries(An[0], An[1], Bn[0], Bn[1], ri, ci)
    scale = oracle.exact_absgemm_entries(An[0], An[1], Bn[0], Bn[1], ri, ci)
    worst = -math.inf
    for t, (i, j) in enumerate(zip(ri, ci)):
        err = abs(frac(Cn[0, i, j]) + frac(Cn[1, i, j]) - exact[t])
        if scale[t] == 0:
            assert err == 0, (label, i, j)
            continue
        assert err <= target * scale[t], (label, i, j, float(err / scale[t]))
        if err:
            worst = max(worst, math.log2(err / scale[t]))
    return worst


ALGOS = ["i8", "bf16"]


def _algo(name):
    ff = _ff()
    return {"i8": ff.GEMM_SLICED_I8, "bf16": ff.GEMM_SLICED_BF16, "fma": ff.GEMM_FMA_LOOP}[name]


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (5, 3, 7), (64, 64, 64), (100, 70, 333),
                                   (130, 257, 200), (33, 65, 1000)])
def test_fma_loop_is_bitexact(M, N, K):
    ff = _ff()
    A = fi.gaussian_ff((M, K), 11 + M)
    B = fi.gaussian_ff((K, N), 12 + N)
    C = ff.ff_gemm(A.cuda(), B.cuda(), algo=ff.GEMM_FMA_LOOP).cpu().numpy()
    Ch, Cl = oracle.gemm_ff_seq(A[0].numpy(), A[1].numpy(), B[0].numpy(), B[1].numpy())
    assert same_bits(C[0], Ch) and same_bits(C[1], Cl)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (5, 3, 7), (64, 64, 64), (100, 70, 333),
                                   (130, 257, 200), (33, 65, 1000)])
def test_sliced_against_exact(algo, M, N, K):
    ff = _ff()
    A = fi.gaussian_ff((M, K), 21 + M).cuda()
    B = fi.gaussian_ff((K, N), 22 + N).cuda()
    C = ff.ff_gemm(A, B, algo=_algo(algo))
    check_entries(A, B, C, range(M), range(N), f"{algo} {M}x{N}x{K}")


def test_sliced_int8_and_bf16_agree_bitwise():
    ff = _ff()
    A = fi.gaussian_ff((200, 700), 31).cuda()
    B = fi.gaussian_ff((700, 150), 32).cuda()
    C8 = ff.ff_gemm(A, B, algo=ff.GEMM_SLICED_I8)
    C16 = ff.ff_gemm(A, B, algo=ff.GEMM_SLICED_BF16)
    again = ff.ff_gemm(A, B, algo=ff.GEMM_SLICED_I8)
    assert torch.equal(C8.view(torch.int32), C16.view(torch.int32))
    assert torch.equal(C8.view(torch.int32), again.view(torch.int32))


@pytest.mark.parametrize("algo", ALGOS + ["fma"])
def test_integer_matrices_are_exact(algo):
    ff = _ff()
    rng = np.random.default_rng(41)
    Ai = rng.integers(-3000, 3000, (96, 300))
    Bi = rng.integers(-3000, 3000, (300, 80))
    A = torch.stack([torch.from_numpy(Ai.astype(np.float32)), torch.zeros(96, 300)]).cuda()
    B = torch.stack([torch.from_numpy(Bi.astype(np.float32)), torch.zeros(300, 80)]).cuda()
    C = ff.ff_gemm(A, B, algo=_algo(algo)).cpu().numpy()
    want = Ai @ Bi
    got = C[0].astype(np.int64) + C[1].astype(np.int64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("algo", ALGOS)
def test_identity_reproduces_single_binade_rows(algo):
    # rows of A inside one binade: the 54-bit fixed point holds every entry's
    # 48 significant bits, and B = I keeps one digit-pair column per entry
    ff = _ff()
    M, K = 70, 96
    mant = fi.random_ff(M * K, 51, 0, 0, max_gap=5).reshape(2, M, K).abs()   # hi in [1, 2)
    lo_sign = torch.sign(fi.random_ff(M * K, 52, 0, 0)[1]).reshape(M, K)
    mant[1] *= lo_sign
    scale = torch.exp2(torch.randint(-20, 20, (M, 1)).float())
    A = (mant * scale).cuda()
    B = torch.stack([torch.eye(K), torch.zeros(K, K)]).cuda()
    C = ff.ff_gemm(A, B, algo=_algo(algo))
    # high words bit for bit; low words by value (an exact zero comes back +0)
    assert torch.equal(C[0].view(torch.int32), A[0].view(torch.int32))
    assert torch.equal(C[1], A[1])


def test_long_k_is_split_into_exact_chunks():
    ff = _ff()
    M, N, K = 64, 48, 16384 + 96
    A = fi.gaussian_ff((M, K), 61).cuda()
    B = fi.gaussian_ff((K, N), 62).cuda()
    for algo in ALGOS:
        C = ff.ff_gemm(A, B, algo=_algo(algo))
        check_entries(A, B, C, range(0, M, 7), range(0, N, 5), f"{algo} long K")


def test_zero_k_gives_zero():
    ff = _ff()
    A = torch.zeros(2, 5, 0, device="cuda")
    B = torch.zeros(2, 0, 6, device="cuda")
    for algo in ALGOS + ["fma"]:
        C = ff.ff_gemm(A, B, algo=_algo(algo))
        torch.cuda.synchronize()
        assert C.shape == (2, 5, 6) and torch.count_nonzero(C) == 0


def test_full_size_4096():
    # C = A B, M = N = K = 4096, entries normal(0,1) split into float-float:
    # 16 seeded 64 x 64 blocks (corners included) against the exact product,
    # the FMA loop bit-exact on one block.
    ff = _ff()
    n = 4096
    _announce("[gpu] gemm 4096^3: generating")
    A = fi.gaussian_ff((n, n), 115004, device="cuda")
    B = fi.gaussian_ff((n, n), 115014, device="cuda")
    _announce("[gpu] gemm 4096^3: sliced int8 and bf16")
    C8 = ff.ff_gemm(A, B, algo=ff.GEMM_SLICED_I8)
    C16 = ff.ff_gemm(A, B, algo=ff.GEMM_SLICED_BF16)
    torch.cuda.synchronize()
    assert torch.equal(C8.view(torch.int32), C16.view(torch.int32))
    rng = np.random.default_rng(115004)
    starts = [(0, 0), (0, n - 64), (n - 64, 0), (n - 64, n - 64)]
    starts += [tuple(int(v) for v in rng.integers(0, n - 64, 2)) for _ in range(12)]
    worst = -math.inf
    for bi, (r0, c0) in enumerate(starts):
        _announce(f"  block {bi} at ({r0}, {c0})")
        w = check_entries(A, B, C8, range(r0, r0 + 64), range(c0, c0 + 64), f"block {r0},{c0}")
        worst = max(worst, w)
    _announce(f"  sliced worst normwise log2 error {worst:.2f}")
    _announce("[gpu] gemm 4096^3: FMA loop, one block bit-exact")
    Cp = ff.ff_gemm(A, B, algo=ff.GEMM_FMA_LOOP)
    torch.cuda.synchronize()
    r0, c0 = starts[5]
    An, Bn = A.cpu().numpy(), B.cpu().numpy()
    Ch, Cl = oracle.gemm_ff_seq(An[0], An[1], Bn[0], Bn[1], rows=(r0, r0 + 64), cols=(c0, c0 + 64))
    Cpn = Cp[:, r0:r0 + 64, c0:c0 + 64].cpu().numpy()
    assert same_bits(Cpn[0], Ch) and same_bits(Cpn[1], Cl)
    del A, B, C8, C16, Cp
    torch.cuda.empty_cache()


@pytest.mark.parametrize("algo", ALGOS + ["fma"])
def test_zero_rows_columns_and_power_of_two_maxima(algo):
    # an all-zero row of A and column of B (no largest entry to scale by)
    # give exact zero words; rows and columns whose largest magnitude is an
    # exact power of two (the boundary of the scale choice) and rows holding
    # a single nonzero entry stay within the normwise bound
    M, K, N = 70, 129, 66
    _announce(f"[gpu] gemm zero rows/columns and power-of-two maxima ({algo})")
    A = fi.gaussian_ff((M, K), 7401)
    B = fi.gaussian_ff((K, N), 7402)
    A[:, 3] = 0.0
    B[:, :, 5] = 0.0
    A[:, 10] = 0.0
    A[0, 10, 17] = 2.0 ** 7                      # a single power-of-two entry
    A[:, 11] = A[:, 11] * 2.0 ** -4              # |entries| < 1, then
    A[0, 11, 40], A[1, 11, 40] = -1.0, 0.0       # largest entry exactly -1
    B[:, :, 7] = B[:, :, 7] * 2.0 ** -7          # |entries| < 2^-3, then
    B[0, 64, 7], B[1, 64, 7] = 2.0 ** -3, 0.0    # largest entry exactly 2^-3
    A, B = A.cuda(), B.cuda()
    C = _ff().ff_gemm(A, B, algo=_algo(algo))
    torch.cuda.synchronize()
    Cn = C.cpu().numpy()
    assert np.all(Cn[:, 3, :] == 0) and np.all(Cn[:, :, 5] == 0)
    rows = [0, 3, 10, 11, M - 1]
    cols = [0, 5, 7, 33, N - 1]
    check_entries(A, B, C, rows, cols, f"zero/pow2 {algo}")


def _wide_range_operands(M, K, N, seed):
    """Rows of A and columns of B spanning 40 binades: half the rows (and
    columns) have every entry scaled by 2^s, s uniform in {-40..0}; the other
    half hold one normal(0,1) entry among entries scaled by 2^-40.  Scaling
    by powers of two keeps both words exact."""
    rng = np.random.default_rng(seed)
    A = fi.gaussian_ff((M, K), seed).double()
    B = fi.gaussian_ff((K, N), seed + 1).double()
    sa = rng.integers(-40, 1, (M, K)).astype(np.float64)
    sa[M // 2:] = -40.0
    sa[np.arange(M // 2, M), rng.integers(0, K, M - M // 2)] = 0.0
    sb = rng.integers(-40, 1, (K, N)).astype(np.float64)
    sb[:, N // 2:] = -40.0
    sb[rng.integers(0, K, N - N // 2), np.arange(N // 2, N)] = 0.0
    A = (A * torch.from_numpy(np.exp2(sa))).float()
    B = (B * torch.from_numpy(np.exp2(sb))).float()
    return A, B


@pytest.mark.parametrize("algo", ALGOS)
def test_wide_dynamic_range_within_the_documented_bound(algo):
    # Rows and columns whose entries span 40 binades, where the normwise
    # 2^-44 target is not promised: every entry must still meet the bound the
    # algorithm documents, |C - exact| <= 2^(e_i - 54) sum_k |B_kj|
    # + 2^(f_j - 54) sum_k (|A_ik| + 2^(e_i - 54))   (digit rounding)
    # + K 2^(e_i + f_j - 47)                          (dropped digit pairs)
    # + 2^-47 |C|                                     (final rounding),
    # with 2^e_i above row i's largest |A_ik| and 2^f_j above column j's
    # largest |B_kj| (taken one binade higher here, for either convention).
    M, K, N = 32, 2048, 32
    _announce(f"[gpu] gemm wide dynamic range {M}x{K}x{N} ({algo})")
    A, B = _wide_range_operands(M, K, N, 7301)
    C = _ff().ff_gemm(A.cuda(), B.cuda(), algo=_algo(algo)).cpu().numpy()
    An, Bn = A.numpy(), B.numpy()
    Av = An[0].astype(np.float64) + An[1].astype(np.float64)
    Bv = Bn[0].astype(np.float64) + Bn[1].astype(np.float64)
    e = np.frexp(np.abs(Av).max(axis=1))[1] + 1
    f = np.frexp(np.abs(Bv).max(axis=0))[1] + 1
    ri, ci = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
    ri, ci = ri.ravel(), ci.ravel()
    exact = oracle.exact_gemm_entries(An[0], An[1], Bn[0], Bn[1], ri, ci)
    scale = oracle.exact_absgemm_entries(An[0], An[1], Bn[0], Bn[1], ri, ci)
    sumB = np.abs(Bv).sum(axis=0)
    sumA = np.abs(Av).sum(axis=1)
    worst_ratio, worst_normwise = 0.0, -math.inf
    for t, (i, j) in enumerate(zip(ri, ci)):
        err = abs(frac(C[0, i, j]) + frac(C[1, i, j]) - exact[t])
        bound = (math.ldexp(sumB[j], int(e[i]) - 54)
                 + math.ldexp(sumA[i] + K * math.ldexp(1.0, int(e[i]) - 54), int(f[j]) - 54)
                 + K * math.ldexp(1.0, int(e[i] + f[j]) - 47)
                 + math.ldexp(abs(float(exact[t])), -47)) * 1.001
        assert float(err) <= bound, (algo, i, j, float(err), bound)
        worst_ratio = max(worst_ratio, float(err) / bound)
        if err and scale[t]:
            worst_normwise = max(worst_normwise, math.log2(err / scale[t]))
    _announce(f"  worst error / documented bound {worst_ratio:.3g}; "
              f"worst normwise log2 error {worst_normwise:.1f}")


@pytest.mark.parametrize("algo", ALGOS + ["fma"])
def test_strided_operands_and_output(algo):
    # leading dimensions larger than the rows (views into wider buffers),
    # one of them not a multiple of 4 and one operand starting 4 bytes past
    # 16-byte alignment: the slicing kernels take their element paths
    ff = _ff()
    M, N, K = 70, 45, 133
    baseA = fi.gaussian_ff((M, K + 5), 71).cuda()
    baseB = fi.gaussian_ff((K, N + 9), 72).cuda()
    A = baseA[:, :, :K]                       # lda = K + 5
    B = baseB[:, :, 1:N + 1]                  # ldb = N + 9, base + 4 bytes
    Cbuf = torch.full((2, M, N + 3), 7.0, device="cuda")
    C = Cbuf[:, :, :N]                        # ldc = N + 3
    ff.ff_gemm(A, B, algo=_algo(algo), out=C)
    torch.cuda.synchronize()
    assert torch.all(Cbuf[:, :, N:] == 7.0)   # padding columns untouched
    Ac, Bc = A.contiguous(), B.contiguous()
    if algo == "fma":
        Cn = C.cpu().numpy()
        Ch, Cl = oracle.gemm_ff_seq(Ac[0].cpu().numpy(), Ac[1].cpu().numpy(),
                                    Bc[0].cpu().numpy(), Bc[1].cpu().numpy())
        assert same_bits(Cn[0], Ch) and same_bits(Cn[1], Cl)
    else:
        check_entries(Ac, Bc, C.contiguous(), range(M), range(N), f"{algo} strided")
        Cref = ff.ff_gemm(Ac, Bc, algo=_algo(algo))
        assert torch.equal(Cref.view(torch.int32), C.contiguous().view(torch.int32))
