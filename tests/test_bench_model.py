"""CPU checks of the byte and work model behind the benchmark's roofline
figures, against hand-computed values for the benchmark workloads (the
disordered 1024x1024 graphene: N = 2,097,152, 6,291,456 stored off-diagonal
elements, S = 8, M = 18 terms at z = pi; the twisted bilayer: N = 4,194,304,
80,955,560 elements, S = 16)."""
import bench

N, NNZ, S = 2_097_152, 6_291_456, 8
VEC64 = 16 * N * S                      # one FP64 state block: 268,435,456 B
MAT64 = NNZ * (4 + 8) + N * 8           # int32 columns, FP64 values, on-site: 92,274,688 B


def test_pass_bytes_fp64_and_fp32():
    assert bench.pass_bytes(N, NNZ, S, 16, 8) == 4 * VEC64 + MAT64 == 1_166_016_512
    assert bench.pass_bytes(N, NNZ, S, 8, 4) == 4 * (VEC64 // 2) + NNZ * 8 + N * 4 == 595_591_168


def test_pair_and_step_bytes():
    assert bench.pair_bytes(N, NNZ, S, 16, 8) == 5 * VEC64 + MAT64 == 1_434_451_968
    # 17 passes plus the FP64 phi0 stream of the correlation
    assert bench.step_bytes(18, N, NNZ, S, 16, 8) == 17 * 1_166_016_512 + VEC64
    # fused schedule at M = 18 (14 middle orders, an even number): FIRST alone
    # (psi in, one vector out), NOB2 with the first middle order (two in, two
    # out), 6 middle pairs, the last middle order with LAST (b_2, b_3, psi in,
    # psi' out), phi0
    fused = (2 * VEC64 + MAT64) + (4 * VEC64 + MAT64) + 6 * (5 * VEC64 + MAT64) + (4 * VEC64 + MAT64) + VEC64
    assert bench.schedule_bytes(18, True, N, NNZ, S, 16, 8) == fused == 11_836_325_888
    assert bench.schedule_bytes(18, False, N, NNZ, S, 16, 8) == bench.step_bytes(18, N, NNZ, S, 16, 8)
    # an odd number of middle orders: FIRST+NOB2 as one launch, 6 middle pairs, the last pair
    odd = (3 * VEC64 + MAT64) + 6 * (5 * VEC64 + MAT64) + (4 * VEC64 + MAT64) + VEC64
    assert bench.schedule_bytes(17, True, N, NNZ, S, 16, 8) == odd == 10_938_744_832
    # the shortest series: M = 4 (FIRST+NOB2, LAST alone), 5 (FIRST+NOB2, the
    # last pair), 6 (FIRST alone, NOB2 with the middle order, the last pair)
    assert bench.schedule_bytes(4, True, N, NNZ, S, 16, 8) == (3 * VEC64 + MAT64) + (4 * VEC64 + MAT64) + VEC64
    assert bench.schedule_bytes(5, True, N, NNZ, S, 16, 8) == (3 * VEC64 + MAT64) + (4 * VEC64 + MAT64) + VEC64
    assert bench.schedule_bytes(6, True, N, NNZ, S, 16, 8) == (
        (2 * VEC64 + MAT64) + (4 * VEC64 + MAT64) + (4 * VEC64 + MAT64) + VEC64)


def test_haydock_and_wide_row_bytes():
    assert bench.hay_iter_bytes(N, NNZ, S, 16, 8) == 6 * VEC64 + MAT64
    assert bench.pass_bytes(4_194_304, 80_955_560, 16, 8, 4) == 2_811_905_344


def test_nnz_update_count_of_the_headline_run():
    # (nnz + N) * S * (M - 1) * (N_t - 1) for 2048 samples
    assert bench.nnz_updates(N, NNZ, S, 18, 2048) == 8_388_608 * 8 * 17 * 2047 == 2_335_321_358_336

