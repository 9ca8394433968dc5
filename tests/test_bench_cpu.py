"""Host-side checks of the benchmark script, without a GPU: the multi-GPU
refusal, and its byte and matrix-core counts against figures worked out by
hand for the 256^2 x Ls 16 workload (4x4 aggregates, 16 null vectors, so 64^2
coarse sites with n = 32 coarse components, coarse Ls 2)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (imports only the standard library at module level)


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_coarse_launch_bytes_worked_example():
    # links by the per-site figure of the coarse stencil: 5 blocks of 32 x 32 BF16
    # complex (4 B) = 20 480 B per site; vectors: 2 slices x 32 FP64 complex (16 B),
    # read and written = 2 048 B per site
    assert bench.coarse_stencil_bytes(4096, 32, 2, 1, 4, 16) == 4096 * (20480 + 2048) == 92_274_688
    # the 3 blocks the kernel stores (site term, two forward hops): 12 288 B per site
    assert bench.coarse_stencil_bytes(4096, 32, 2, 1, 4, 16, link_blocks=3) == 4096 * (12288 + 2048) == 58_720_256
    # 16 right-hand sides: the links once, the vectors 16 times
    assert bench.coarse_stencil_bytes(4096, 32, 2, 16, 4, 16) == 4096 * (20480 + 16 * 2048)


def test_coarse_matrix_core_count_worked_example():
    # one tile of two columns: 2 waves per site (16 rows each), 10 inner steps of 16
    # complex entries over the five 32 x 32 blocks, a hi and a lo product each
    assert bench.coarse_mfma_per_launch(4096, 32, 2, 1) == 4096 * 2 * 10 * 2 == 163_840
    # four columns still fit one tile; 32 (slice, column) pairs take four tiles of 8
    assert bench.coarse_mfma_per_launch(4096, 32, 4, 1) == 163_840
    assert bench.coarse_mfma_per_launch(4096, 32, 2, 16) == 4 * 163_840
    # 9 pairs: two tiles of 8
    assert bench.coarse_mfma_per_launch(64, 16, 9, 1) == 64 * 1 * 2 * 2 * 5


def test_coarse_a_bytes_worked_example():
    # two launches on the 3 stored blocks: 2 x 12 288 B of links per site; vectors
    # FP64 in (16 B), FP32 intermediate out and in (8 B each), FP64 out (16 B) on
    # 2 slices x 32 components: 2 x 32 x 48 = 3 072 B per site
    assert bench.coarse_a_bytes(58_720_256, 4096, 32, 2, 1, 16) == 4096 * (24576 + 3072) == 113_246_208
    # FP32 vectors: the intermediate is FP32 already, two whole launches
    f32_launch = bench.coarse_stencil_bytes(4096, 32, 2, 1, 4, 8, link_blocks=3)
    assert bench.coarse_a_bytes(f32_launch, 4096, 32, 2, 1, 8) == 2 * f32_launch


def test_whole_solve_byte_model_worked_example():
    # one fine FP32 apply at 256^2 x 16: 2 x 16 x 65536 x 2 x 8 B of vectors plus
    # 2 x 65536 x 8 B of links = 34 603 008 B
    fine = 34_603_008
    coarse_vec = 4096 * 2 * 32 * 16
    # GCR(6), Gram form: per cycle sum_{j<5} (2j + 5) = 45 passes, the last step's
    # multi-dot (7) and its update of x and the residual (13 read, 2 written): 67
    # passes per 6 iterations; one coarse A per iteration
    got = bench.solve_model_bytes(10, 12, 6, 256, 16, 113_246_208, coarse_vec)
    want = 10 * fine + 12 * 113_246_208 + 12 * 67 / 6 * coarse_vec
    assert abs(got - want) <= 1e-6 * want
    # GCR(8), orthogonalising form: per cycle sum_{j<8} (2j + 7) = 112 vector passes less
    # the direction copy after the last one, plus 8 + 4 for the solution update and
    # restart: 123 passes per 8 iterations
    got = bench.solve_model_bytes(10, 16, 8, 256, 16, 113_246_208, coarse_vec)
    want = 10 * fine + 16 * 113_246_208 + 16 * 123 / 8 * coarse_vec
    assert abs(got - want) <= 1e-6 * want


def test_smoother_byte_model_worked_example():
    # 20 steps in cycles of 5: 6 passes for the initial residual; per cycle
    # Gram form (cycles of 5): sum_{j<4} (2j + 5) = 32 passes, the last step's multi-dot
    # (6) and its fused update of z and the residual (11 read, 2 written): 51 per cycle,
    # after an initial residual of 4: 4 + 4 * 51 = 208
    assert bench.smoother_model_passes(20, 5) == 208
    # orthogonalising form (cycles of 7, above the Gram limit): sum_{j<7} (2j + 7) = 91
    # less the last direction copy, and a solution update of 9; 14 = 7 + 7:
    # 6 + 2 * 99 + 2 = 206
    assert bench.smoother_model_passes(14, 7) == 206
    # the paper's 8 steps in one cycle: 6 + (64 + 48 - 1) + 10 = 127
    assert bench.smoother_model_passes(8, 0) == 127 == bench.smoother_model_passes(8, 8)
    assert bench.smoother_model_passes(0, 5) == 0
    fine_vec = 16 * 256 * 256 * 2 * 8
    base = bench.solve_model_bytes(10, 12, 6, 256, 16, 113_246_208, 4096 * 2 * 32 * 16)
    got = bench.solve_model_bytes(10, 12, 6, 256, 16, 113_246_208, 4096 * 2 * 32 * 16, kcycles=3, smooth_iters=20,
                                  smooth_restart=5)
    assert got - base == 3 * 208 * fine_vec

