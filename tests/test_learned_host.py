"""Host-side pieces of the learned-prox pipeline (no GPU): the crop layout
that turns recorded 512^2 prox inputs into 128^2 training pairs."""
import numpy as np
import torch

from paper_2411_00688_amd import learned


def test_crops_are_the_row_major_tiles_of_each_image():
    rng = np.random.default_rng(0)
    V = torch.tensor(rng.standard_normal((3, 10, 14)), dtype=torch.float32)
    C = learned.crops(V, 4)          # 2 x 3 tiles per image, the ragged edge dropped
    assert C.shape == (3 * 2 * 3, 4, 4) and C.is_contiguous()
    k = 0
    for m in range(3):
        for a in range(2):
            for b in range(3):
                assert torch.equal(C[k], V[m, 4 * a:4 * a + 4, 4 * b:4 * b + 4])
                k += 1


def test_crops_of_exact_size_images_are_the_images():
    V = torch.arange(2 * 8 * 8, dtype=torch.float32).reshape(2, 8, 8)
    assert torch.equal(learned.crops(V, 8), V)


def test_crops_reject_images_smaller_than_a_crop():
    V = torch.zeros(1, 5, 9)
    try:
        learned.crops(V, 6)
    except ValueError:
        return
    raise AssertionError("expected ValueError")
