"""Host-side size checks of the Renderer wrappers (pure shape logic, run on the CPU): a backward
or batched call whose buffers do not match the forward's layout is refused with ValueError
before any pointer reaches the library, where the kernels would read or add out of bounds."""
import pytest
import torch

from paper_2602_22625_amd.render import check_backward_args, check_batch_args


def z(*shape):
    return torch.zeros(*shape)


def test_backward_needs_a_forward():
    with pytest.raises(RuntimeError):
        check_backward_args(None, dL_dimage=z(3, 4, 4))


def test_backward_sizes_match_the_forward():
    fwd = (10, 6 * 5)  # 10 primitives, a 6 x 5 canvas
    check_backward_args(fwd, dL_dimage=z(3, 6, 5), dL_dalpha=z(6, 5), out=z(10, 8), n_params=10)
    check_backward_args(fwd, target=z(3, 6, 5), out=z(10, 8))
    with pytest.raises(ValueError):
        check_backward_args(fwd, dL_dimage=z(3, 6, 4))            # image of another size
    with pytest.raises(ValueError):
        check_backward_args(fwd, target=z(3, 7, 5))
    with pytest.raises(ValueError):
        check_backward_args(fwd, dL_dimage=z(3, 6, 5), dL_dalpha=z(5, 5))
    with pytest.raises(ValueError):
        check_backward_args(fwd, dL_dimage=z(3, 6, 5), out=z(9, 8))  # fewer gradient rows
    with pytest.raises(ValueError):
        check_backward_args(fwd, dL_dimage=z(3, 6, 5), out=z(10, 7))
    with pytest.raises(ValueError):
        check_backward_args(fwd, dL_dimage=z(3, 6, 5), n_params=9)


def test_batch_sizes_cover_every_image():
    # (H, W, N, prim_offset, pixel_offset)
    descs = [(4, 4, 3, 0, 0), (2, 8, 5, 3, 16)]
    rows, npix = check_batch_args(descs, z(8, 8), z(8), image=z(3 * 32), alpha=z(32),
                                  target=z(3 * 32), out=z(8, 8))
    assert (rows, npix) == (8, 32)
    with pytest.raises(ValueError):
        check_batch_args(descs, z(7, 8), z(8))                    # a row past params
    with pytest.raises(ValueError):
        check_batch_args(descs, z(8, 8), z(7))
    with pytest.raises(ValueError):
        check_batch_args(descs, z(8, 8), z(8), image=z(3 * 31))
    with pytest.raises(ValueError):
        check_batch_args(descs, z(8, 8), z(8), alpha=z(31))
    with pytest.raises(ValueError):
        check_batch_args(descs, z(8, 8), z(8), target=z(3 * 30))
    with pytest.raises(ValueError):
        check_batch_args(descs, z(8, 8), z(8), out=z(7, 8))
    with pytest.raises(ValueError):
        check_batch_args([], z(8, 8), z(8))
