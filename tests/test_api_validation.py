"""CPU checks of the Python binding's argument validation: every malformed
operand is rejected with ValueError/TypeError before any pointer reaches the
C library (a wrong dtype, shape or layout would otherwise make the kernels
read or write outside the buffers).  No GPU work is started."""
import pytest
import torch

from paper_2209_11002_amd import api


def _f(*shape, dtype=torch.float32):
    return torch.zeros(shape, dtype=dtype)


def test_dense_operands_reject_bf16_x():
    with pytest.raises(TypeError, match="float32"):
        api.loss_fwd(_f(5, 40, dtype=torch.bfloat16), _f(3, 40), _f(40, 3))


@pytest.mark.parametrize("A,B,msg", [
    (_f(3, 41), _f(40, 3), "B must have shape"),     # N of A differs from X: B checked against A's p
    (_f(3, 40), _f(41, 3), "B must have shape"),
    (_f(3, 40), _f(40, 4), "B must have shape"),
    (_f(3, 40, dtype=torch.float64), _f(40, 3), "A must be float32"),
    (_f(3, 40), _f(3, 40).t(), "B must be contiguous"),
])
def test_dense_operands_shapes(A, B, msg):
    X = _f(5, 40)
    if A.shape[1] != 40:
        msg = "A must have shape"
    with pytest.raises((ValueError, TypeError), match=msg):
        api.loss_bwd(X, A, B, torch.ones(()))


def test_dense_operands_need_gpu():
    with pytest.raises(ValueError, match="GPU"):
        api.loss_fwd(_f(5, 40), _f(3, 40), _f(40, 3))


def test_mirror_steps_check_gradient_shape():
    with pytest.raises(ValueError, match="gA must have shape"):
        api.mirror_step_A(_f(3, 40), _f(3, 39), 0.1)
    with pytest.raises(TypeError, match="gB must be float32"):
        api.mirror_step_B(_f(40, 3), _f(40, 3, dtype=torch.float16), 0.1)
    with pytest.raises(ValueError, match="GPU"):
        api.mirror_step_A(_f(3, 40), _f(3, 40), 0.1)


def test_x_dtype_and_layout():
    with pytest.raises(TypeError, match="float32 or bfloat16"):
        api.fit(_f(5, 40, dtype=torch.float16), 3)
    with pytest.raises(ValueError, match="contiguous 2-D"):
        api.fit(_f(40, 5).t(), 3)
    with pytest.raises(ValueError, match="GPU"):
        api.fit(_f(5, 40), 3)


def test_ragged_images_share_dtype():
    imgs = [_f(5, 40), _f(6, 50, dtype=torch.bfloat16)]
    with pytest.raises(ValueError, match="share the dtype"):
        api.fit_ragged(imgs, [3, 3], [0, 1], [1.0, 1.0])
    with pytest.raises(ValueError, match="equal length"):
        api.fit_ragged(imgs[:1], [3, 3], [0], [1.0])


def test_check_f32_reports_each_defect():
    dev = torch.device("cpu")
    api._check_f32("o", _f(2, 3), (2, 3), dev)
    with pytest.raises(ValueError, match="shape"):
        api._check_f32("o", _f(3, 2), (2, 3), dev)
    with pytest.raises(TypeError, match="float32"):
        api._check_f32("o", _f(2, 3, dtype=torch.float64), (2, 3), dev)
    with pytest.raises(ValueError, match="contiguous"):
        api._check_f32("o", _f(3, 2).t(), (2, 3), dev)
    with pytest.raises(ValueError, match="on cuda"):
        api._check_f32("o", _f(2, 3), (2, 3), torch.device("cuda:0"))
