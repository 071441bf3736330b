"""The measurement aids on the device: vmat_read_stream reads every element
of its buffer once, and vmat_read_write_stream reads the same and writes
every chunk of its write buffer (a buffer of ones sums to its length; a
write buffer filled with NaN comes back without one), for write volumes
from none to more chunks than the grid has waves."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402


@pytest.mark.parametrize("n4,grid", [(1, 1), (4096, 3), (262144, 8), (262147, 64), (1 << 20, 256)])
def test_read_stream_reads_every_element_once(n4, grid):
    buf = torch.ones(4 * n4, dtype=torch.float32, device="cuda")
    part = torch.full((grid,), float("nan"), dtype=torch.float32, device="cuda")
    P.vmat.read_stream(buf, part, grid)
    torch.cuda.synchronize()
    assert part.double().sum().item() == 4 * n4


@pytest.mark.parametrize("n4,grid,chunks", [
    (4096, 3, 0),            # no writes
    (4096, 3, 5),            # fewer chunks than the 12 waves
    (262144, 8, 1000),       # more chunks than waves, more than read steps
    (262147, 64, 77),        # ragged read, chunks on some waves only
    (1 << 20, 256, 10240),   # 1.25 chunks per wave, 4 read steps
    (16, 256, 3000),         # read shorter than one grid stride
])
def test_read_write_stream_reads_all_and_writes_every_chunk(n4, grid, chunks):
    buf = torch.ones(4 * n4, dtype=torch.float32, device="cuda")
    wbuf = torch.full((chunks * 64,), float("nan"), dtype=torch.float64, device="cuda")
    part = torch.full((grid,), float("nan"), dtype=torch.float32, device="cuda")
    P.vmat.read_write_stream(buf, wbuf, part, grid)
    torch.cuda.synchronize()
    assert part.double().sum().item() == 4 * n4
    assert not torch.isnan(wbuf).any().item()
