"""GPU test of the worklist push micro-benchmark (Section III): both iteration spaces and both ways
of pushing deactivate exactly `count` nodes per iteration and time every iteration."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


@pytest.mark.parametrize("atomic", [False, True])
@pytest.mark.parametrize("nowl", [False, True])
@pytest.mark.parametrize("n,count", [(100_000, 1000), (12_345, 1000), (5000, 7)])
def test_push_microbench_sizes(n, count, nowl, atomic):
    import paper_1912_01478_amd as ip
    print("[gpu] push microbench n=%d count=%d nowl=%s atomic=%s" % (n, count, nowl, atomic), flush=True)
    tti, sizes = ip.push_microbench(n, count, nowl=nowl, atomic=atomic)
    k = (n + count - 1) // count
    assert len(sizes) == k and len(tti) == k
    assert (sizes == n - count * np.arange(k)).all()
    assert (tti > 0).all()


def test_push_microbench_rejects_bad_arguments():
    import paper_1912_01478_amd as ip
    with pytest.raises(ip.IpgcError):
        ip.push_microbench(0, 1000)
