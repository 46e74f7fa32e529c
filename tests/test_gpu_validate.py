"""Host fault injection through emc_validate: non-unit quaternions, non-finite weights
or used pixel coordinates, and negative or non-finite model values are each refused
with EMC_ERR_INVALID_ARG and a message naming the check; valid contents (quaternion
norms within 1e-5 of 1, masked pixels with any coordinates) pass."""
import numpy as np
import pytest

from emc_inputs import tiny_problem

pytestmark = pytest.mark.gpu


def _geo(emc, t, quat=None, q=None, log_w=None):
    import torch

    return emc.Geometry(t["grid_n"], torch.as_tensor(t["q"] if q is None else q), torch.as_tensor(t["mask"]),
                        torch.as_tensor(t["quat"] if quat is None else quat),
                        torch.as_tensor(t["log_w"] if log_w is None else log_w), 10)


def test_validate_accepts_and_refuses(gpu_lib):
    import torch

    emc = gpu_lib
    t = tiny_problem(41, grid_n=12, n_pix=80, n_rot=50, n_data=10)
    model = torch.as_tensor(t["model"], dtype=torch.float32, device="cuda")
    emc.emc_validate(_geo(emc, t))
    emc.emc_validate(_geo(emc, t), model)
    # norms within the tolerance pass (FP32 storage of a unit quaternion is within 1e-7)
    quat = np.asarray(t["quat"]).copy()
    quat[3] *= 1.0 + 4e-6
    emc.emc_validate(_geo(emc, t, quat=quat), model)
    # a masked pixel's coordinates are never read
    q = np.asarray(t["q"]).copy()
    masked = int(np.flatnonzero(t["mask"] == 0)[0])
    q[masked] = np.nan
    emc.emc_validate(_geo(emc, t, q=q), model)

    def refused(fragment, **kw):
        m = kw.pop("model", model)
        with pytest.raises(emc.EmcError) as e:
            emc.emc_validate(_geo(emc, t, **kw), m)
        assert e.value.status == emc.EMC_ERR_INVALID_ARG
        assert fragment in str(e.value), str(e.value)

    quat = np.asarray(t["quat"]).copy()
    quat[7] *= 1.001
    refused("quaternion", quat=quat)
    quat = np.asarray(t["quat"]).copy()
    quat[0] = np.nan
    refused("quaternion", quat=quat)
    lw = np.asarray(t["log_w"]).copy()
    lw[5] = -np.inf
    refused("weight", log_w=lw)
    q = np.asarray(t["q"]).copy()
    q[int(np.flatnonzero(t["mask"])[3])] = [0.0, np.inf, 1.0]
    refused("pixel", q=q)
    bad = model.clone()
    bad[17] = float("nan")
    refused("model", model=bad)
    bad = model.clone()
    bad[-1] = -1e-3
    refused("model", model=bad)
