"""The selector weights file names the features and network it was trained
for; the loader refuses any other (host logic, no GPU)."""
import os

import numpy as np
import pytest

from paper_2603_29975_amd import MLP_PARAMS, selector

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2603_29975_amd", "selector_weights.npz")


def test_committed_weights_match_the_library():
    theta, margin, target, meta = selector.load(WEIGHTS, with_meta=True)
    assert theta.dtype == np.float32 and theta.size == MLP_PARAMS
    assert "feature_spec" not in meta
    assert str(np.load(WEIGHTS)["feature_spec"]) == selector.FEATURE_SPEC


def test_other_or_missing_spec_is_refused(tmp_path):
    z = np.load(WEIGHTS, allow_pickle=False)
    fields = {k: z[k] for k in z.files}
    other = dict(fields, feature_spec=np.asarray(selector.FEATURE_SPEC.replace("(32)", "(33)")))
    np.savez(tmp_path / "other.npz", **other)
    with pytest.raises(ValueError, match="features"):
        selector.load(str(tmp_path / "other.npz"))
    missing = {k: v for k, v in fields.items() if k != "feature_spec"}
    np.savez(tmp_path / "missing.npz", **missing)
    with pytest.raises(ValueError, match="features"):
        selector.load(str(tmp_path / "missing.npz"))
    short = dict(fields, theta=fields["theta"][:-1])
    np.savez(tmp_path / "short.npz", **short)
    with pytest.raises(ValueError, match="parameters"):
        selector.load(str(tmp_path / "short.npz"))
