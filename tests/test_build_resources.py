"""The build's record of per-kernel resources (compiler remarks -> liblbrr_resources.json)."""
import json
import os

import pytest

from paper_1505_06900_amd import build as B

SAMPLE = """\
kernels.hpp:195:1: remark: Function Name: _ZN4lbrr6k_stepINS_5D3Q27ELi4EfEEvPKT1_PS2_NS_8StepArgsE [-Rpass-analysis=kernel-resource-usage]
kernels.hpp:195:1: remark:     TotalSGPRs: 33 [-Rpass-analysis=kernel-resource-usage]
kernels.hpp:195:1: remark:     VGPRs: 39 [-Rpass-analysis=kernel-resource-usage]
kernels.hpp:195:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
kernels.hpp:195:1: remark:     Dynamic Stack: False [-Rpass-analysis=kernel-resource-usage]
kernels.hpp:195:1: remark:     Occupancy [waves/SIMD]: 8 [-Rpass-analysis=kernel-resource-usage]
kernels.hpp:195:1: warning: something else
mk.hpp:9:1: remark: Function Name: _Z3foov [-Rpass-analysis=kernel-resource-usage]
mk.hpp:9:1: remark:     LDS Size [bytes/block]: 55296 [-Rpass-analysis=kernel-resource-usage]
"""


def test_remarks_are_parsed_per_kernel():
    r = B.parse_resource_remarks(SAMPLE)
    k = "_ZN4lbrr6k_stepINS_5D3Q27ELi4EfEEvPKT1_PS2_NS_8StepArgsE"
    assert set(r) == {k, "_Z3foov"}
    assert r[k] == {"TotalSGPRs": 33, "VGPRs": 39, "ScratchSize [bytes/lane]": 0, "Dynamic Stack": "False",
                    "Occupancy [waves/SIMD]": 8}
    assert r["_Z3foov"] == {"LDS Size [bytes/block]": 55296}


def test_built_library_records_the_step_kernels():
    if not os.path.exists(B.RESOURCES):
        pytest.skip("library not built")
    res = json.load(open(B.RESOURCES))
    step = [v for k, v in res.items() if "k_step<lbrr::D3Q27, 4, float>" in k]
    assert step and step[0]["ScratchSize [bytes/lane]"] == 0 and step[0]["VGPRs Spill"] == 0
