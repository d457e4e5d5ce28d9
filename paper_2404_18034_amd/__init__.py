"""Batched prox-linear SCP with CTCS and customized PIPG for 6-DoF powered-descent Monte
Carlo on AMD MI355X (gfx950).

``paper_2404_18034_amd.api`` is the binding of the HIP library (``include/scp_batch.h``);
``paper_2404_18034_amd.instances`` draws the seeded synthetic problem instances.
"""
from . import api, instances  # noqa: F401

__all__ = ["instances", "api"]
