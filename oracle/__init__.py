"""FP64 CPU oracle of the localized EVD clutter filter (TEST INFRASTRUCTURE).

This package is the checker, not the product: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it. It shares no code with the HIP library and never imports it.

Parity notes: every function cites the passage of the paper it follows and is
pinned by the ``-m "not gpu"`` tests against closed forms, identities, library
routines (LAPACK ``eigh``/``svd``) or brute force. The MLP forward/backward is
pinned by central finite differences and a one-layer closed form.
"""
from .lcf_oracle import (Threshold, Window, window_boxes, window_table, casorati,
                         covariance, evd, rule_weights, knee_k,
                         knee_curvature, median_k, slope_k, power_weights, ncc_curve, ncc_k, mlp_gate, sigmoid_weights, projector, filter_packet, filter_stream,
                         CUT_FIXED_K, CUT_KNEE, CUT_EXPLICIT, CUT_MLP, CUT_MEDIAN, CUT_SLOPE, CUT_POWER, CUT_NCC, NCC_FN,
                         SHAPE_HARD, SHAPE_SIGMOID, PD_EQ13, PD_SUM,
                         PD_EQ13_COMPENSATED, FLAG_MLP_FALLBACK, GATE_SHARE)

__all__ = [n for n in dir() if not n.startswith("_")]
