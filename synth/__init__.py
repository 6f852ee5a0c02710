"""Seeded synthetic ultrafast-Doppler IQ packets.

Stand-ins for the paper's phantom, kidney and liver recordings (Experimental
Studies section), which are not available: tissue speckle far above blood,
slow sinusoidal axial tissue motion, horizontal vessels of moving speckle and
white noise. This module holds none of the clutter filter's arithmetic; it only
makes inputs, and both the HIP path and the FP64 oracle consume them.

Layout of every packet: complex64, C-contiguous ``[nt][ny][nx]`` (frame-major,
each frame row-major with x fastest).
"""
from .packets import (PacketSpec, make_packet, spec_small, spec_clinical,
                      spec_precision, spec_learned, batch_specs, tube_mask)

__all__ = ["PacketSpec", "make_packet", "spec_small", "spec_clinical",
           "spec_precision", "spec_learned", "batch_specs", "tube_mask"]
