"""A step loop captured as one HIP graph.

Small workloads (the 8,000-particle cube) are bound by kernel launches: a
fluid step is about thirteen launches of a few microseconds each.  The
library's calls only enqueue work on the caller's stream, allocate nothing
and never synchronise, so a run of steps can be captured once (through
PyTorch's graph capture, on its capture stream) and replayed with one launch
per replay.  Every pointer a step uses is fixed for the life of the Sim
(the two particle arrays alternate, so a graph holds an even number of
steps and ends with the arrays in the roles it started with); the time step
is read on the device, so a dt that changes from step to step is followed.
"""
from __future__ import annotations

import torch


class StepGraph:
    """`steps` (even) steps of `sim` as one replayable graph."""

    def __init__(self, sim, steps: int = 2):
        if steps < 2 or steps % 2:
            raise ValueError("a step graph holds an even number of steps")
        self.sim, self.steps = sim, steps
        self.graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        done = sim.steps_done
        with torch.cuda.graph(self.graph):
            for _ in range(steps):
                sim.step()
        # capturing recorded the steps without running them: the arrays and
        # the diagnostics slot are back in their roles, the count is not
        sim.steps_done = done

    def replay(self, times: int = 1):
        """Run the captured steps `times` times on the current stream."""
        for _ in range(times):
            self.graph.replay()
            self.sim.steps_done += self.steps
