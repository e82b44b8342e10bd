"""Oracle of the staged path's pipeline timing model -- TEST INFRASTRUCTURE ONLY.

A literal, slow simulation of the schedule of the paper's Algorithm 2 on one
GPU: batches n = 1..N, steps k = 1..N+2; at step k the scalable stream runs
Stage A of batch k and then Stage C of batch k-2, the non-scalable stream
runs Stage B of batch k-1 (indices outside 1..N are skipped, as the paper's
text on Algorithm 2 states).  Each step ends when both streams are idle.
With ``concurrent`` False the two streams are one (stages of a step run back
to back, the comm-overlap-only structure of Fig. 5b with no communication).
"""


def simulate(nsys, batch, t_a, t_b, t_c, concurrent=True):
    nb = -(-nsys // batch)
    clock = 0.0
    for k in range(1, nb + 3):
        stream1 = []                      # Stage A (batch k), then Stage C (batch k-2)
        stream2 = []                      # Stage B (batch k-1)
        if 1 <= k <= nb:
            stream1.append(t_a)
        if 1 <= k - 1 <= nb:
            stream2.append(t_b)
        if 1 <= k - 2 <= nb:
            stream1.append(t_c)
        if concurrent:
            step = max(sum(stream1), sum(stream2))
        else:
            step = sum(stream1) + sum(stream2)
        clock += step
    return clock
