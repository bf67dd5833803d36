"""CPU stand-in for the GPU executor of the serving loop (tests only): flows from the oracle,
completion after a scripted delay on a fake clock."""
import oracle
from paper_1306_2461_amd.serve import BudgetExceeded


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt):
        self.t += dt


class FakeExecutor:
    def __init__(self, levels, radius, iters, budget_bytes=0, delay=0.01, clock=None, ring=0):
        self.levels, self.radius, self.iters = levels, radius, iters
        self.budget = budget_bytes
        self.delay = delay
        self.clock = clock or FakeClock()
        self.resident = 0
        self.prev = {}
        self.pushes = []
        self.next_handle = 1
        self.open_handles = {}
        self.ring = ring            # pushes in flight at most (0 = unbounded)
        self.inflight = []
        self.busy_count = 0

    def session_bytes(self, H, W):
        return 2 * H * W * 2 + 16 * H * W

    def open(self, H, W):
        need = self.session_bytes(H, W)
        if self.budget and self.resident + need > self.budget:
            raise BudgetExceeded(f"need {need}, left {self.budget - self.resident}")
        h = self.next_handle
        self.next_handle += 1
        self.resident += need
        self.open_handles[h] = need
        return h

    def close(self, h):
        self.resident -= self.open_handles.pop(h)
        self.prev.pop(h, None)

    def submit(self, items, keep=None):
        from paper_1306_2461_amd.serve import Busy
        self.inflight = [d for d in self.inflight if self.clock() < d]
        if self.ring and len(self.inflight) >= self.ring:
            self.busy_count += 1
            raise Busy("ring full")
        keep = [True] * len(items) if keep is None else keep
        out = []
        for h, f in items:
            if h in self.prev:
                u, v = oracle.flow(self.prev[h], f, self.levels, self.radius, self.iters)
                out.append((u, v, 1))
            else:
                out.append((None, None, 0))
            self.prev[h] = f
        self.pushes.append(len(items))
        self.inflight.append(self.clock() + self.delay)
        out = [o if k else (None, None, o[2]) for o, k in zip(out, keep)]
        return {"due": self.clock() + self.delay, "out": out}

    def ready(self, token):
        return self.clock() >= token["due"]

    def wait(self, token):
        if self.clock() < token["due"]:
            self.clock.advance(token["due"] - self.clock())

    def finish(self, token):
        return token["out"]
