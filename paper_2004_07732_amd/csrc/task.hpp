// Coroutine task used by the solver's host code (internal).
//
// A solve reads Krylov scalars back to the host at a few points (once per fine
// GCR iteration, once per coarsest restart cycle, ...).  Written as coroutines,
// those points are suspension points: a single solve resumes at once after a
// stream synchronisation, while the batched driver keeps many hierarchies in
// flight from one host thread and resumes each one when its stream has caught
// up (see StreamWait in mg.hpp).
#pragma once

#include <coroutine>
#include <exception>
#include <utility>

namespace dwf {

// Task<int>: a lazily started coroutine returning a status code.  Awaiting a
// task starts it and resumes the awaiting coroutine when it finishes
// (symmetric transfer, so deep call chains do not grow the host stack).
class Task {
public:
    struct promise_type {
        int value = 0;
        std::coroutine_handle<> cont{};
        Task get_return_object() { return Task{std::coroutine_handle<promise_type>::from_promise(*this)}; }
        std::suspend_always initial_suspend() noexcept { return {}; }
        struct Final {
            bool await_ready() noexcept { return false; }
            std::coroutine_handle<> await_suspend(std::coroutine_handle<promise_type> h) noexcept {
                auto c = h.promise().cont;
                return c ? c : std::noop_coroutine();
            }
            void await_resume() noexcept {}
        };
        Final final_suspend() noexcept { return {}; }
        void return_value(int v) { value = v; }
        void unhandled_exception() { std::terminate(); }
    };
    using handle = std::coroutine_handle<promise_type>;

    Task() = default;
    explicit Task(handle h) : h_(h) {}
    Task(Task&& o) noexcept : h_(std::exchange(o.h_, {})) {}
    Task& operator=(Task&& o) noexcept {
        if (this != &o) {
            if (h_) h_.destroy();
            h_ = std::exchange(o.h_, {});
        }
        return *this;
    }
    Task(const Task&) = delete;
    Task& operator=(const Task&) = delete;
    ~Task() {
        if (h_) h_.destroy();
    }

    bool await_ready() const noexcept { return false; }
    std::coroutine_handle<> await_suspend(std::coroutine_handle<> c) noexcept {
        h_.promise().cont = c;
        return h_;
    }
    int await_resume() const noexcept { return h_.promise().value; }

    // top-level control (the driver): start, test completion, read the status
    void start() { h_.resume(); }
    bool done() const { return !h_ || h_.done(); }
    int result() const { return h_.promise().value; }

private:
    handle h_{};
};

}  // namespace dwf
