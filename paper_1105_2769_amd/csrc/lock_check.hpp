// A mutex and its scoped lock annotated for Clang's thread-safety analysis
// (-Wthread-safety, an error in this library's build): a member declared
// MB_GUARDED_BY(m) may only be read or written while m is held, and a
// function declared MB_REQUIRES(m) only be called with m held; the compiler
// checks every use.  Host code only.
#pragma once

#include <mutex>

#define MB_CAPABILITY(x) __attribute__((capability(x)))
#define MB_SCOPED_CAPABILITY __attribute__((scoped_lockable))
#define MB_GUARDED_BY(x) __attribute__((guarded_by(x)))
#define MB_ACQUIRE(...) __attribute__((acquire_capability(__VA_ARGS__)))
#define MB_RELEASE(...) __attribute__((release_capability(__VA_ARGS__)))
#define MB_REQUIRES(...) __attribute__((requires_capability(__VA_ARGS__)))

namespace mb {

class MB_CAPABILITY("mutex") Mutex {
public:
    void lock() MB_ACQUIRE() { m_.lock(); }
    void unlock() MB_RELEASE() { m_.unlock(); }
    std::mutex &native() { return m_; }

private:
    std::mutex m_;
};

// Holds the mutex for its scope.  native() is the underlying unique_lock for
// condition-variable waits, which release and retake the mutex inside the
// wait; the analysis treats the mutex as held throughout, which is what the
// code around the wait sees.
class MB_SCOPED_CAPABILITY Lock {
public:
    explicit Lock(Mutex &m) MB_ACQUIRE(m) : lk_(m.native()) {}
    ~Lock() MB_RELEASE() {}
    std::unique_lock<std::mutex> &native() { return lk_; }

private:
    std::unique_lock<std::mutex> lk_;
};

}  // namespace mb
